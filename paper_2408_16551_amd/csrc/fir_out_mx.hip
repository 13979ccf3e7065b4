// Polyphase FIR instantiations for one output mode: block-scaled FP8 output (E4M3 codes, one E8M0 scale per 32 floats).
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_mx(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_MX>(a, vec, s); }

hipError_t launch_fir_batch_mode_mx(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_MX>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
