// Polyphase FIR instantiations for one output mode: FP32 output rows plus per-frame partial maxima.
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_amax(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_AMAX>(a, vec, s); }

hipError_t launch_fir_batch_mode_amax(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_AMAX>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
