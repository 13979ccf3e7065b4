// Polyphase FIR instantiations for one output mode: FP32 output rows.
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_f32(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_F32>(a, vec, s); }

hipError_t launch_fir_batch_mode_f32(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_F32>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
