// Polyphase FIR instantiations for the per-frame scaled forms: a pass that
// only finds each frame's partial maxima, and the FP8 E4M3 codes written with
// the frame's scale once its exponent is known.
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_amaxonly(FirArgs& a, int vec, hipStream_t s) {
    return launch_mode<FIR_OUT_AMAXONLY>(a, vec, s);
}

hipError_t launch_fir_mode_fp8f(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_FP8F>(a, vec, s); }

hipError_t launch_fir_batch_mode_amaxonly(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_AMAXONLY>(t, max_m, all_exact, grid, s);
}

hipError_t launch_fir_batch_mode_fp8f(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_FP8F>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
