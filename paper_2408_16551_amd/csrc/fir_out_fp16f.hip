// Polyphase FIR instantiations for the per-frame scaled fp16 operands: the
// frame's values times 2^-e_f as fp16 (RNE), and the fp16 hi + lo pieces
// (lo = RNE((x - hi) 2^11)).
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_fp16f(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_FP16F>(a, vec, s); }

hipError_t launch_fir_mode_fp16fx2(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_FP16FX2>(a, vec, s); }

hipError_t launch_fir_batch_mode_fp16f(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_FP16F>(t, max_m, all_exact, grid, s);
}

hipError_t launch_fir_batch_mode_fp16fx2(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_FP16FX2>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
