// Polyphase FIR instantiations for the bf16 operand outputs: bf16 (RNE) and
// bf16 hi + lo pieces, written straight in the DFT GEMM's operand form.
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_bf16(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_BF16>(a, vec, s); }

hipError_t launch_fir_mode_bf16x2(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_BF16X2>(a, vec, s); }

hipError_t launch_fir_batch_mode_bf16(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_BF16>(t, max_m, all_exact, grid, s);
}

hipError_t launch_fir_batch_mode_bf16x2(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    return launch_batch_mode<FIR_OUT_BF16X2>(t, max_m, all_exact, grid, s);
}

}  // namespace tina
