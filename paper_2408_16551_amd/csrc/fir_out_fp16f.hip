// Polyphase FIR instantiations for the per-frame scaled fp16 operands: the
// frame's values times 2^-e_f as fp16 (RNE), and the fp16 hi + lo pieces
// (lo = RNE((x - hi) 2^11)).
#include "fir_kernels.h"

namespace tina {

hipError_t launch_fir_mode_fp16f(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_FP16F>(a, vec, s); }

hipError_t launch_fir_mode_fp16fx2(FirArgs& a, int vec, hipStream_t s) { return launch_mode<FIR_OUT_FP16FX2>(a, vec, s); }

}  // namespace tina
