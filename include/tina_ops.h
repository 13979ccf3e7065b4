/*
 * tina_ops.h -- the two signal-processing building blocks of the filter bank
 * as standalone calls (C ABI): the unfolding (sliding-window) operation and a
 * plain FIR filter with arbitrary taps.
 *
 * TINA (arXiv 2408.16551) maps both onto a standard convolution: the unfold
 * with an identity kernel (Sec. 4.4, Eqs. (17)-(19)) and the FIR with the
 * taps as kernel (Sec. 4.3, Eqs. (15)-(16)).  Here they are direct kernels:
 * the unfold is a pure gather (its output is width/stride times larger than
 * the input, which is the memory cost the paper reports for it, Sec. 5.1),
 * and the FIR keeps a sliding window of the input in LDS and registers.
 *
 * Conventions as in tina_pfb.h: tina_status results, tina_last_error(),
 * validation before any work is enqueued, device pointers, asynchronous on
 * `stream` (a hipStream_t passed as void*; NULL = default stream).
 */
#ifndef TINA_OPS_H
#define TINA_OPS_H

#include <stdint.h>

#include "tina_pfb.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Unfold (Sec. 4.4, Eq. (17), with a stride): Y[i][j] = x[i*stride + j] for
 * i < rows = (n - width)/stride + 1 and j < width (rows = 0 when n < width).
 * x: n float32 values (device); y: rows x width float32 (device, row-major).
 * capacity_rows: rows y can hold (INVALID_ARGUMENT if fewer than needed).
 * *rows_out (may be NULL) receives rows.  width >= 1, stride >= 1.
 */
tina_status tina_unfold(const float* d_x, int64_t n, int64_t width, int64_t stride, float* d_y,
                        int64_t capacity_rows, int64_t* rows_out, void* stream);

typedef struct tina_fir_s* tina_fir_t;

/*
 * FIR filter (Sec. 4.3, Eq. (15)): y[i] = sum_{k=0}^{K-1} a[k] x[i-k], with
 * x[i] = 0 before the first sample.  The taps a[0..K) (host doubles, copied
 * and rounded to float32) are bound to a FIR object on `device`;
 * 1 <= K <= 8192.  sample_type: TINA_SAMPLE_R32 or TINA_SAMPLE_C64 (real
 * taps applied to re and im alike).
 */
tina_status tina_fir_create(int device, const double* taps, int32_t n_taps, int32_t sample_type, tina_fir_t* out);
tina_status tina_fir_destroy(tina_fir_t fir);

/* Filter n samples at d_x into n samples at d_y (device; d_y must not
 * overlap d_x). */
tina_status tina_fir_execute(tina_fir_t fir, const void* d_x, int64_t n, void* d_y, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TINA_OPS_H */
