// Plan-time generation on the device, in FP64: the prototype window and the
// DFT operand in each precision form.
//
// Prototype (the paper only says the taps are divided between the P branches,
// Sec. 5.2): h[n] = sinc((n - (L-1)/2)/P) * w[n], L = P*M, symmetric window.
//
// DFT operand (Sec. 4.1, Eq. (12): Z = X F, F[p][k] = exp(-2 pi i p k/P)),
// stored transposed as Bt[n][k] so both GEMM operands are K-contiguous:
//   real input (K = P rows of y, N = P columns):
//     column 0 = Re X_0 (all ones), column 1 = Re X_{P/2} ((-1)^p),
//     columns 2k, 2k+1 (1 <= k < P/2) = cos(2 pi pk/P), -sin(2 pi pk/P);
//     Im X_0 and Im X_{P/2} are identically zero and get no column.
//   complex input (K = 2P: re, im of each branch; N = 2P: re, im of each channel):
//     2x2 block (p, k) = [[cos, -sin], [sin, cos]] (rows re/im of y_p,
//     columns re/im of X_k), angle 2 pi ((p k) mod P) / P.
#include "internal.h"

#include <math.h>

namespace tina {
namespace {

__global__ void window_kernel(double* h64, float* h32, int P, int M, int window) {
    const int64_t L = (int64_t)P * M;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L) return;
    const double t = ((double)n - 0.5 * (double)(L - 1)) / (double)P;  // exact
    const double sinc = (t == 0.0) ? 1.0 : sinpi(t) / (M_PI * t);
    double w = 1.0;
    if (L > 1) {
        const double u = 2.0 * (double)n / (double)(L - 1);  // cos(2 pi n/(L-1)) = cospi(u)
        switch (window) {
            case 1: w = 0.5 - 0.5 * cospi(u); break;
            case 2: w = 0.54 - 0.46 * cospi(u); break;
            case 3: w = 0.42 - 0.5 * cospi(u) + 0.08 * cospi(2.0 * u); break;
            default: w = 1.0; break;
        }
    }
    const double h = sinc * w;
    h64[n] = h;
    h32[n] = __double2float_rn(h);
}

__global__ void taps_to_f32_kernel(const double* h64, float* h32, int64_t L) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < L) h32[n] = __double2float_rn(h64[n]);
}

// Round v to `sig` significant bits, round-to-nearest-even, with the binade
// clamped below at 2^min_exp (gradual underflow of the target format).
__device__ inline double round_sig(double v, int sig, int min_exp) {
    if (v == 0.0) return 0.0;
    int e = ilogb(v);
    if (e < min_exp) e = min_exp;
    const int s = sig - 1 - e;
    return ldexp(rint(ldexp(v, s)), -s);
}

__device__ inline uint16_t bf16_bits_exact(double r) {  // r exactly representable in bf16
    return (uint16_t)(__float_as_uint((float)r) >> 16);
}
__device__ inline uint16_t f16_bits_exact(double r) {   // r exactly representable in fp16
    _Float16 h = (_Float16)(float)r;
    return __builtin_bit_cast(uint16_t, h);
}
// OCP FP8 E4M3 encoding of a value exactly on its grid, |r| <= 448.
__device__ inline uint8_t e4m3_bits_exact(double r) {
    if (r == 0.0) return 0;  // +0 for either signed zero
    const uint8_t sgn = r < 0.0 ? 0x80 : 0;
    const double a = fabs(r);
    int e = ilogb(a);
    if (e < -6) return sgn | (uint8_t)(int)ldexp(a, 9);         // subnormal: a = m * 2^-9
    int mant = (int)ldexp(a, 3 - e) - 8;                         // a = (1 + mant/8) * 2^e
    return sgn | (uint8_t)((e + 7) << 3) | (uint8_t)mant;
}

// Value of Bt[n][k] in FP64.  inverse: the inverse DFT of Sec. 4.2, Eq. (14)
// (angle +2 pi p k / P, scaled by 1/P; complex frames only).
__device__ inline double dft_entry(int64_t n, int64_t k, int P, int cplx, int inverse) {
    if (inverse) {
        const int64_t p = n >> 1, ch = k >> 1;  // output sample p, input channel ch
        const int64_t r = (p * ch) % P;
        double s, c;
        sincospi(2.0 * (double)r / (double)P, &s, &c);
        const int out_im = (int)(n & 1), in_im = (int)(k & 1);
        // (a + ib)(c + is) / P: re = (a c - b s) / P, im = (a s + b c) / P
        double v;
        if (out_im == in_im) v = c;
        else v = in_im ? -s : s;
        return v / (double)P;
    }
    if (!cplx) {
        if (n == 0) return 1.0;
        if (n == 1) return (k & 1) ? -1.0 : 1.0;
        const int64_t ch = n >> 1;
        const int64_t r = (k * ch) % P;
        double s, c;
        sincospi(2.0 * (double)r / (double)P, &s, &c);
        return (n & 1) ? -s : c;
    }
    const int64_t ch = n >> 1, p = k >> 1;
    const int64_t r = (p * ch) % P;
    double s, c;
    sincospi(2.0 * (double)r / (double)P, &s, &c);
    const int col_im = (int)(n & 1), row_im = (int)(k & 1);
    if (col_im == row_im) return c;
    return row_im ? s : -s;  // (row im, col re) = sin ; (row re, col im) = -sin
}

template <int FORM>
__global__ void dft_operand_kernel(void* piece0, void* piece1, int P, int cplx, int inverse) {
    const int64_t N = cplx ? 2 * (int64_t)P : P;
    const int64_t K = N;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * K) return;
    const int64_t n = idx / K, k = idx % K;
    const double v = dft_entry(n, k, P, cplx, inverse);
    if constexpr (FORM == FORM_FP32) {
        ((float*)piece0)[idx] = __double2float_rn(v);
    } else if constexpr (FORM == FORM_BF16 || FORM == FORM_BF16X3) {
        const double hi = round_sig(v, 8, -126);
        ((uint16_t*)piece0)[idx] = bf16_bits_exact(hi);
        if constexpr (FORM == FORM_BF16X3) ((uint16_t*)piece1)[idx] = bf16_bits_exact(round_sig(v - hi, 8, -126));
    } else if constexpr (FORM == FORM_FP16 || FORM == FORM_FP16X3) {
        const double hi = round_sig(v, 11, -14);
        ((uint16_t*)piece0)[idx] = f16_bits_exact(hi);
        if constexpr (FORM == FORM_FP16X3)
            ((uint16_t*)piece1)[idx] = f16_bits_exact(round_sig(ldexp(v - hi, 11), 11, -14));
    } else {
        ((uint8_t*)piece0)[idx] = e4m3_bits_exact(round_sig(v, 4, -6));
    }
}

// Block-scaled FP8 operand: thread t handles row n = t / (K/32), block b =
// t % (K/32) of Bt: the 32 FP64 entries, the smallest power-of-two scale 2^e
// (e in [-127, 127]) with max|v| <= 448 * 2^e, E4M3 codes of v * 2^-e
// (round to nearest even) and the E8M0 scale byte e + 127.
__global__ void mx_operand_kernel(uint8_t* codes, uint8_t* scales, int P, int cplx) {
    const int64_t N = cplx ? 2 * (int64_t)P : P;
    const int64_t K = N, nb = K / 32;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nb) return;
    const int64_t n = t / nb, k0 = (t % nb) * 32;
    double v[32], amax = 0.0;
    for (int i = 0; i < 32; ++i) {
        v[i] = dft_entry(n, k0 + i, P, cplx, 0);
        amax = fmax(amax, fabs(v[i]));
    }
    int e = 0;
    if (amax > 0.0) {
        e = -127;
        while (e < 127 && ldexp(448.0, e) < amax) ++e;
    }
    for (int i = 0; i < 32; ++i) codes[n * K + k0 + i] = e4m3_bits_exact(round_sig(ldexp(v[i], -e), 4, -6));
    scales[t] = (uint8_t)(e + 127);
}

// Block-reversed FP32 taps of the synthesis FIR: g'[(M-1-m) P + p] = h[m P + p].
__global__ void synthesis_taps_kernel(const double* h64, float* g32, int P, int M) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)P * M) return;
    const int64_t b = j / P, p = j % P;
    g32[j] = __double2float_rn(h64[(M - 1 - b) * P + p]);
}

}  // namespace

hipError_t launch_window(double* h64, float* h32, int P, int M, int window, hipStream_t s) {
    const int64_t L = (int64_t)P * M;
    hipLaunchKernelGGL(window_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, h64, h32, P, M,
                       window);
    return hipGetLastError();
}

hipError_t launch_taps_to_f32(const double* h64, float* h32, int64_t L, hipStream_t s) {
    hipLaunchKernelGGL(taps_to_f32_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, h64, h32, L);
    return hipGetLastError();
}

hipError_t launch_synthesis_taps(const double* h64, float* g32, int P, int M, hipStream_t s) {
    const int64_t L = (int64_t)P * M;
    hipLaunchKernelGGL(synthesis_taps_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, h64, g32, P, M);
    return hipGetLastError();
}

hipError_t launch_dft_operand(void* piece0, void* piece1, int P, int cplx, int form, hipStream_t s, int inverse) {
    const int64_t N = cplx ? 2 * (int64_t)P : P;
    const int64_t total = N * N;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (form == FORM_MXFP8) {
        if (inverse || N % 32 != 0) return hipErrorInvalidValue;
        const int64_t blocks = N * (N / 32);
        hipLaunchKernelGGL(mx_operand_kernel, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s, (uint8_t*)piece0,
                           (uint8_t*)piece1, P, cplx);
        return hipGetLastError();
    }
    switch (form) {
        case FORM_FP32: hipLaunchKernelGGL(dft_operand_kernel<FORM_FP32>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        case FORM_BF16: hipLaunchKernelGGL(dft_operand_kernel<FORM_BF16>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        case FORM_BF16X3: hipLaunchKernelGGL(dft_operand_kernel<FORM_BF16X3>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        case FORM_FP16: hipLaunchKernelGGL(dft_operand_kernel<FORM_FP16>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        case FORM_FP16X3: hipLaunchKernelGGL(dft_operand_kernel<FORM_FP16X3>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        case FORM_FP8: hipLaunchKernelGGL(dft_operand_kernel<FORM_FP8>, grid, block, 0, s, piece0, piece1, P, cplx, inverse); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tina
