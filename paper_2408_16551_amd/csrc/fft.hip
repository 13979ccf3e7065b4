// Factored DFT across the branches (the paper allows a "Discrete or Fast"
// Fourier transform after the FIR, Sec. 5.2): for P = P1 * P2, frame values
// y[p1*P2 + p2] (p1 < P1, p2 < P2),
//   1. A[k1][p2]  = sum_{p1} y[p1*P2 + p2] W_{P1}^{p1 k1}      (P2 DFTs of size P1)
//   2. A'[k1][p2] = A[k1][p2] W_P^{p2 k1}                         (twiddles)
//   3. X[k1 + P1 k2] = sum_{p2} A'[k1][p2] W_{P2}^{p2 k2}        (P1 DFTs of size P2)
// with W_n = exp(-2 pi i / n); the result equals the dense DFT of Eq. (12).
// Steps 1 and 3 are small complex matrix products, computed on the MFMA units
// in FP32 as real products of realified operands:
//   step 1: [Cr; Ci] = [[Fr, -Fi], [Fi, Fr]] . [Yr; Yi]   (F = DFT_{P1}^T)
//   step 3: [Xr, Xi] = [A'r, A'i] . [[Gr, Gi], [-Gi, Gr]]   (G = DFT_{P2})
// Flops per frame: 8 P (P1 + P2) instead of the dense 8 P^2.
//
// One block (256 threads) walks frames; the realified DFT matrices (one
// matrix when P1 = P2: the two coincide) sit in LDS for the whole launch and
// each frame passes through an LDS buffer three times (input, twiddled
// intermediate, output staging).  Row strides are padded so that the
// 16x16x4 MFMA fragment reads are free of bank conflicts.
#include <math.h>

#include "internal.h"

namespace tina {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Plan-time tables, in FP64 then rounded:
//   mat (2Q x 2Q, row-major, stride 2Q): [[cos, -sin], [sin, cos]] blocks with
//     angle 2 pi ((a b) mod Q) / Q -- realified DFT_Q as the B operand of
//     step 3 (rows = K) and, identically, the transposed A operand of step 1;
//   tw (P x 2): cos, sin of 2 pi r / P.
__global__ void fft_mat_kernel(float* mat, int Q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 2 * Q;
    if (idx >= n * n) return;
    const int a = idx / n, b = idx % n;
    const int ia = a % Q, ib = b % Q;
    double s, c;
    sincospi(2.0 * (double)((int64_t)ia * ib % Q) / (double)Q, &s, &c);
    const bool ra = a < Q, rb = b < Q;  // real half of K (rows) / of N (columns)
    double v;
    if (ra == rb) v = c;
    else v = ra ? -s : s;  // (re row, im col) = -sin ; (im row, re col) = +sin
    mat[idx] = __double2float_rn(v);
}

__global__ void fft_twiddle_kernel(float* tw, int P) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P) return;
    double s, c;
    sincospi(2.0 * (double)r / (double)P, &s, &c);
    tw[2 * r] = __double2float_rn(c);
    tw[2 * r + 1] = __double2float_rn(s);
}

// Stride of an LDS matrix whose 16x16x4 fragments read 4 rows x 16
// consecutive columns: stride = 16 (mod 32) keeps the two rows a half-wave
// reads on disjoint banks.
constexpr int stride16(int cols) { return (cols % 32 == 16) ? cols : cols + 16; }

template <int P1, int P2, bool CPLX>
struct FftShape {
    static constexpr int P = P1 * P2;
    static constexpr int K1 = CPLX ? 2 * P1 : P1;              // step-1 K (real input: no imaginary rows)
    static constexpr int S_M1 = stride16(2 * P1);              // step-1 matrix stride
    static constexpr int S_M3 = stride16(2 * P2);              // step-3 matrix stride
    static constexpr bool SHARED = (P1 == P2);                 // one matrix serves both steps
    static constexpr int MAT_FLOATS = 2 * P1 * S_M1 + (SHARED ? 0 : 2 * P2 * S_M3);
    static constexpr int S_Y = stride16(P2);                   // step-1 B buffer: K1 rows x P2
    static constexpr int S_A = 2 * P2 + 2;                      // step-3 A buffer: P1 rows x 2 P2 (stride = 2 mod 32)
    static constexpr int OUT_FLOATS = 2 * P + 2 * (P / 32) + 2; // padded output staging
    static constexpr int BUF_A = K1 * S_Y, BUF_B = P1 * S_A;
    static constexpr int BUF = BUF_A > BUF_B ? (BUF_A > OUT_FLOATS ? BUF_A : OUT_FLOATS)
                                             : (BUF_B > OUT_FLOATS ? BUF_B : OUT_FLOATS);
    static constexpr int LDS_BYTES = 4 * (MAT_FLOATS + BUF);
};

// Padded position of complex output k in the staging buffer.
__device__ __forceinline__ int out_pos(int k) { return 2 * k + 2 * (k >> 5); }

// Where frame f of a launch lives.  OneChunk: the frames of one call (rows
// of y and out).  ItemFrames: the frames of several batch items with the
// same P, one after the other (item i owns launch frames [f0_i, f0_i + F_i));
// each frame is found by a binary search over the items' first frames.  The
// arithmetic per frame is the same for both, so a batched item's output is
// bit for bit that of its own call.
struct OneChunk {
    const float* y;
    int64_t ldy;
    float* out;
    int64_t ldo, F;
    __device__ const float* yrow(int64_t f) const { return y + f * ldy; }
    __device__ float* orow(int64_t f) const { return out + f * ldo; }
};
struct ItemFrames {
    const FftItem* it;
    int n;
    int64_t F;
    __device__ int find(int64_t f) const {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (it[mid].f0 <= f) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
    __device__ const float* yrow(int64_t f) const {
        const FftItem& x = it[find(f)];
        return x.y + (f - x.f0) * x.ldy;
    }
    __device__ float* orow(int64_t f) const {
        const FftItem& x = it[find(f)];
        return x.out + (f - x.f0) * x.ldo;
    }
};

template <int P1, int P2, bool CPLX, class FA>
__global__ __launch_bounds__(256) void fft_dft_kernel(const FA fa, const float* __restrict__ mat1,
                                                      const float* __restrict__ mat3, const float* __restrict__ tw) {
    const int64_t F = fa.F;
    using S = FftShape<P1, P2, CPLX>;
    extern __shared__ float lds[];
    float* M1 = lds;                                   // [2 P1][S_M1] (K rows x M cols), step 1 (transposed A)
    float* M3 = S::SHARED ? lds : lds + 2 * P1 * S::S_M1;  // [2 P2][S_M3] (K rows x N cols), step 3 (B)
    float* buf = lds + S::MAT_FLOATS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lc = lane & 15, lk = lane >> 4;

    // DFT matrices into LDS once per block.
    for (int i = tid; i < 4 * P1 * P1; i += 256) M1[(i / (2 * P1)) * S::S_M1 + i % (2 * P1)] = mat1[i];
    if constexpr (!S::SHARED)
        for (int i = tid; i < 4 * P2 * P2; i += 256) M3[(i / (2 * P2)) * S::S_M3 + i % (2 * P2)] = mat3[i];

    constexpr int U1 = (P1 / 16) * (P2 / 16);  // step-1 units: (row block of k1, column block of p2)
    constexpr int U3 = (P1 / 16) * (P2 / 16);  // step-3 units: (row block of k1, column block of k2)
    constexpr int K3 = 2 * P2;

    for (int64_t f = blockIdx.x; f < F; f += gridDim.x) {
        __syncthreads();  // matrices written / previous frame's staging read
        // Frame into buf as [Yr; Yi]: row p1 (re) and K1/2 + p1 (im), column p2.
        const float* yf = fa.yrow(f);
        if constexpr (CPLX) {
            for (int i = tid; i < S::P; i += 256) {
                const float2 v = *reinterpret_cast<const float2*>(yf + 2 * i);
                const int p1 = i / P2, p2 = i % P2;
                buf[p1 * S::S_Y + p2] = v.x;
                buf[(P1 + p1) * S::S_Y + p2] = v.y;
            }
        } else {
            for (int i = tid; i < S::P; i += 256) buf[(i / P2) * S::S_Y + i % P2] = yf[i];
        }
        __syncthreads();

        // Step 1 (+ twiddles): each unit gives Re and Im of a 16 x 16 block of
        // A; a wave's units advance together through K so that their MFMAs
        // are independent of each other.
        constexpr int J1 = (U1 + 3) / 4;
        f32x4 cr1[J1], ci1[J1];
#pragma unroll
        for (int j = 0; j < J1; ++j) {
            cr1[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            ci1[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        for (int kb = 0; kb < S::K1 / 4; ++kb) {
            const int k = kb * 4 + lk;
#pragma unroll
            for (int j = 0; j < J1; ++j) {
                const int u = wave + 4 * j;
                if (u < U1) {
                    const int rb = u / (P2 / 16), cb = u % (P2 / 16);
                    const float a_re = M1[k * S::S_M1 + rb * 16 + lc];
                    const float a_im = M1[k * S::S_M1 + P1 + rb * 16 + lc];
                    const float b = buf[k * S::S_Y + cb * 16 + lc];
                    cr1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re, b, cr1[j], 0, 0, 0);
                    ci1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_im, b, ci1[j], 0, 0, 0);
                }
            }
        }
        float ar[J1][4], ai[J1][4];
#pragma unroll
        for (int j = 0; j < J1; ++j) {
            const int u = wave + 4 * j;
            if (u < U1) {
                const int rb = u / (P2 / 16), cb = u % (P2 / 16);
                const int p2 = cb * 16 + lc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k1 = rb * 16 + 4 * lk + r;
                    const int idx = (p2 * k1) & (S::P - 1);
                    const float wc = tw[2 * idx], ws = tw[2 * idx + 1];
                    ar[j][r] = cr1[j][r] * wc + ci1[j][r] * ws;   // (cr + i ci)(wc - i ws)
                    ai[j][r] = ci1[j][r] * wc - cr1[j][r] * ws;
                }
            }
        }
        __syncthreads();  // every wave is done reading the frame
#pragma unroll
        for (int j = 0; j < J1; ++j) {
            const int u = wave + 4 * j;
            if (u < U1) {
                const int rb = u / (P2 / 16), cb = u % (P2 / 16);
                const int p2 = cb * 16 + lc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k1 = rb * 16 + 4 * lk + r;
                    buf[k1 * S::S_A + p2] = ar[j][r];
                    buf[k1 * S::S_A + P2 + p2] = ai[j][r];
                }
            }
        }
        __syncthreads();

        // Step 3: X[k1 + P1 k2] from [A'r, A'i] . G, units again interleaved.
        constexpr int J3 = (U3 + 3) / 4;
        f32x4 xr[J3], xi[J3];
#pragma unroll
        for (int j = 0; j < J3; ++j) {
            xr[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            xi[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        for (int kb = 0; kb < K3 / 4; ++kb) {
            const int k = kb * 4 + lk;
#pragma unroll
            for (int j = 0; j < J3; ++j) {
                const int u = wave + 4 * j;
                if (u < U3) {
                    const int rb = u / (P2 / 16), cb = u % (P2 / 16);
                    const float a = buf[(rb * 16 + lc) * S::S_A + k];
                    const float b_re = M3[k * S::S_M3 + cb * 16 + lc];
                    const float b_im = M3[k * S::S_M3 + P2 + cb * 16 + lc];
                    xr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b_re, xr[j], 0, 0, 0);
                    xi[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b_im, xi[j], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // done reading A'
#pragma unroll
        for (int j = 0; j < J3; ++j) {
            const int u = wave + 4 * j;
            if (u < U3) {
                const int rb = u / (P2 / 16), cb = u % (P2 / 16);
                const int k2 = cb * 16 + lc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k1 = rb * 16 + 4 * lk + r;
                    const int k = k1 + P1 * k2;
                    buf[out_pos(k)] = xr[j][r];
                    buf[out_pos(k) + 1] = xi[j][r];
                }
            }
        }
        __syncthreads();
        float* of = fa.orow(f);
        constexpr int KOUT = CPLX ? S::P : S::P / 2 + 1;
        for (int k = tid; k < KOUT; k += 256) {
            float2 v = make_float2(buf[out_pos(k)], buf[out_pos(k) + 1]);
            if (!CPLX && (k == 0 || k == S::P / 2)) v.y = 0.0f;  // real input: these are real
            *reinterpret_cast<float2*>(of + 2 * k) = v;
        }
    }
}

// Complex frames with P = Q * Q, Q = 64 (P = 4096): the same three steps with
// both DFT matrices held in registers and every product on
// v_mfma_f32_32x32x2_f32.  Four waves share a frame.  Step 1: wave w computes
// rows k1 = 16 w .. 16 w + 15 (real and imaginary parts: 32 realified rows) of
// C = DFT_Q Y over all Q columns p2; its slice of the realified DFT matrix (Q
// floats per lane) is loaded once per launch.  The summed index is ordered
// (p1, re/im), so each MFMA's B operand is 64 consecutive floats of the frame
// as it lies in memory (and in LDS: no transposition, no bank conflicts).
// The real and imaginary parts of an output land in one lane, which applies
// the twiddle W_P^{p2 k1} (its Q / 2 twiddles are also kept in registers).
// Step 3: wave w computes columns k2 = 16 w .. 16 w + 15 (real and imaginary:
// 32 realified columns) of X = A' DFT_Q over all Q rows k1, its slice of the
// realified matrix again in registers, A' read from LDS (row stride 2 Q + 2
// floats: conflict-free).  The next frame's input is loaded into registers
// during step 1 and stored to LDS before step 3.
constexpr int kFq = 64;                     // Q
constexpr int kFqS = 2 * kFq + 2;           // A' row stride (floats)
constexpr int kFqLds = 4 * (2 * kFq * kFq + kFq * kFqS);

template <class FA>
__global__ __launch_bounds__(256) void fft_q64_kernel(const FA fa, const float* __restrict__ tw) {
    const int64_t F = fa.F;
    constexpr int Q = kFq, P = Q * Q;
    typedef float f32x16 __attribute__((ext_vector_type(16)));
    extern __shared__ float lds[];
    float* Yb = lds;              // the frame: complex samples p1 Q + p2, re then im
    float* As = lds + 2 * P;      // A'[k1][p2] as (re, im), row stride kFqS
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = lane & 31, h = lane >> 5;

    // Step-1 operand A[row][k]: row = (part r / 16, k1 = 16 w + r % 16), k =
    // (p1 = j, h): Re rows take (cos, sin), Im rows (-sin, cos) of 2 pi k1 p1 / Q.
    // Step-3 operand B[k][col]: k = (p2 = j, h), col = (part r / 16, k2 = 16 w
    // + r % 16): Re columns take (cos, sin), Im columns (-sin, cos).  With
    // P = Q^2 the angle 2 pi m / Q is table entry m Q of the P-point table.
    float a1[Q], b3[Q];
    {
        const int x = 16 * w + (r & 15);  // k1 of the step-1 row, k2 of the step-3 column
        const bool im = r >= 16;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const int m = (x * j) & (Q - 1);
            const float c = tw[2 * m * Q], sn = tw[2 * m * Q + 1];
            const float v = im ? (h ? c : -sn) : (h ? sn : c);
            a1[j] = v;
            b3[j] = v;
        }
    }
    // Twiddles of the lane's step-1 outputs: column block nb, element v < 8
    // holds (re, im) at (v, v + 8) for k1 = 16 w + 8 (v / 4) + 4 h + v % 4,
    // p2 = 32 nb + r.
    float twc[2][8], tws[2][8];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int k1 = 16 * w + 8 * (v >> 2) + 4 * h + (v & 3), p2 = 32 * nb + r;
            const int idx = (p2 * k1) & (P - 1);
            twc[nb][v] = tw[2 * idx];
            tws[nb][v] = tw[2 * idx + 1];
        }

    // Frame loads: 2 P floats = 512 float4, two per thread.
    float4 pre[8];
    auto load_frame = [&](int64_t f) {
        const float4* src = reinterpret_cast<const float4*>(fa.yrow(f));
#pragma unroll
        for (int i = 0; i < 8; ++i) pre[i] = src[tid + 256 * i];
    };
    auto store_frame = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i) reinterpret_cast<float4*>(Yb)[tid + 256 * i] = pre[i];
    };

    int64_t f = blockIdx.x;
    if (f < F) {
        load_frame(f);
        store_frame();
    }
    __syncthreads();
    for (; f < F; f += gridDim.x) {
        const int64_t fn = f + gridDim.x;
        if (fn < F) load_frame(fn);

        // Step 1: two 32 x 32 column blocks, Q MFMAs each over k = (p1, re/im).
        f32x16 c1[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) c1[nb][v] = 0.0f;
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const float bv = Yb[(j * Q + 32 * nb + r) * 2 + h];
                c1[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[j], bv, c1[nb], 0, 0, 0);
            }
        // Twiddle and write A'[k1][p2].
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const float cr = c1[nb][v], ci = c1[nb][v + 8];
                const float wc = twc[nb][v], ws = tws[nb][v];
                const int k1 = 16 * w + 8 * (v >> 2) + 4 * h + (v & 3), p2 = 32 * nb + r;
                *reinterpret_cast<float2*>(As + k1 * kFqS + 2 * p2) =
                    make_float2(cr * wc + ci * ws, ci * wc - cr * ws);  // (cr + i ci)(wc - i ws)
            }
        __syncthreads();  // A' complete; every wave is done with the frame in Yb
        if (fn < F) store_frame();

        // Step 3: two 32 x 32 row blocks (k1), Q MFMAs each over k = (p2, re/im).
        f32x16 x3[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) x3[rb][v] = 0.0f;
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const float av = As[(32 * rb + r) * kFqS + 2 * j + h];
                x3[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b3[j], x3[rb], 0, 0, 0);
            }
        // X[k1 + Q k2]: element v of row block rb is k1 = 32 rb + 8 (v / 4) +
        // 4 h + v % 4, the lane's column (part r / 16, k2 = 16 w + r % 16).
        float* of = fa.orow(f) + 2 * (Q * (16 * w + (r & 15))) + (r >> 4);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) of[2 * (32 * rb + 8 * (v >> 2) + 4 * h + (v & 3))] = x3[rb][v];
        __syncthreads();  // the next frame is in Yb; every wave is done with A'
    }
}

template <int P1, int P2, bool CPLX, class FA>
hipError_t launch_fft_t(const FA& fa, const float* mat1, const float* mat3, const float* tw, int cus, hipStream_t s) {
    using S = FftShape<P1, P2, CPLX>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fft_dft_kernel<P1, P2, CPLX, FA>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS_BYTES);
        if (e != hipSuccess) return e;
        attr = true;
    }
    int blocks_per_cu = (160 * 1024) / (S::LDS_BYTES + 1024);
    if (blocks_per_cu < 1) blocks_per_cu = 1;
    if (blocks_per_cu > 4) blocks_per_cu = 4;
    int64_t grid = (int64_t)cus * blocks_per_cu;
    if (grid > fa.F) grid = fa.F;
    hipLaunchKernelGGL((fft_dft_kernel<P1, P2, CPLX, FA>), dim3((unsigned)grid), dim3(256), S::LDS_BYTES, s, fa, mat1,
                       mat3, tw);
    return hipGetLastError();
}

// Complex P = 4096 with 16-byte aligned rows: the register-resident kernel.
template <class FA>
hipError_t launch_q64(const FA& fa, const float* tw, int cus, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fft_q64_kernel<FA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kFqLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    int64_t grid = 2 * (int64_t)cus;  // two blocks per CU (65.5 KiB of LDS each)
    if (grid > fa.F) grid = fa.F;
    hipLaunchKernelGGL((fft_q64_kernel<FA>), dim3((unsigned)grid), dim3(256), kFqLds, s, fa, tw);
    return hipGetLastError();
}

template <class FA>
hipError_t launch_fft_any(const FA& fa, int P, bool cplx, bool q64_ok, const float* mat1, const float* mat3,
                          const float* tw, int cus, hipStream_t s) {
    if (fa.F <= 0) return hipSuccess;
    if (cplx && P == kFq * kFq && q64_ok) return launch_q64(fa, tw, cus, s);
    switch (P) {
        case 256: return cplx ? launch_fft_t<16, 16, true>(fa, mat1, mat3, tw, cus, s)
                              : launch_fft_t<16, 16, false>(fa, mat1, mat3, tw, cus, s);
        case 512: return cplx ? launch_fft_t<32, 16, true>(fa, mat1, mat3, tw, cus, s)
                              : launch_fft_t<32, 16, false>(fa, mat1, mat3, tw, cus, s);
        case 1024: return cplx ? launch_fft_t<32, 32, true>(fa, mat1, mat3, tw, cus, s)
                               : launch_fft_t<32, 32, false>(fa, mat1, mat3, tw, cus, s);
        case 2048: return cplx ? launch_fft_t<64, 32, true>(fa, mat1, mat3, tw, cus, s)
                               : launch_fft_t<64, 32, false>(fa, mat1, mat3, tw, cus, s);
        case 4096: return cplx ? launch_fft_t<64, 64, true>(fa, mat1, mat3, tw, cus, s)
                               : launch_fft_t<64, 64, false>(fa, mat1, mat3, tw, cus, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool fft_supported(int P) { return P >= 256 && P <= 4096 && (P & (P - 1)) == 0; }

void fft_factors(int P, int& P1, int& P2) {
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    P1 = 1 << ((lg + 1) / 2);
    P2 = P / P1;
}

int fft_lds_bytes(int P, bool cplx) {
    switch (P) {
        case 256: return cplx ? FftShape<16, 16, true>::LDS_BYTES : FftShape<16, 16, false>::LDS_BYTES;
        case 512: return cplx ? FftShape<32, 16, true>::LDS_BYTES : FftShape<32, 16, false>::LDS_BYTES;
        case 1024: return cplx ? FftShape<32, 32, true>::LDS_BYTES : FftShape<32, 32, false>::LDS_BYTES;
        case 2048: return cplx ? FftShape<64, 32, true>::LDS_BYTES : FftShape<64, 32, false>::LDS_BYTES;
        case 4096: return cplx ? FftShape<64, 64, true>::LDS_BYTES : FftShape<64, 64, false>::LDS_BYTES;
        default: return 0;
    }
}

hipError_t launch_fft_tables(float* mat1, float* mat3, float* tw, int P, hipStream_t s) {
    int P1, P2;
    fft_factors(P, P1, P2);
    hipLaunchKernelGGL(fft_mat_kernel, dim3((4 * P1 * P1 + 255) / 256), dim3(256), 0, s, mat1, P1);
    if (P1 != P2) hipLaunchKernelGGL(fft_mat_kernel, dim3((4 * P2 * P2 + 255) / 256), dim3(256), 0, s, mat3, P2);
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3((P + 255) / 256), dim3(256), 0, s, tw, P);
    return hipGetLastError();
}

hipError_t launch_twiddle_table(float* tw, int P, hipStream_t s) {
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3((P + 255) / 256), dim3(256), 0, s, tw, P);
    return hipGetLastError();
}

hipError_t launch_fft_dft(const FftArgs& a, hipStream_t s) {
    const OneChunk fa{a.y, a.ldy, a.out, a.ldo, a.F};
    const bool q64_ok = a.ldy % 4 == 0 && ((uintptr_t)a.y & 15) == 0;
    return launch_fft_any(fa, a.P, a.cplx != 0, q64_ok, a.mat1, a.mat3, a.tw, a.cus, s);
}

hipError_t launch_fft_batch(const FftItem* items, int n, int64_t F, int P, bool cplx, bool q64_ok, const float* mat1,
                            const float* mat3, const float* tw, int cus, hipStream_t s) {
    const ItemFrames fa{items, n, F};
    return launch_fft_any(fa, P, cplx, q64_ok, mat1, mat3, tw, cus, s);
}

}  // namespace tina
