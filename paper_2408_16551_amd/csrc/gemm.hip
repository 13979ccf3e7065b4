// DFT across branches as a dense matrix product on the MFMA units
// (Sec. 4.1, Eq. (12): Z = X F, cast as a pointwise convolution, Sec. 3.2):
//   C[f][n] = sum_k A[f][k] * Bt[n][k]
// A = polyphase FIR output (FP32, frames x K), Bt = the DFT operand from
// gen.hip (N x K, K-contiguous), C = channel outputs (FP32 accumulation),
// written straight to the complex64 output rows.
//
// Tiling: 128 x 128 output tile per 256-thread block (2 x 2 waves, 64 x 64
// per wave as 2 x 2 MFMA 32x32 blocks), K staged through LDS 128 bytes of
// each operand row at a time, with the next tile prefetched into registers
// while the current one is multiplied.  A is converted to the operand form
// while it is staged (bf16/fp16 hi+lo pieces, per-frame power-of-two scale,
// FP8); Bt arrives pre-converted from the plan.  Each lane reads the 16-byte
// K-slice of its row that the MFMA operand layout asks for; the same slice
// of the same K indices goes to A and B lanes, so the K order inside an
// instruction never has to be known.
#include "internal.h"

#include <stdlib.h>

namespace tina {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// EB: operand bytes per element in LDS; NP: pieces per operand; SLAB: bytes
// of a row consumed by one MFMA; SCALED: per-frame scale; MX: A arrives as
// block-scaled FP8 (codes + one scale byte per 32 K), B likewise.
template <int FORM> struct FT;
template <> struct FT<FORM_FP32> { static constexpr int EB = 4, NP = 1, SLAB = 32; static constexpr bool SCALED = false, MX = false; };
template <> struct FT<FORM_BF16> { static constexpr int EB = 2, NP = 1, SLAB = 32; static constexpr bool SCALED = false, MX = false; };
template <> struct FT<FORM_BF16X3> { static constexpr int EB = 2, NP = 2, SLAB = 32; static constexpr bool SCALED = false, MX = false; };
template <> struct FT<FORM_FP16> { static constexpr int EB = 2, NP = 1, SLAB = 32; static constexpr bool SCALED = true, MX = false; };
template <> struct FT<FORM_FP16X3> { static constexpr int EB = 2, NP = 2, SLAB = 32; static constexpr bool SCALED = true, MX = false; };
template <> struct FT<FORM_FP8> { static constexpr int EB = 1, NP = 1, SLAB = 64; static constexpr bool SCALED = true, MX = false; };
template <> struct FT<FORM_MXFP8> { static constexpr int EB = 1, NP = 1, SLAB = 64; static constexpr bool SCALED = false, MX = true; };

constexpr int BM = 128, BN = 128;     // block tile
constexpr int ROWB = 128;             // bytes of each operand row per K tile
constexpr int RS = ROWB + 16;         // LDS row stride: 16-byte pad keeps 16-byte reads conflict-free
constexpr int NT = 256;               // threads per block
constexpr int GROUP_M = 8;            // m-tiles swept per column of n-tiles

// Per-frame scale 2^e with the frame's largest |y| * 2^-e <= limit.
__device__ inline int frame_exponent(float amax, float limit) {
    if (!(amax > 0.0f) || !isfinite(amax)) return 0;
    int e;
    frexpf(amax / limit, &e);  // amax/limit in [2^(e-1), 2^e)
    while (e > -120 && ldexpf(limit, e - 1) >= amax) --e;
    while (e < 120 && ldexpf(limit, e) < amax) ++e;
    return e;
}

__device__ inline uint32_t bf16_pair(float a, float b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)b) << 16);
}
__device__ inline uint32_t f16_pair(float a, float b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
}
__device__ inline float bf16_round(float a) { return (float)(__bf16)a; }
__device__ inline float f16_round(float a) { return (float)(_Float16)a; }

// The MFMAs of one K slab for the wave's 2 x 2 blocks.  Products are issued
// term-major (every block's hi*hi, then every block's hi*lo, ...), so MFMAs
// that accumulate into the same registers are four instructions apart.
// af[bm][piece][read], bf[bn][piece][read]: the lane's 16-byte K slices.
// sa/sb (block-scaled form): the lane's E8M0 scale in the low byte, one per
// 32-K block of the lane's row / column.
template <int FORM, int NP, int RD>
__device__ __forceinline__ void mfma_slab(const uint4 (&af)[2][NP][RD], const uint4 (&bf)[2][NP][RD],
                                          f32x16 (&acc)[2][2], f32x16 (&acc2)[2][2], const int (&sa)[2],
                                          const int (&sb)[2]) {
    if constexpr (FORM == FORM_FP32) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    const f32x4 av = __builtin_bit_cast(f32x4, af[bm][0][0]);
                    const f32x4 bv = __builtin_bit_cast(f32x4, bf[bn][0][0]);
                    acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], bv[e], acc[bm][bn], 0, 0, 0);
                }
    } else if constexpr (FORM == FORM_BF16 || FORM == FORM_BF16X3) {
        // BF16X3: hi*hi, hi*lo and lo*hi all accumulate into acc (the small
        // terms are added in FP32, at FP32 accumulation accuracy).
        constexpr int NT = FORM == FORM_BF16X3 ? 3 : 1;
#pragma unroll
        for (int term = 0; term < NT; ++term)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    const int pa = term == 2 ? 1 : 0, pb = term == 1 ? 1 : 0;
                    const bf16x8 a = __builtin_bit_cast(bf16x8, af[bm][pa < NP ? pa : 0][0]);
                    const bf16x8 b = __builtin_bit_cast(bf16x8, bf[bn][pb < NP ? pb : 0][0]);
                    acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[bm][bn], 0, 0, 0);
                }
    } else if constexpr (FORM == FORM_FP16 || FORM == FORM_FP16X3) {
        // FP16X3: the two cross terms carry the lo pieces' 2^11 and go to acc2.
        constexpr int NT = FORM == FORM_FP16X3 ? 3 : 1;
#pragma unroll
        for (int term = 0; term < NT; ++term)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    const int pa = term == 2 ? 1 : 0, pb = term == 1 ? 1 : 0;
                    const f16x8 a = __builtin_bit_cast(f16x8, af[bm][pa < NP ? pa : 0][0]);
                    const f16x8 b = __builtin_bit_cast(f16x8, bf[bn][pb < NP ? pb : 0][0]);
                    if (term == 0) acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[bm][bn], 0, 0, 0);
                    else acc2[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc2[bm][bn], 0, 0, 0);
                }
    } else {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                i32x8 av, bv;
                const uint4 a0 = af[bm][0][0], a1 = af[bm][0][RD - 1];
                const uint4 b0 = bf[bn][0][0], b1 = bf[bn][0][RD - 1];
                av[0] = a0.x; av[1] = a0.y; av[2] = a0.z; av[3] = a0.w;
                av[4] = a1.x; av[5] = a1.y; av[6] = a1.z; av[7] = a1.w;
                bv[0] = b0.x; bv[1] = b0.y; bv[2] = b0.z; bv[3] = b0.w;
                bv[4] = b1.x; bv[5] = b1.y; bv[6] = b1.z; bv[7] = b1.w;
                // Formats 0/0 = FP8 E4M3 for both operands.  Per-frame form:
                // block scales 2^0 (E8M0 127); block-scaled form: the lane's own.
                if constexpr (FORM == FORM_MXFP8)
                    acc[bm][bn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[bm][bn], 0, 0, 0, sa[bm],
                                                                                  0, sb[bn]);
                else
                    acc[bm][bn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[bm][bn], 0, 0, 0,
                                                                                  0x7f7f7f7f, 0, 0x7f7f7f7f);
            }
    }
}

template <int FORM>
struct GemmSmem {
    static constexpr int NP = FT<FORM>::NP;
    uint8_t tiles[2 * NP * BM * RS];  // NP A pieces then NP B pieces, BM (= BN) rows of RS bytes
    float inv[BM], sc[BM];            // per-frame scale and its inverse
    uint32_t mxs[FT<FORM>::MX ? BM + BN : 1];  // block scales of the K tile: 4 bytes per A row, then B row
};

// Map a logical tile index L of an nm x nn grid: groups of GROUP_M m-tiles
// sweep all n-tiles, so they share each B column block and their A rows.
__device__ inline void grouped_tile(int64_t L, int64_t nm, int64_t nn, int64_t& m0, int64_t& n0) {
    const int64_t gsz_full = GROUP_M * nn;
    const int64_t grp = L / gsz_full, first_m = grp * GROUP_M;
    const int64_t gsz = min((int64_t)GROUP_M, nm - first_m);
    const int64_t within = L - grp * gsz_full;
    m0 = (first_m + within % gsz) * BM;
    n0 = (within / gsz) * BN;
}

// One BM x BN output tile at (m0, n0).  Called by every thread of the block.
template <int FORM>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t m0, int64_t n0, GemmSmem<FORM>& sm) {
    using ft = FT<FORM>;
    constexpr int NP = ft::NP, EB = ft::EB, SLAB = ft::SLAB;
    constexpr int BK = ROWB / EB;                 // K elements per tile
    constexpr int ACPR = BK / 4;                  // A float4 chunks per row
    constexpr int ACH = ft::MX ? 1 : BM * ACPR / NT;  // A float4 chunks per thread (FP32 A)
    constexpr int BCH = BN * (ROWB / 16) / NT;    // B 16-byte chunks per thread per piece
    constexpr int NSLAB = ROWB / SLAB;
    constexpr int RD = SLAB / 32;                 // 16-byte reads per lane per slab

    uint8_t* As = sm.tiles;                 // NP pieces of BM x RS
    uint8_t* Bs = sm.tiles + NP * BM * RS;  // NP pieces of BN x RS
    float* s_inv = sm.inv;
    float* s_sc = sm.sc;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lh = lane >> 5;

    __syncthreads();  // the previous tile of a persistent block is done with LDS

    if constexpr (ft::SCALED) {
        if (tid < BM) {
            const int64_t f = m0 + tid;
            float amax = 0.0f;
            if (f < g.F)
                for (int q = 0; q < g.nparts; ++q) amax = fmaxf(amax, g.amax[f * g.nparts + q]);
            const int e = frame_exponent(amax, FORM == FORM_FP8 ? 448.0f : 32768.0f);
            s_inv[tid] = ldexpf(1.0f, -e);
            s_sc[tid] = ldexpf(1.0f, e);
        }
        __syncthreads();
    }

    static_assert(!ft::MX || (BM + BN == NT && NP == 1), "block-scaled form: one scale word per thread");
    float4 ra[ACH];
    uint4 rb[NP][BCH];
    uint4 rqa[ft::MX ? BCH : 1];  // block-scaled form: A codes
    uint32_t rsc = 0;             // block-scaled form: this thread's scale word
    const uint8_t* Bp[2] = {(const uint8_t*)g.B0, (const uint8_t*)g.B1};
    const int64_t KB = (int64_t)g.K * EB;  // bytes per Bt row

    auto load_tile = [&](int k0) {
        if constexpr (ft::MX) {
            // K % 128 == 0 (checked at plan time): every K tile is whole.
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                const int64_t f = m0 + row;
                rqa[i] = f < g.F ? *reinterpret_cast<const uint4*>(g.Aq + f * g.lda + k0 + kc * 16)
                                 : make_uint4(0u, 0u, 0u, 0u);
            }
            const int64_t nb = g.K / 32;
            if (tid < BM) {
                const int64_t f = m0 + tid;
                rsc = f < g.F ? *reinterpret_cast<const uint32_t*>(g.Aqs + f * nb + k0 / 32) : 0x7f7f7f7fu;
            } else {
                const int64_t n = n0 + tid - BM;
                rsc = n < g.N ? *reinterpret_cast<const uint32_t*>((const uint8_t*)g.B1 + n * nb + k0 / 32)
                              : 0x7f7f7f7fu;
            }
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                const int64_t n = n0 + row;
                rb[0][i] = n < g.N ? *reinterpret_cast<const uint4*>(Bp[0] + n * KB + (int64_t)k0 + kc * 16)
                                   : make_uint4(0u, 0u, 0u, 0u);
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < ACH; ++i) {
            const int c = tid + i * NT, row = c / ACPR, kc = c % ACPR;
            const int64_t f = m0 + row;
            const int k = k0 + kc * 4;
            if (f < g.F && k < g.K) ra[i] = *reinterpret_cast<const float4*>(g.A + f * g.lda + k);
            else ra[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                const int64_t n = n0 + row;
                const int64_t kb = (int64_t)k0 * EB + kc * 16;
                if (n < g.N && kb < KB) rb[p][i] = *reinterpret_cast<const uint4*>(Bp[p] + n * KB + kb);
                else rb[p][i] = make_uint4(0u, 0u, 0u, 0u);
            }
    };

    auto store_tile = [&]() {
        if constexpr (ft::MX) {
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                *reinterpret_cast<uint4*>(As + row * RS + kc * 16) = rqa[i];
                *reinterpret_cast<uint4*>(Bs + row * RS + kc * 16) = rb[0][i];
            }
            sm.mxs[tid] = rsc;
            return;
        }
#pragma unroll
        for (int i = 0; i < ACH; ++i) {
            const int c = tid + i * NT, row = c / ACPR, kc = c % ACPR;
            const float4 x = ra[i];
            uint8_t* dst0 = As + row * RS + kc * 4 * EB;
            if constexpr (FORM == FORM_FP32) {
                *reinterpret_cast<float4*>(dst0) = x;
            } else if constexpr (FORM == FORM_BF16 || FORM == FORM_BF16X3) {
                *reinterpret_cast<uint2*>(dst0) = make_uint2(bf16_pair(x.x, x.y), bf16_pair(x.z, x.w));
                if constexpr (FORM == FORM_BF16X3) {
                    const float lx = x.x - bf16_round(x.x), ly = x.y - bf16_round(x.y);
                    const float lz = x.z - bf16_round(x.z), lw = x.w - bf16_round(x.w);
                    *reinterpret_cast<uint2*>(dst0 + BM * RS) = make_uint2(bf16_pair(lx, ly), bf16_pair(lz, lw));
                }
            } else if constexpr (FORM == FORM_FP16 || FORM == FORM_FP16X3) {
                const float s = s_inv[row];
                const float x0 = x.x * s, x1 = x.y * s, x2 = x.z * s, x3 = x.w * s;
                *reinterpret_cast<uint2*>(dst0) = make_uint2(f16_pair(x0, x1), f16_pair(x2, x3));
                if constexpr (FORM == FORM_FP16X3) {
                    const float l0 = (x0 - f16_round(x0)) * 2048.0f, l1 = (x1 - f16_round(x1)) * 2048.0f;
                    const float l2 = (x2 - f16_round(x2)) * 2048.0f, l3 = (x3 - f16_round(x3)) * 2048.0f;
                    *reinterpret_cast<uint2*>(dst0 + BM * RS) = make_uint2(f16_pair(l0, l1), f16_pair(l2, l3));
                }
            } else {
                const float s = s_inv[row];
                const float x0 = fminf(fmaxf(x.x * s, -448.f), 448.f), x1 = fminf(fmaxf(x.y * s, -448.f), 448.f);
                const float x2 = fminf(fmaxf(x.z * s, -448.f), 448.f), x3 = fminf(fmaxf(x.w * s, -448.f), 448.f);
                int w = __builtin_amdgcn_cvt_pk_fp8_f32(x0, x1, 0, false);
                w = __builtin_amdgcn_cvt_pk_fp8_f32(x2, x3, w, true);
                *reinterpret_cast<int*>(dst0) = w;
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                *reinterpret_cast<uint4*>(Bs + p * BN * RS + row * RS + kc * 16) = rb[p][i];
            }
    };

    f32x16 acc[2][2], acc2[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc[i][j][v] = 0.f; acc2[i][j][v] = 0.f; }

    const int nk = (g.K + BK - 1) / BK;
    load_tile(0);
    store_tile();
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        if (t + 1 < nk) load_tile((t + 1) * BK);
#pragma unroll
        for (int s = 0; s < NSLAB; ++s) {
            uint4 af[2][NP][RD], bf[2][NP][RD];
            // The lane's 16-byte reads of the slab.  For the 64-K FP8 MFMA
            // this puts the instruction's K index equal to the byte offset in
            // the slab (bytes 0-15 of lane half lh are K 16 lh.., bytes 16-31
            // are K 32 + 16 lh..), so its 32-K scale block b is bytes
            // [32 b, 32 b + 32) of the slab, whose scale lane half b supplies.
            auto off = [&](int q) { return s * SLAB + q * 32 + lh * 16; };
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int q = 0; q < RD; ++q) {
                        const int row = wm * 64 + bm * 32 + lr;
                        af[bm][p][q] = *reinterpret_cast<const uint4*>(As + p * BM * RS + row * RS + off(q));
                    }
#pragma unroll
            for (int bn = 0; bn < 2; ++bn)
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int q = 0; q < RD; ++q) {
                        const int row = wn * 64 + bn * 32 + lr;
                        bf[bn][p][q] = *reinterpret_cast<const uint4*>(Bs + p * BN * RS + row * RS + off(q));
                    }
            int sa[2] = {0, 0}, sb[2] = {0, 0};
            if constexpr (ft::MX) {
                const int sh = 8 * (2 * s + lh);  // byte of the word = 32-K block of the K tile
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    sa[b] = (int)(sm.mxs[wm * 64 + b * 32 + lr] >> sh);
                    sb[b] = (int)(sm.mxs[BM + wn * 64 + b * 32 + lr] >> sh);
                }
            }
            mfma_slab<FORM, NP, RD>(af, bf, acc, acc2, sa, sb);
        }
        __syncthreads();
        if (t + 1 < nk) {
            store_tile();
            __syncthreads();
        }
    }

    // Epilogue: combine pieces, undo the frame scale, write complex64 rows.
    const float corr = (FORM == FORM_FP16X3) ? (1.0f / 2048.0f) : 1.0f;
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            const int64_t col = n0 + wn * 64 + bn * 32 + lr;
            if (col >= g.N) continue;
            int64_t oc = col;
            if (g.real_pack) oc = col >= 2 ? col : (col == 0 ? 0 : (int64_t)g.N);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int rloc = wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * lh + (v & 3);
                const int64_t row = m0 + rloc;
                if (row >= g.F) continue;
                float val = acc[bm][bn][v];
                if constexpr (FORM == FORM_FP16X3) val += acc2[bm][bn][v] * corr;
                if constexpr (ft::SCALED) val *= s_sc[rloc];
                float* o = g.out + row * g.ldo;
                o[oc] = val;
                if (g.real_pack && col < 2) o[oc + 1] = 0.0f;  // Im X_0, Im X_{P/2}
            }
        }
}

template <int FORM>
__global__ __launch_bounds__(NT) void dft_gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) GemmSmem<FORM> sm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, m0, n0);
    gemm_tile<FORM>(g, m0, n0, sm);
}

// Batched GEMM, one block per tile of any item: block b serves tile
// i = b / 8 of XCD x = b % 8's contiguous, cost-balanced range of tiles (see
// BatchTable); blocks past the end of their range return at once.  (A
// persistent loop over tiles keeps per-tile state live across iterations and
// halves the occupancy, so each block does one tile.)
template <int FORM>
__global__ __launch_bounds__(NT) void dft_gemm_batch_kernel(const BatchTable* __restrict__ t) {
    __shared__ __attribute__((aligned(16))) GemmSmem<FORM> sm;
    const int x = blockIdx.x & 7;
    const int64_t u = t->gemm_bounds[x] + (blockIdx.x >> 3);
    if (u >= t->gemm_bounds[x + 1]) return;
    const int it = batch_find(t->items, t->n_items, u, /*stage=*/1);
    const GemmArgs& g = t->items[it].gemm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(u - t->items[it].gemm_unit0, nm, nn, m0, n0);
    gemm_tile<FORM>(g, m0, n0, sm);
}

template <int FORM>
hipError_t launch_form(const GemmArgs& g, hipStream_t s) {
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL(dft_gemm_kernel<FORM>, dim3((unsigned)(nm * nn)), dim3(NT), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_batch(const BatchTable* t, int form, int grid, hipStream_t s) {
    switch (form) {
        case FORM_FP32: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_FP32>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_BF16: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_BF16>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_BF16X3: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_BF16X3>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_FP16: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_FP16>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_FP16X3: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_FP16X3>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_FP8: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_FP8>, dim3(grid), dim3(NT), 0, s, t); break;
        case FORM_MXFP8: hipLaunchKernelGGL(dft_gemm_batch_kernel<FORM_MXFP8>, dim3(grid), dim3(NT), 0, s, t); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dft_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.F <= 0) return hipSuccess;
    switch (g.form) {
        case FORM_FP32: return launch_form<FORM_FP32>(g, s);
        case FORM_BF16: return launch_form<FORM_BF16>(g, s);
        case FORM_BF16X3: return launch_form<FORM_BF16X3>(g, s);
        case FORM_FP16: return launch_form<FORM_FP16>(g, s);
        case FORM_FP16X3: return launch_form<FORM_FP16X3>(g, s);
        case FORM_FP8: return launch_form<FORM_FP8>(g, s);
        case FORM_MXFP8: return (g.K % 128 == 0) ? launch_form<FORM_MXFP8>(g, s) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tina
