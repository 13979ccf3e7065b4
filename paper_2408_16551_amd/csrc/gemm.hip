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

#include <type_traits>

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

constexpr int BM = 128;               // block tile rows (frames); columns BN = 64 * WN
constexpr int ROWB = 128;             // bytes of each operand row per K tile
constexpr int RS = ROWB + 16;         // LDS row stride: 16-byte pad keeps 16-byte reads conflict-free
constexpr int NT = 256;               // threads per block
constexpr int GROUP_M = 16;           // m-tiles swept per column of n-tiles

__device__ inline uint32_t bf16_pair(float a, float b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)b) << 16);
}
__device__ inline uint32_t f16_pair(float a, float b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
}
__device__ inline float bf16_round(float a) { return (float)(__bf16)a; }
__device__ inline float f16_round(float a) { return (float)(_Float16)a; }

// The MFMAs of one K slab for the wave's 2 x WN blocks.  Products are issued
// term-major (every block's hi*hi, then every block's hi*lo, ...), so MFMAs
// that accumulate into the same registers are four instructions apart.
// af[bm][piece][read], bf[bn][piece][read]: the lane's 16-byte K slices.
// sa/sb (block-scaled form): the lane's E8M0 scale in the low byte, one per
// 32-K block of the lane's row / column.
template <int FORM, int NP, int RD, int TM, int WN>
__device__ __forceinline__ void mfma_block(const uint4 (&af)[TM][NP][RD], const uint4 (&bf)[WN][NP][RD],
                                           f32x16 (&acc)[TM][WN], f32x16 (&acc2)[TM][WN], const int (&sa)[TM],
                                           const int (&sb)[WN]) {
    if constexpr (FORM == FORM_FP32) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int bm = 0; bm < TM; ++bm)
#pragma unroll
                for (int bn = 0; bn < WN; ++bn) {
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
            for (int bm = 0; bm < TM; ++bm)
#pragma unroll
                for (int bn = 0; bn < WN; ++bn) {
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
            for (int bm = 0; bm < TM; ++bm)
#pragma unroll
                for (int bn = 0; bn < WN; ++bn) {
                    const int pa = term == 2 ? 1 : 0, pb = term == 1 ? 1 : 0;
                    const f16x8 a = __builtin_bit_cast(f16x8, af[bm][pa < NP ? pa : 0][0]);
                    const f16x8 b = __builtin_bit_cast(f16x8, bf[bn][pb < NP ? pb : 0][0]);
                    if (term == 0) acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[bm][bn], 0, 0, 0);
                    else acc2[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc2[bm][bn], 0, 0, 0);
                }
    } else {
#pragma unroll
        for (int bm = 0; bm < TM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
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

// FP8 E4M3 product with E8M0 scales taken from byte oa of sa and byte ob of
// sb (the instruction's scale operand selectors are immediates: after
// unrolling oa and ob are constants and the switch folds away).
__device__ __forceinline__ f32x16 mfma_f8_scaled_sel(const i32x8& a, const i32x8& b, const f32x16& c, int sa, int sb,
                                                     int oa, int ob) {
#define TINA_MX_CASE(A, B) \
    case A * 4 + B: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, A, sa, B, sb);
    switch (oa * 4 + ob) {
        TINA_MX_CASE(0, 0) TINA_MX_CASE(0, 1) TINA_MX_CASE(0, 2) TINA_MX_CASE(0, 3)
        TINA_MX_CASE(1, 0) TINA_MX_CASE(1, 1) TINA_MX_CASE(1, 2) TINA_MX_CASE(1, 3)
        TINA_MX_CASE(2, 0) TINA_MX_CASE(2, 1) TINA_MX_CASE(2, 2) TINA_MX_CASE(2, 3)
        TINA_MX_CASE(3, 0) TINA_MX_CASE(3, 1) TINA_MX_CASE(3, 2) default: break;
    }
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 3, sa, 3, sb);
#undef TINA_MX_CASE
}

template <int FORM, int NP, int RD, int WN>
__device__ __forceinline__ void mfma_slab(const uint4 (&af)[2][NP][RD], const uint4 (&bf)[WN][NP][RD],
                                          f32x16 (&acc)[2][WN], f32x16 (&acc2)[2][WN], const int (&sa)[2],
                                          const int (&sb)[WN]) {
    mfma_block<FORM, NP, RD, 2, WN>(af, bf, acc, acc2, sa, sb);
}

template <int FORM, int WN>
struct GemmSmem {
    static constexpr int NP = FT<FORM>::NP, BN = 64 * WN;
    uint8_t tiles[NP * (BM + BN) * RS];  // NP A pieces (BM rows), then NP B pieces (BN rows), RS bytes a row
};

// Map a logical tile index L of an nm x nn grid: groups of GROUP_M m-tiles
// sweep all n-tiles, so they share each B column block and their A rows.
__device__ inline void grouped_tile(int64_t L, int64_t nm, int64_t nn, int BN, int64_t& m0, int64_t& n0) {
    const int64_t gsz_full = GROUP_M * nn;
    const int64_t grp = L / gsz_full, first_m = grp * GROUP_M;
    const int64_t gsz = min((int64_t)GROUP_M, nm - first_m);
    const int64_t within = L - grp * gsz_full;
    m0 = (first_m + within % gsz) * BM;
    n0 = (within / gsz) * BN;
}

// Epilogue of a tile: combine pieces, undo the frame scale (s_sc, per-frame
// scaled forms), write complex64 rows.
template <int FORM, int WN>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int64_t m0, int64_t n0, const f32x16 (&acc)[2][WN],
                                              const f32x16 (&acc2)[2][WN], const float* s_sc) {
    using ft = FT<FORM>;
    constexpr int WC = 32 * WN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lh = lane >> 5;
    const float corr = (FORM == FORM_FP16X3) ? (1.0f / 2048.0f) : 1.0f;
    // Element v of block (bm, bn) sits at row rb + bm * 32 + 8 * (v >> 2) +
    // (v & 3) of the lane's column: its offset from the lane's first row is a
    // wave-uniform multiple of ldo.  Tiles with every row present skip the row
    // test; the zero imaginary parts of X_0 and X_{P/2} are written apart.
    const int64_t rb = m0 + wm * 64 + 4 * lh;
    float* const obase = g.out + rb * g.ldo;
    auto store_rows = [&](auto check_rows) {
        constexpr bool CHECK = decltype(check_rows)::value;
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
            const int64_t col = n0 + wn * WC + bn * 32 + lr;
            if (col >= g.N) continue;
            int64_t oc = col;
            if (g.real_pack) oc = col >= 2 ? col : (col == 0 ? 0 : (int64_t)g.N);
            float* const ocol = obase + oc;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int rr = bm * 32 + 8 * (v >> 2) + (v & 3);  // row offset from rb
                    if (CHECK && rb + rr >= g.F) continue;
                    float val = acc[bm][bn][v];
                    if constexpr (FORM == FORM_FP16X3) val += acc2[bm][bn][v] * corr;
                    if constexpr (ft::SCALED) val *= s_sc[wm * 64 + 4 * lh + rr];
                    ocol[(int64_t)rr * g.ldo] = val;
                }
            if (g.real_pack && col < 2) {  // Im X_0, Im X_{P/2}
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int rr = bm * 32 + 8 * (v >> 2) + (v & 3);
                        if (CHECK && rb + rr >= g.F) continue;
                        ocol[(int64_t)rr * g.ldo + 1] = 0.0f;
                    }
            }
        }
    };
    if (m0 + BM <= g.F) store_rows(std::false_type{});
    else store_rows(std::true_type{});
}


// One BM x BN output tile at (m0, n0), BN = 64 * WN: 2 x 2 waves, each
// 64 x 32 WN as 2 x WN MFMA blocks, with A read as FP32 rows: FP32, and bf16
// (one piece, or hi + lo) converted while it is staged (the synthesis bank's
// inverse DFT takes its FP32 channel frames this way).  The analysis bank's
// reduced forms take A in operand form from the FIR (gemm_tile_raw).  Called
// by every thread of the block.
//
// COMP (FP32): compensated K accumulation.  Each K tile's products go to
// block accumulators blk; at the tile's end the block sum is added to the
// running sum acc by an error-free transformation (Knuth's TwoSum), and the
// rounding error of that addition is where the next tile's block accumulation
// starts.  The error of the result is then that of summing one K tile (32
// products) plus one rounding per tile, instead of a rounding at the size of
// the whole running sum for each of the K products: channels far below the
// frame's strongest one keep their accuracy.
// Operand entries from the twiddle table tw (cos, sin of 2 pi r / P for
// r < P, FP32-rounded from FP64 as the materialised operand is), so both give
// the same bits.  Real input: row 0 is X_0, row 1 X_{P/2} (packed), row
// n >= 2 cos (even n) or -sin (odd n) of channel n / 2 at sample k.
__device__ __forceinline__ float table_entry_real(const float2* tw, int P, int n, int k) {
    if (n < 2) return (n == 1 && (k & 1)) ? -1.0f : 1.0f;
    const float2 t = tw[(k * (n >> 1)) & (P - 1)];
    return (n & 1) ? -t.y : t.x;
}

// Four entries Bt[n][k..k+3] (k a multiple of 4; K, a multiple of 4, bounds
// them all at once).  Complex input (n = 2 channel + im output, k = 2 sample
// + im input) reads the table twice, for samples k/2 and k/2 + 1 of channel
// n/2: (cos, sin) for the real output row, (-sin, cos) for the imaginary one.
// Real input reads it four times.
__device__ __forceinline__ float4 table_frag(const float2* tw, int P, bool cplx, int n, int k, int N, int K) {
    if (n >= N || k >= K) return make_float4(0.f, 0.f, 0.f, 0.f);
    if (cplx) {
        const int ch = n >> 1, p0 = k >> 1;
        const float2 t0 = tw[(p0 * ch) & (P - 1)], t1 = tw[((p0 + 1) * ch) & (P - 1)];
        return (n & 1) ? make_float4(-t0.y, t0.x, -t1.y, t1.x) : make_float4(t0.x, t0.y, t1.x, t1.y);
    }
    return make_float4(table_entry_real(tw, P, n, k), table_entry_real(tw, P, n, k + 1),
                       table_entry_real(tw, P, n, k + 2), table_entry_real(tw, P, n, k + 3));
}

template <int FORM, int WN, bool COMP = false, bool TABLE = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t m0, int64_t n0, GemmSmem<FORM, WN>& sm,
                                          const float2* tws = nullptr) {
    constexpr int BN = 64 * WN, WC = 32 * WN;  // block tile columns, columns per wave
    using ft = FT<FORM>;
    static_assert(FORM == FORM_FP32 || FORM == FORM_BF16 || FORM == FORM_BF16X3, "FP32 A, converted to bf16 at most");
    static_assert(!COMP || FORM == FORM_FP32, "compensated accumulation: FP32 products");
    constexpr int NP = ft::NP, EB = ft::EB, SLAB = ft::SLAB;
    constexpr int CPR = ROWB / 16;                // 16-byte chunks per row
    constexpr int BK = ROWB / EB;                 // K elements per tile
    constexpr int ACPR = BK / 4;                  // A float4 chunks per row
    constexpr int ACH = BM * ACPR / NT;           // A float4 chunks per thread (FP32 A)
    constexpr int BCH = BN * (ROWB / 16) / NT;    // B 16-byte chunks per thread per piece
    constexpr int NSLAB = ROWB / SLAB;
    constexpr int RD = SLAB / 32;                 // 16-byte reads per lane per slab

    uint8_t* As = sm.tiles;                 // NP pieces of BM x RS
    uint8_t* Bs = sm.tiles + NP * BM * RS;  // NP pieces of BN x RS (not used by the table form)
    const bool tcplx = !g.real_pack;        // table form: complex input, and P
    const int tP = tcplx ? g.K / 2 : g.K;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lh = lane >> 5;

    __syncthreads();  // the previous tile of a persistent block is done with LDS

    float4 ra[ACH];
    uint4 rb[NP][BCH];
    const uint8_t* Bp[2] = {(const uint8_t*)g.B0, (const uint8_t*)g.B1};
    const int64_t KB = (int64_t)g.K * EB;  // bytes per Bt row

    auto load_tile = [&](int k0) {
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
                const int c = tid + i * NT, row = c / CPR, kc = c % CPR;
                const int64_t n = n0 + row;
                const int64_t kb = (int64_t)k0 * EB + kc * 16;
                if constexpr (!TABLE) {  // the table form assembles its B fragments in the slab loop
                    if (n < g.N && kb < KB) rb[p][i] = *reinterpret_cast<const uint4*>(Bp[p] + n * KB + kb);
                    else rb[p][i] = make_uint4(0u, 0u, 0u, 0u);
                }
            }
    };

    auto store_tile = [&]() {
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
            }
        }
        if constexpr (!TABLE) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int i = 0; i < BCH; ++i) {
                    const int c = tid + i * NT, row = c / CPR, kc = c % CPR;
                    *reinterpret_cast<uint4*>(Bs + p * BN * RS + row * RS + kc * 16) = rb[p][i];
                }
        }
    };

    f32x16 acc[2][WN], acc2[2][WN];  // COMP: acc2 = the block accumulators
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) { acc[i][j][v] = 0.f; acc2[i][j][v] = 0.f; }

    const int nk = (g.K + BK - 1) / BK;
    load_tile(0);
    store_tile();
    __syncthreads();
    // Table form: the B fragments of slab (t, s) come from the table alone, so
    // those of the next slab are formed while this slab's products run.
    uint4 bnext[WN];
    auto table_frags = [&](int t, int s) {
#pragma unroll
        for (int bn = 0; bn < WN; ++bn)
            bnext[bn] = __builtin_bit_cast(uint4, table_frag(tws, tP, tcplx, (int)n0 + wn * WC + bn * 32 + lr,
                                                             t * BK + s * (SLAB / 4) + lh * 4, g.N, g.K));
    };
    if constexpr (TABLE) {
        static_assert(NP == 1 && RD == 1 && FORM == FORM_FP32, "the table form is FP32");
        table_frags(0, 0);
    }
    for (int t = 0; t < nk; ++t) {
        if (t + 1 < nk) load_tile((t + 1) * BK);
#pragma unroll
        for (int s = 0; s < NSLAB; ++s) {
            uint4 af[2][NP][RD], bf[WN][NP][RD];
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
            for (int bn = 0; bn < WN; ++bn)
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int q = 0; q < RD; ++q) {
                        const int row = wn * WC + bn * 32 + lr;
                        if constexpr (TABLE) {
                            bf[bn][p][q] = bnext[bn];  // formed during the previous slab
                        } else {
                            bf[bn][p][q] = *reinterpret_cast<const uint4*>(Bs + p * BN * RS + row * RS + off(q));
                        }
                    }
            if constexpr (TABLE) {  // the next slab's fragments (past the last: repeats in-range reads)
                if (s + 1 < NSLAB) table_frags(t, s + 1);
                else table_frags(t + 1 < nk ? t + 1 : t, 0);
            }
            const int sa[2] = {0, 0}, sb[WN] = {};
            if constexpr (COMP) mfma_slab<FORM, NP, RD, WN>(af, bf, acc2, acc, sa, sb);
            else mfma_slab<FORM, NP, RD, WN>(af, bf, acc, acc2, sa, sb);
        }
        if constexpr (COMP) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const float a = acc[i][j][v], b = acc2[i][j][v];
                        const float sum = a + b, bv = sum - a;
                        acc2[i][j][v] = (a - (sum - bv)) + (b - bv);
                        acc[i][j][v] = sum;
                    }
        }
        __syncthreads();
        if (t + 1 < nk) {
            store_tile();
            __syncthreads();
        }
    }
    if constexpr (COMP) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[i][j][v] += acc2[i][j][v];
    }

    gemm_epilogue<FORM, WN>(g, m0, n0, acc, acc2, nullptr);
}

// FIR fused into the FP32 GEMM: the A tile of K tile t (frames m0.., K
// columns k0..k0+BK) is computed in the tile from the input stream instead of
// being read from a workspace the FIR kernel wrote.  The BM + M - 1 input
// rows it needs (frame f of the tile reads frames f - M + 1..f) and the taps
// of its columns are staged in LDS with the B tile; then every thread forms
// its A chunks with the FIR kernel's FMA order (tap 0 times the newest frame,
// then fused multiply-adds for m = 1..M-1), so A -- and the output -- are bit
// for bit those of the two-kernel path.  MT: the largest M (compile time);
// EXACT: M == MT.
struct FusedArgs {
    GemmArgs g;   // g.A unused
    FirArgs x;    // input stream, taps, frame numbering (x.y unused)
};

template <int WN, int MT>
struct FusedSmem {
    static constexpr int BN = 64 * WN, BK = ROWB / 4, XR = BM + MT - 1;
    uint8_t tiles[(BM + BN) * RS];  // A (BM rows), then B (BN rows), RS bytes a row
    float4 xs[XR * (BK / 4)];       // input rows of the K tile, BK floats each (no pad: 16 lanes read 2 rows)
    float ts[MT * BK];              // taps of the K tile's columns, tap m at ts[m * BK + column]
};

template <int WN, int MT, bool EXACT>
__device__ __forceinline__ void gemm_tile_fused(const FusedArgs& fa, int64_t m0, int64_t n0, FusedSmem<WN, MT>& sm) {
    constexpr int FORM = FORM_FP32;
    constexpr int BN = 64 * WN, WC = 32 * WN;
    constexpr int BK = ROWB / 4, K4 = BK / 4;           // K floats per tile, float4 chunks per row
    constexpr int XR = BM + MT - 1;                      // input rows staged per K tile
    constexpr int XCH = (XR * K4 + NT - 1) / NT;         // input float4 chunks per thread
    constexpr int TCH = (MT * BK + NT - 1) / NT;         // taps per thread
    constexpr int ACH = BM * K4 / NT;                    // A chunks per thread
    constexpr int BCH = BN * (ROWB / 16) / NT;
    constexpr int NSLAB = ROWB / FT<FORM>::SLAB, SLAB = FT<FORM>::SLAB, RD = 1;
    const GemmArgs& g = fa.g;
    const FirArgs& a = fa.x;
    const int M = EXACT ? MT : a.M;

    uint8_t* As = sm.tiles;
    uint8_t* Bs = sm.tiles + BM * RS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lh = lane >> 5;
    const int64_t KB = (int64_t)g.K * 4;
    const int64_t x0 = m0 - (M - 1);  // frame of staged row 0 (may be negative: history)

    float4 rx[XCH];
    float rt[TCH];
    uint4 rb[BCH];
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int i = 0; i < XCH; ++i) {
            const int c = tid + i * NT, j = c / K4, k4 = c % K4;
            const int64_t f = x0 + j;  // frame of this row
            rx[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < BM + M - 1 && f < g.F) {
                const int64_t e = (a.g0 + f + a.M - 1) * (int64_t)a.W + k0 + 4 * k4;  // float in prefix ++ chunk
                const float* p = e >= a.plen ? a.chunk + (e - a.plen) : a.prefix + e;
                if (e >= a.plen || a.prefix) rx[i] = *reinterpret_cast<const float4*>(p);
            }
        }
#pragma unroll
        for (int i = 0; i < TCH; ++i) {
            const int c = tid + i * NT, m = c / BK, kk = c % BK;
            rt[i] = (c < MT * BK && (EXACT || m < M)) ? a.taps[(int64_t)(M - 1 - m) * a.P + (k0 + kk) / a.cf] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < BCH; ++i) {
            const int c = tid + i * NT, row = c >> 3, kc = c & 7;
            const int64_t n = n0 + row, kb = (int64_t)k0 * 4 + kc * 16;
            rb[i] = (n < g.N && kb < KB) ? *reinterpret_cast<const uint4*>((const uint8_t*)g.B0 + n * KB + kb)
                                         : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    // Stage the loaded tile, then form A in LDS.  Contains a barrier: called
    // by every thread at the same point.
    auto store_tile = [&]() {
#pragma unroll
        for (int i = 0; i < XCH; ++i) {
            const int c = tid + i * NT;
            if (c < XR * K4) sm.xs[c] = rx[i];
        }
#pragma unroll
        for (int i = 0; i < TCH; ++i) {
            const int c = tid + i * NT;
            if (c < MT * BK) sm.ts[c] = rt[i];
        }
#pragma unroll
        for (int i = 0; i < BCH; ++i) {
            const int c = tid + i * NT, row = c >> 3, kc = c & 7;
            *reinterpret_cast<uint4*>(Bs + row * RS + kc * 16) = rb[i];
        }
        __syncthreads();
        // A thread's ACH chunks share its column group k4 = tid % K4 (NT is a
        // multiple of K4), so they share the taps; rows r = tid / K4 + i NT / K4.
        const int k4 = tid % K4, r0 = tid / K4;
        const float4* xr = sm.xs + (r0 + M - 1) * K4 + k4;  // staged row of frame m0 + r0
        float4 fa4[ACH];
        {
            const float4 t = *reinterpret_cast<const float4*>(sm.ts + 4 * k4);
#pragma unroll
            for (int i = 0; i < ACH; ++i) {
                const float4 v = xr[i * (NT / K4) * K4];
                fa4[i] = make_float4(t.x * v.x, t.y * v.y, t.z * v.z, t.w * v.w);
            }
        }
#pragma unroll 2
        for (int m = 1; m < (EXACT ? MT : M); ++m) {
            const float4 t = *reinterpret_cast<const float4*>(sm.ts + m * BK + 4 * k4);
#pragma unroll
            for (int i = 0; i < ACH; ++i) {
                const float4 v = xr[i * (NT / K4) * K4 - m * K4];
                fa4[i].x = fmaf(t.x, v.x, fa4[i].x);
                fa4[i].y = fmaf(t.y, v.y, fa4[i].y);
                fa4[i].z = fmaf(t.z, v.z, fa4[i].z);
                fa4[i].w = fmaf(t.w, v.w, fa4[i].w);
            }
        }
#pragma unroll
        for (int i = 0; i < ACH; ++i)
            *reinterpret_cast<float4*>(As + (r0 + i * (NT / K4)) * RS + k4 * 16) = fa4[i];
    };

    f32x16 acc[2][WN], acc2[2][WN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    __syncthreads();  // the previous tile of a persistent block is done with LDS
    const int nk = (g.K + BK - 1) / BK;
    load_tile(0);
    store_tile();
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        if (t + 1 < nk) load_tile((t + 1) * BK);
#pragma unroll
        for (int s = 0; s < NSLAB; ++s) {
            uint4 af[2][1][RD], bf[WN][1][RD];
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
                af[bm][0][0] = *reinterpret_cast<const uint4*>(As + (wm * 64 + bm * 32 + lr) * RS + s * SLAB + lh * 16);
#pragma unroll
            for (int bn = 0; bn < WN; ++bn)
                bf[bn][0][0] = *reinterpret_cast<const uint4*>(Bs + (wn * WC + bn * 32 + lr) * RS + s * SLAB + lh * 16);
            const int sa[2] = {0, 0}, sb[WN] = {};
            mfma_slab<FORM, 1, RD, WN>(af, bf, acc, acc2, sa, sb);
        }
        __syncthreads();
        if (t + 1 < nk) {
            store_tile();
            __syncthreads();
        }
    }
    gemm_epilogue<FORM, WN>(g, m0, n0, acc, acc2, nullptr);
}

// Raw-operand tile: A arrives in the operand form (NP pieces of EB-byte
// elements, K contiguous, row stride g.lda elements; block-scaled FP8 also
// with a scale byte per 32 K; per-frame scaled forms with the frame's
// exponent in g.fexp, undone in the epilogue), so a K tile of A is copied to
// LDS like B, with no conversion and a quarter (FP8) or half (16-bit) of the
// FP32 A registers.
// One-piece forms keep two LDS buffers, so one barrier per K tile suffices
// and the stores of tile t + 1 overlap other waves' products on tile t;
// two-piece forms keep one buffer (two barriers).
template <int FORM, int WN>
struct RawSmem {
    static constexpr int NP = FT<FORM>::NP, BN = 64 * WN, LB = NP == 1 ? 2 : 1;
    uint8_t tiles[LB][NP * (BM + BN) * RS];
    uint32_t mxs[LB][FT<FORM>::MX ? BM + BN : 1];  // scale words of the K tile: A rows, then B rows
    float fsc[FT<FORM>::SCALED ? BM : 1];           // per-frame scaled forms: 2^e_f of the tile's rows
};

template <int FORM, int WN>
__device__ __forceinline__ void gemm_tile_raw(const GemmArgs& g, int64_t m0, int64_t n0, RawSmem<FORM, WN>& sm) {
    using ft = FT<FORM>;
    constexpr int BN = 64 * WN, WC = 32 * WN;
    constexpr int NP = ft::NP, EB = ft::EB, SLAB = ft::SLAB, LB = RawSmem<FORM, WN>::LB;
    constexpr int BK = ROWB / EB;               // K elements per tile
    constexpr int QCH = BM * (ROWB / 16) / NT;  // A 16-byte chunks per thread per piece
    constexpr int BCH = BN * (ROWB / 16) / NT;  // B 16-byte chunks per thread per piece
    constexpr int NSLAB = ROWB / SLAB;
    constexpr int RD = SLAB / 32;
    static_assert(!ft::MX || (BM + BN == NT && NP == 1), "block-scaled form: one scale word per thread");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 31, lh = lane >> 5;
    const uint8_t* Ap[2] = {g.Aq, g.Aq1};
    const uint8_t* Bp[2] = {(const uint8_t*)g.B0, (const uint8_t*)g.B1};
    const int64_t AB = g.lda * EB, KB = (int64_t)g.K * EB;  // bytes per A row, valid bytes per row
    const int64_t nb = g.K / 32;                             // scale bytes per row (block-scaled form)

    struct Stage {
        uint4 a[NP][QCH];
        uint4 b[NP][BCH];
        uint32_t sc;
    };
    auto load = [&](Stage& r, int k0) {
        const int64_t kb0 = (int64_t)k0 * EB;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < QCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                const int64_t f = m0 + row, kb = kb0 + kc * 16;
                r.a[p][i] = (f < g.F && kb < KB) ? *reinterpret_cast<const uint4*>(Ap[p] + f * AB + kb)
                                                 : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                const int64_t n = n0 + row, kb = kb0 + kc * 16;
                r.b[p][i] = (n < g.N && kb < KB) ? *reinterpret_cast<const uint4*>(Bp[p] + n * KB + kb)
                                                 : make_uint4(0u, 0u, 0u, 0u);
            }
        }
        if constexpr (ft::MX) {  // K % 128 == 0 (checked at plan time): whole 4-byte scale words
            if (tid < BM) {
                const int64_t f = m0 + tid;
                r.sc = f < g.F ? *reinterpret_cast<const uint32_t*>(g.Aqs + f * nb + k0 / 32) : 0x7f7f7f7fu;
            } else {
                const int64_t n = n0 + tid - BM;
                r.sc = n < g.N ? *reinterpret_cast<const uint32_t*>((const uint8_t*)g.B1 + n * nb + k0 / 32)
                               : 0x7f7f7f7fu;
            }
        }
    };
    auto store = [&](const Stage& r, int buf) {
        uint8_t* As = sm.tiles[buf];
        uint8_t* Bs = sm.tiles[buf] + NP * BM * RS;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < QCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                *reinterpret_cast<uint4*>(As + p * BM * RS + row * RS + kc * 16) = r.a[p][i];
            }
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NT, row = c >> 3, kc = c & 7;
                *reinterpret_cast<uint4*>(Bs + p * BN * RS + row * RS + kc * 16) = r.b[p][i];
            }
        }
        if constexpr (ft::MX) sm.mxs[buf][tid] = r.sc;
    };

    f32x16 acc[2][WN], acc2[2][WN];  // acc2: the fp16 cross terms (FP16X3 only)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[i][j][v] = 0.f;
                if constexpr (FORM == FORM_FP16X3) acc2[i][j][v] = 0.f;
            }

    auto compute = [&](int buf) {
        const uint8_t* As = sm.tiles[buf];
        const uint8_t* Bs = sm.tiles[buf] + NP * BM * RS;
#pragma unroll
        for (int s = 0; s < NSLAB; ++s) {
            uint4 af[2][NP][RD], bf[WN][NP][RD];
            // For the 64-K FP8 MFMA these reads make the instruction's K index
            // equal to the byte offset in the slab (bytes 0-15 of lane half lh
            // are K 16 lh.., bytes 16-31 are K 32 + 16 lh..), so its 32-K scale
            // block b is bytes [32 b, 32 b + 32) of the slab, whose scale lane
            // half b supplies.
            auto off = [&](int q) { return s * SLAB + q * 32 + lh * 16; };
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int q = 0; q < RD; ++q)
                        af[bm][p][q] = *reinterpret_cast<const uint4*>(As + p * BM * RS + (wm * 64 + bm * 32 + lr) * RS + off(q));
#pragma unroll
            for (int bn = 0; bn < WN; ++bn)
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int q = 0; q < RD; ++q)
                        bf[bn][p][q] = *reinterpret_cast<const uint4*>(Bs + p * BN * RS + (wn * WC + bn * 32 + lr) * RS + off(q));
            int sa[2] = {0, 0}, sb[WN] = {};
            if constexpr (ft::MX) {
                const int sh = 8 * (2 * s + lh);  // byte of the word = 32-K block of the K tile
#pragma unroll
                for (int b = 0; b < 2; ++b) sa[b] = (int)(sm.mxs[buf][wm * 64 + b * 32 + lr] >> sh);
#pragma unroll
                for (int b = 0; b < WN; ++b) sb[b] = (int)(sm.mxs[buf][BM + wn * WC + b * 32 + lr] >> sh);
            }
            mfma_slab<FORM, NP, RD, WN>(af, bf, acc, acc2, sa, sb);
        }
    };

    __syncthreads();  // the previous tile of a persistent block is done with LDS
    if constexpr (ft::SCALED) {  // read by the epilogue, after the barriers below
        if (tid < BM) sm.fsc[tid] = m0 + tid < g.F ? ldexpf(1.0f, g.fexp[m0 + tid]) : 1.0f;
    }
    const int nk = (g.K + BK - 1) / BK;
    Stage r;
    load(r, 0);
    store(r, 0);
    if (nk > 1) load(r, BK);
    __syncthreads();
    // Tile t sits in LDS buffer t % LB.  While tile t is multiplied, the
    // registers hold tile t + 1; it is then stored to the other buffer and the
    // loads of tile t + 2 are issued.
    for (int t = 0; t < nk; ++t) {
        compute(LB == 2 ? (t & 1) : 0);
        if constexpr (LB == 1) __syncthreads();
        if (t + 1 < nk) {
            store(r, LB == 2 ? ((t + 1) & 1) : 0);
            if (t + 2 < nk) load(r, (t + 2) * BK);
        }
        __syncthreads();
    }
    gemm_epilogue<FORM, WN>(g, m0, n0, acc, acc2, ft::SCALED ? sm.fsc : nullptr);
}

// ------------------------------------------------------------- wide tiles
// Raw-operand tile for the single-stream path: 8 waves (512 threads) in a
// WGM x WGN grid, each wave TM x TN MFMA 32 x 32 blocks, so that each 16-byte
// LDS read feeds more MFMA cycles and each byte fetched from L2 feeds more
// products than in the 128 x 128 tile (whose two 64 x 64-wave blocks per CU
// need as many LDS bytes per cycle as the LDS delivers).  One block per CU:
// two LDS stages of K tiles (one barrier per K tile), the next tile's global
// loads in flight in registers during a whole K tile of products.
// ROWB: bytes of an operand row per K tile and piece (two 64-K slabs for
// per-frame FP8; one for block-scaled FP8, whose scale words with two slabs'
// fragments would not fit the registers).
template <int FORM> struct WideCfg {  // 256 x 256 tiles, waves of 128 x 64
    static constexpr int WGM = 2, WGN = 4, TM = 4, TN = 2;
    static constexpr int ROWB = FORM == FORM_MXFP8 ? 64 : 128 / FT<FORM>::NP;
};
template <> struct WideCfg<FORM_FP16X3> {  // two accumulators: 128 x 256 tiles, waves of 64 x 64
    static constexpr int WGM = 2, WGN = 4, TM = 2, TN = 2, ROWB = 64;
};

template <int FORM>
struct WideGeom {
    using cfg = WideCfg<FORM>;
    static constexpr int WGM = cfg::WGM, WGN = cfg::WGN, TM = cfg::TM, TN = cfg::TN;
    static constexpr int NP = FT<FORM>::NP, EB = FT<FORM>::EB, SLAB = FT<FORM>::SLAB, RD = SLAB / 32;
    static constexpr int NTH = 64 * WGM * WGN;
    static constexpr int BM = 32 * WGM * TM, BN = 32 * WGN * TN;
    static constexpr int ROWB = cfg::ROWB;
    static constexpr int RS = ROWB + 16;    // LDS row stride: 16 rows of 16-byte reads hit distinct banks
    static constexpr int CPR = ROWB / 16;   // 16-byte chunks per row
    static constexpr int STAGE = NP * (BM + BN) * RS;
    static constexpr int QCH = BM * CPR / NTH, BCH = BN * CPR / NTH;  // chunks per thread per piece
    static constexpr int BK = ROWB / EB;    // K elements per tile
    static constexpr int NSLAB = ROWB / SLAB;
    static_assert(BM * CPR % NTH == 0 && BN * CPR % NTH == 0, "whole chunks per thread");
    static_assert(NSLAB >= 1, "a K tile holds whole MFMA slabs");
};

// Scale groups (block-scaled form) and frame scales (per-frame scaled forms)
// as empty bases when unused, so the bf16 hi + lo form's two stages fill the
// 160 KiB of LDS exactly.  A scale group holds the E8M0 scales of 8 64-K
// slabs arranged for the MFMA's scale operand: for slab k, wave row (column)
// block w, lane row r and lane half h, one word (half-word for the two column
// blocks) whose byte x is the scale of MFMA block row (column) x -- the
// block's operand selector picks it.
template <int WGM, int WGN, bool ON> struct WideMx {
    uint32_t mxa[2][8][WGM][64];
    uint16_t mxb[2][8][WGN][64];
};
template <int WGM, int WGN> struct WideMx<WGM, WGN, false> {};
template <int N, bool ON> struct WideFsc { float fsc[N]; };
template <int N> struct WideFsc<N, false> {};

template <int FORM>
struct WideSmem : WideMx<WideGeom<FORM>::WGM, WideGeom<FORM>::WGN, FT<FORM>::MX>,
                  WideFsc<WideGeom<FORM>::BM, FT<FORM>::SCALED> {
    uint8_t tiles[2][WideGeom<FORM>::STAGE];
};

constexpr int WIDE_GROUP_M = 8;  // m-tiles swept per column of n-tiles (a CU-round of an XCD is ~ 8 x 4 tiles)

template <int FORM>
__device__ __forceinline__ void gemm_tile_wide(const GemmArgs& g, int64_t m0, int64_t n0, WideSmem<FORM>& sm) {
    using G = WideGeom<FORM>;
    using ft = FT<FORM>;
    constexpr int NP = G::NP, EB = G::EB, SLAB = G::SLAB, RD = G::RD, RS = G::RS, CPR = G::CPR;
    constexpr int TM = G::TM, TN = G::TN, NTH = G::NTH, BM = G::BM, BN = G::BN, BK = G::BK;
    constexpr int QCH = G::QCH, BCH = G::BCH, NSLAB = G::NSLAB;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / G::WGN, wn = wave % G::WGN;
    const int lr = lane & 31, lh = lane >> 5;
    const uint8_t* Ap[2] = {g.Aq, g.Aq1};
    const uint8_t* Bp[2] = {(const uint8_t*)g.B0, (const uint8_t*)g.B1};
    const int64_t AB = g.lda * EB, KB = (int64_t)g.K * EB;
    const int64_t nb = g.K / 32;

    // Buffer loads: a resource per operand piece based at the tile's first
    // row, its range ending at the last row present (rows past it read as
    // zero), a per-chunk lane offset that stays fixed, and the K tile's byte
    // offset as the scalar offset.  K is a whole number of K tiles.
    __amdgpu_buffer_rsrc_t ra[NP], rbs[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int64_t ar = g.F - m0 < BM ? g.F - m0 : BM, br = g.N - n0 < BN ? g.N - n0 : BN;
        ra[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(Ap[p] + m0 * AB), (short)0,
                                                  (int)(ar * AB), 0x00020000);
        rbs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(Bp[p] + n0 * KB), (short)0,
                                                   (int)(br * KB), 0x00020000);
    }
    uint32_t va[QCH], vb[BCH];
#pragma unroll
    for (int i = 0; i < QCH; ++i) {
        const int c = tid + i * NTH;
        va[i] = (uint32_t)((c / CPR) * AB + (c % CPR) * 16);
    }
#pragma unroll
    for (int i = 0; i < BCH; ++i) {
        const int c = tid + i * NTH;
        vb[i] = (uint32_t)((c / CPR) * KB + (c % CPR) * 16);
    }
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

    struct Stage {
        uint4 a[NP][QCH];
        uint4 b[NP][BCH];
    };
    // Block-scaled form: the scale bytes of a row (2 per 64-K slab, K % 128
    // == 0) move in groups of 16 bytes -- 8 slabs, SPG K tiles -- one row per
    // thread (A rows, then B rows), through two LDS group buffers chosen by
    // group parity.  Group g + 1 is loaded when group g's first tile starts
    // and stored SPG / 2 tiles later, after the last reads of group g - 1 from
    // the same buffer and before group g + 1's first reads; the lane then
    // reads its word for the slab and lane half straight into the scale
    // operand.  Buffer loads: bytes past a row's end are the next row's (for K
    // tiles that do not exist), past the last row zero.
    constexpr int SPG = 8 / NSLAB;                                        // K tiles per scale group
    const int ng = ((g.K + BK - 1) / BK + SPG - 1) / SPG;  // scale groups (block-scaled form)
    __amdgpu_buffer_rsrc_t rsc = ra[0];
    uint32_t vsc = 0;
    uint4 scn = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (ft::MX) {
        static_assert(BM + BN == NTH && BM % 64 == 0 && 8 % NSLAB == 0 && SPG >= 2 && TM <= 4 && TN <= 2,
                      "one scale row per thread, whole waves per operand, a scale byte per MFMA block");
        const int64_t ar = g.F - m0 < BM ? g.F - m0 : BM, br = g.N - n0 < BN ? g.N - n0 : BN;
        if (__builtin_amdgcn_readfirstlane(wave) < BM / 64) {
            rsc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.Aqs + m0 * nb), (short)0, (int)(ar * nb), 0x00020000);
            vsc = (uint32_t)(tid * nb);
        } else {
            rsc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>((const uint8_t*)g.B1 + n0 * nb), (short)0,
                                                    (int)(br * nb), 0x00020000);
            vsc = (uint32_t)((tid - BM) * nb);
        }
    }
    auto load_group = [&](int gi) {
        return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rsc, vsc, gi * 16, 0));
    };
    auto store_group = [&](int slot, uint4 v) {
        if constexpr (ft::MX) {
            // This thread's row: block x of wave row (column) block w, lane row r.
            const bool isa = __builtin_amdgcn_readfirstlane(wave) < BM / 64;
            const int rr = isa ? tid : tid - BM, r = rr & 31, x = (rr >> 5) % (isa ? TM : TN), w = (rr >> 5) / (isa ? TM : TN);
            uint8_t* base = isa ? reinterpret_cast<uint8_t*>(&sm.mxa[slot][0][w][0])
                                : reinterpret_cast<uint8_t*>(&sm.mxb[slot][0][w][0]);
            const int wb = isa ? 4 : 2;                           // bytes per entry
            const int kstride = wb * 64 * (isa ? G::WGM : G::WGN);  // bytes from one 64-K slab to the next
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 8; ++k)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    base[k * kstride + (2 * r + h) * wb + x] = (uint8_t)(wv[k >> 1] >> (8 * (2 * (k & 1) + h)));
        }
    };
    auto load = [&](Stage& r, int k0) {
        const int32_t kb0 = k0 * EB;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < QCH; ++i)
                r.a[p][i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(ra[p], va[i], kb0, 0));
#pragma unroll
            for (int i = 0; i < BCH; ++i)
                r.b[p][i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rbs[p], vb[i], kb0, 0));
        }
    };
    auto store = [&](const Stage& r, int buf) {
        uint8_t* As = sm.tiles[buf];
        uint8_t* Bs = sm.tiles[buf] + NP * BM * RS;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < QCH; ++i) {
                const int c = tid + i * NTH, row = c / CPR, kc = c % CPR;
                *reinterpret_cast<uint4*>(As + p * BM * RS + row * RS + kc * 16) = r.a[p][i];
            }
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                const int c = tid + i * NTH, row = c / CPR, kc = c % CPR;
                *reinterpret_cast<uint4*>(Bs + p * BN * RS + row * RS + kc * 16) = r.b[p][i];
            }
        }
    };

    f32x16 acc[TM][TN], acc2[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[i][j][v] = 0.f;
                if constexpr (FORM == FORM_FP16X3) acc2[i][j][v] = 0.f;
            }

    __syncthreads();
    if constexpr (ft::SCALED) {
        for (int i = tid; i < BM; i += NTH) sm.fsc[i] = m0 + i < g.F ? ldexpf(1.0f, g.fexp[m0 + i]) : 1.0f;
    }
    const int nk = (g.K + BK - 1) / BK;

    {
        // A software pipeline over units (slab s, MFMA block row bm) of every
        // K tile.  The A fragment(s) of unit u + 2 and the B fragments of the
        // next slab are read while unit u's products run; the next tile's LDS
        // stores and the global loads of the tile after it are spread over the
        // tile's first units; and the last two units' products are issued
        // after the barrier, behind the reads of the next tile's first units,
        // so the matrix units keep working across the barrier.  A fence after
        // each unit keeps this order.  For the 64-K FP8 instruction an operand
        // is two 16-byte reads, 32 bytes apart.  Split forms issue their three
        // products (hi hi, hi lo, lo hi) per accumulator in that order, slab by
        // slab, as the 128 x 128 tile does, so both give the same bits.
        typedef int i32x4 __attribute__((ext_vector_type(4)));
        using FragT = std::conditional_t<RD == 2, i32x8, uint4>;
        constexpr int U = NSLAB * TM, NCH = NP * (QCH + BCH), CPU = (NCH + U - 3) / (U - 2);
        static_assert(U % 4 == 0, "the A ring of 4 fragments wraps at tile boundaries");
        auto rd = [&](const uint8_t* p) -> FragT {
            if constexpr (RD == 2) {
                const i32x4 lo = *reinterpret_cast<const i32x4*>(p);
                const i32x4 hi = *reinterpret_cast<const i32x4*>(p + 32);
                return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            } else {
                return *reinterpret_cast<const uint4*>(p);
            }
        };
        FragT a[4][NP], b[2][TN][NP];
        int sa[2], sb[2];  // block-scaled form: scale words, byte x for MFMA block row / column x
        auto rdA = [&](int buf, int u, FragT (&d)[NP]) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
                d[p] = rd(sm.tiles[buf] + p * BM * RS + ((wm * TM + u % TM) * 32 + lr) * RS + (u / TM) * SLAB + lh * 16);
        };
        auto rdB = [&](int buf, int sl, int par, int kt) {
            const uint8_t* Bs = sm.tiles[buf] + NP * BM * RS;
#pragma unroll
            for (int bn = 0; bn < TN; ++bn)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    b[par][bn][p] = rd(Bs + p * BN * RS + ((wn * TN + bn) * 32 + lr) * RS + sl * SLAB + lh * 16);
            sa[par] = 0x7f7f7f7f;
            sb[par] = 0x7f7f7f7f;
            if constexpr (ft::MX) {  // slab sl of K tile kt: the lane's row, the lane half's 32-K block
                const int ks = kt * NSLAB + sl, slot = (ks >> 3) & 1;
                sa[par] = (int)sm.mxa[slot][ks & 7][wm][2 * lr + lh];
                sb[par] = (int)sm.mxb[slot][ks & 7][wn][2 * lr + lh];
            }
        };
        auto mf = [&](int u, int par) {
            const int bm = u % TM;
            constexpr int NTERM = NP == 2 ? 3 : 1;
#pragma unroll
            for (int term = 0; term < NTERM; ++term)
#pragma unroll
                for (int bn = 0; bn < TN; ++bn) {
                    const FragT& x = a[u % 4][term == 2 ? 1 : 0];
                    const FragT& y = b[par][bn][term == 1 ? 1 : 0];
                    if constexpr (FORM == FORM_BF16 || FORM == FORM_BF16X3)
                        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x),
                                                                              __builtin_bit_cast(bf16x8, y), acc[bm][bn], 0, 0, 0);
                    else if constexpr (FORM == FORM_FP16 || FORM == FORM_FP16X3) {
                        // FP16X3: the cross terms carry the lo pieces' 2^11 and go to acc2.
                        if (term == 0)
                            acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, x),
                                                                                 __builtin_bit_cast(f16x8, y), acc[bm][bn], 0, 0, 0);
                        else
                            acc2[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, x),
                                                                                  __builtin_bit_cast(f16x8, y), acc2[bm][bn], 0, 0, 0);
                    } else {  // FP8 E4M3 operands (formats 0/0) with unit or block scales, byte bm / bn of the scale words
                        acc[bm][bn] = mfma_f8_scaled_sel(x, y, acc[bm][bn], sa[par], sb[par], bm, bn);
                    }
                }
        };
        // One K tile t in LDS buffer tt (tiles alternate buffers; the loop
        // below is unrolled by two so that tt and every register index are
        // compile-time constants).  On entry the reads of units 0 and 1 and of
        // slab 0's B fragments are in flight; r holds tile t + 1.  At the last
        // tile the stores, loads and next-tile reads repeat valid addresses
        // and go unused.
        Stage r;
        auto tile = [&](int t, int tt) {
            const int nbuf = tt ^ 1, par0 = (tt * NSLAB) & 1;
            const int t2 = t + 2 < nk ? t + 2 : nk - 1;
            const int32_t kb2 = t2 * BK * EB;
#pragma unroll
            for (int u = 0; u < U - 2; ++u) {
                const int u2 = u + 2, s2 = u2 / TM;
                if (u2 % TM == 0) rdB(tt, s2, (par0 + s2) & 1, t);
                rdA(tt, u2, a[u2 % 4]);
                // The next tile's LDS stores and the loads of the tile after
                // it, CPU chunks per unit, each chunk's load reissued right
                // after its store frees the registers.
#pragma unroll
                for (int cc = 0; cc < CPU; ++cc) {
                    const int c = u * CPU + cc, p = c / (QCH + BCH), q = c % (QCH + BCH);
                    if (c >= NCH) continue;
                    if (q < QCH) {
                        const int e = tid + q * NTH;
                        *reinterpret_cast<uint4*>(sm.tiles[nbuf] + p * BM * RS + (e / CPR) * RS + (e % CPR) * 16) =
                            r.a[p][q];
                        r.a[p][q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(ra[p], va[q], kb2, 0));
                    } else {
                        const int e = tid + (q - QCH) * NTH;
                        *reinterpret_cast<uint4*>(sm.tiles[nbuf] + NP * BM * RS + p * BN * RS + (e / CPR) * RS +
                                                  (e % CPR) * 16) = r.b[p][q - QCH];
                        r.b[p][q - QCH] =
                            __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rbs[p], vb[q - QCH], kb2, 0));
                    }
                }
                if constexpr (ft::MX) {
                    const int gi = t / SPG;
                    if (u == 0 && gi >= 1 && gi + 1 < ng) {
                        if (t % SPG == 0) scn = load_group(gi + 1);
                        if (t % SPG == SPG / 2) store_group((gi + 1) & 1, scn);
                    }
                }
                mf(u, (par0 + u / TM) & 1);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            rdB(nbuf, 0, (par0 + NSLAB) & 1, t + 1);
            rdA(nbuf, 0, a[0]);
            rdA(nbuf, 1, a[1]);
            mf(U - 2, (par0 + NSLAB - 1) & 1);
            mf(U - 1, (par0 + NSLAB - 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
        };
        {
            // Both first tiles' loads in flight together: one memory latency
            // before the first products, not two.
            Stage r0;
            uint4 g0, g1;
            if constexpr (ft::MX) {
                g0 = load_group(0);
                g1 = ng > 1 ? load_group(1) : g0;
            }
            load(r0, 0);
            load(r, (nk > 1 ? 1 : 0) * BK);
            store(r0, 0);
            if constexpr (ft::MX) {
                store_group(0, g0);
                store_group(1, g1);
            }
        }
        __syncthreads();
        rdB(0, 0, 0, 0);
        rdA(0, 0, a[0]);
        rdA(0, 1, a[1]);
        for (int t = 0; t < nk; t += 2) {
            tile(t, 0);
            if (t + 1 < nk) tile(t + 1, 1);
        }
    }

    // Epilogue: element v of block (bm, bn) is row 32 (wm TM + bm) + 8 (v >> 2) +
    // 4 lh + (v & 3), column 32 (wn TN + bn) + lr of the tile.  Buffer stores
    // on a resource that ends at the last frame (stores past it are dropped):
    // the lane's row and column are its vector offset, the element's row
    // offset (a compile-time multiple of the row stride) the scalar offset.
    const float corr = (FORM == FORM_FP16X3) ? (1.0f / 2048.0f) : 1.0f;
    const int64_t rows = g.F - m0 < BM ? g.F - m0 : BM;
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(g.out + m0 * g.ldo, (short)0,
                                                                          (int)(rows * g.ldo * 4), 0x00020000);
    const int rl = wm * TM * 32 + 4 * lh;  // the lane's first row in the tile
    const int32_t ldo4 = (int32_t)g.ldo * 4;
#pragma unroll
    for (int bn = 0; bn < TN; ++bn) {
        const int64_t col = n0 + (wn * TN + bn) * 32 + lr;
        if (col >= g.N) continue;
        int64_t oc = col;
        if (g.real_pack) oc = col >= 2 ? col : (col == 0 ? 0 : (int64_t)g.N);
        const uint32_t vo = (uint32_t)((rl * g.ldo + oc) * 4);
#pragma unroll
        for (int bm = 0; bm < TM; ++bm)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int rr = bm * 32 + 8 * (v >> 2) + (v & 3);
                float val = acc[bm][bn][v];
                if constexpr (FORM == FORM_FP16X3) val += acc2[bm][bn][v] * corr;
                if constexpr (ft::SCALED) val *= sm.fsc[rl + rr];
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, val), ro, vo, rr * ldo4, 0);
            }
        if (g.real_pack && col < 2) {  // Im X_0, Im X_{P/2}
#pragma unroll
            for (int bm = 0; bm < TM; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int rr = bm * 32 + 8 * (v >> 2) + (v & 3);
                    __builtin_amdgcn_raw_buffer_store_b32(0u, ro, vo + 4, rr * ldo4, 0);
                }
        }
    }
}

template <int FORM>
__global__ __launch_bounds__(WideGeom<FORM>::NTH) __attribute__((amdgpu_waves_per_eu(2)))
void dft_gemm_wide_kernel(GemmArgs g) {
    using G = WideGeom<FORM>;
    __shared__ __attribute__((aligned(16))) WideSmem<FORM> sm;
    const int64_t nm = (g.F + G::BM - 1) / G::BM, nn = (g.N + G::BN - 1) / G::BN;
    const int64_t L = xcd_logical_block(blockIdx.x, (int64_t)gridDim.x);
    const int64_t gsz_full = WIDE_GROUP_M * nn;
    const int64_t grp = L / gsz_full, first_m = grp * WIDE_GROUP_M;
    const int64_t gsz = min((int64_t)WIDE_GROUP_M, nm - first_m);
    const int64_t within = L - grp * gsz_full;
    gemm_tile_wide<FORM>(g, (first_m + within % gsz) * G::BM, (within / gsz) * G::BN, sm);
}

template <int FORM, int WN>
__global__ __launch_bounds__(NT) void dft_gemm_kernel(GemmArgs g) {
    constexpr int BN = 64 * WN;
    __shared__ __attribute__((aligned(16))) GemmSmem<FORM, WN> sm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, BN, m0, n0);
    gemm_tile<FORM, WN>(g, m0, n0, sm);
}

// FP32 with the DFT operand assembled from a P-entry twiddle table in LDS
// (the table after the A tile buffer, 8 P bytes, loaded once per block)
// instead of read from the materialised N x K operand: every lane forms its
// B fragments from the table, one slab ahead of the products that use them.
constexpr size_t kTableTileBytes = (size_t)BM * RS;  // the table form stages only A tiles

template <int WN>
__global__ __launch_bounds__(NT) void dft_gemm_table_kernel(GemmArgs g, int P) {
    constexpr int BN = 64 * WN;
    extern __shared__ __attribute__((aligned(16))) uint8_t dyn[];
    // The tile storage holds the A tile only (the table form never touches
    // the B rows of GemmSmem); the table follows it.
    GemmSmem<FORM_FP32, WN>& sm = *reinterpret_cast<GemmSmem<FORM_FP32, WN>*>(dyn);
    float2* tws = reinterpret_cast<float2*>(dyn + kTableTileBytes);
    const float2* tw = reinterpret_cast<const float2*>(g.tw);
    for (int r = threadIdx.x; r < P; r += NT) tws[r] = tw[r];  // gemm_tile's first barrier publishes it
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, BN, m0, n0);
    gemm_tile<FORM_FP32, WN, false, true>(g, m0, n0, sm, tws);
}

// FP32 with compensated K accumulation: 128 x 128 tiles (the running sums
// and the block accumulators of 2 x 2 MFMA blocks per wave fit 2 waves per
// SIMD, so one wave's additions overlap the other's products).
template <int WN>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void dft_gemm_comp_kernel(GemmArgs g) {
    constexpr int BN = 64 * WN;
    __shared__ __attribute__((aligned(16))) GemmSmem<FORM_FP32, WN> sm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, BN, m0, n0);
    gemm_tile<FORM_FP32, WN, true>(g, m0, n0, sm);
}

// Held to 2 waves per SIMD: the fp16 hi + lo form with its second accumulator
// otherwise took 331 registers and one wave (2 waves with 4 spilled registers
// measured 10-20% faster); the other forms fit 2 waves anyway.
template <int FORM, int WN>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void dft_gemm_raw_kernel(GemmArgs g) {
    constexpr int BN = 64 * WN;
    __shared__ __attribute__((aligned(16))) RawSmem<FORM, WN> sm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, BN, m0, n0);
    gemm_tile_raw<FORM, WN>(g, m0, n0, sm);
}

template <int WN, int MT, bool EXACT>
__global__ __launch_bounds__(NT, 2) void dft_gemm_fused_kernel(FusedArgs fa) {
    constexpr int BN = 64 * WN;
    __shared__ __attribute__((aligned(16))) FusedSmem<WN, MT> sm;
    const int64_t nm = (fa.g.F + BM - 1) / BM, nn = (fa.g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(xcd_logical_block(blockIdx.x, (int64_t)gridDim.x), nm, nn, BN, m0, n0);
    gemm_tile_fused<WN, MT, EXACT>(fa, m0, n0, sm);
}

// Batched GEMM, one block per tile of any item: block b serves tile
// i = b / 8 of XCD x = b % 8's contiguous, cost-balanced range of tiles (see
// BatchTable); blocks past the end of their range return at once.  (A
// persistent loop over tiles keeps per-tile state live across iterations and
// halves the occupancy, so each block does one tile.)  RAW: A in operand form.
template <int FORM, bool RAW, int WN = kGemmBN / 64>
__global__ __launch_bounds__(NT) void dft_gemm_batch_kernel(const BatchTable* __restrict__ t) {
    constexpr int BN = 64 * WN;
    static_assert(kGemmBM == BM, "batch planner and kernel agree on the tile");
    using Smem = std::conditional_t<RAW, RawSmem<FORM, WN>, GemmSmem<FORM, WN>>;
    __shared__ __attribute__((aligned(16))) Smem sm;
    const int x = blockIdx.x & 7;
    const int64_t u = t->gemm_bounds[x] + (blockIdx.x >> 3);
    if (u >= t->gemm_bounds[x + 1]) return;
    const int it = batch_find(t->items, t->n_items, u, /*stage=*/1);
    const GemmArgs& g = t->items[it].gemm;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    int64_t m0, n0;
    grouped_tile(u - t->items[it].gemm_unit0, nm, nn, BN, m0, n0);
    if constexpr (RAW) gemm_tile_raw<FORM, WN>(g, m0, n0, sm);
    else gemm_tile<FORM, WN>(g, m0, n0, sm);
}

// Batched GEMM on the wide tiles: block b serves tile b / 8 of XCD b % 8's
// range, as dft_gemm_batch_kernel, each item's tiles mapped as the
// single-stream wide kernel maps them (same tiles, same bits).
template <int FORM>
__global__ __launch_bounds__(WideGeom<FORM>::NTH) __attribute__((amdgpu_waves_per_eu(2)))
void dft_gemm_batch_wide_kernel(const BatchTable* __restrict__ t) {
    using G = WideGeom<FORM>;
    __shared__ __attribute__((aligned(16))) WideSmem<FORM> sm;
    const int x = blockIdx.x & 7;
    const int64_t u = t->gemm_bounds[x] + (blockIdx.x >> 3);
    if (u >= t->gemm_bounds[x + 1]) return;
    const int it = batch_find(t->items, t->n_items, u, /*stage=*/1);
    const GemmArgs g = t->items[it].gemm;  // a private copy: read through the table, fields would be reloaded
    const int64_t nm = (g.F + G::BM - 1) / G::BM, nn = (g.N + G::BN - 1) / G::BN;
    const int64_t L = u - t->items[it].gemm_unit0;
    const int64_t gsz_full = WIDE_GROUP_M * nn;
    const int64_t grp = L / gsz_full, first_m = grp * WIDE_GROUP_M;
    const int64_t gsz = min((int64_t)WIDE_GROUP_M, nm - first_m);
    const int64_t within = L - grp * gsz_full;
    gemm_tile_wide<FORM>(g, (first_m + within % gsz) * G::BM, (within / gsz) * G::BN, sm);
}

// Columns per wave: 4 MFMA blocks (128 x 256 tiles) for FP32, whose long
// K tiles hide latency at 2 blocks per CU and whose tile count then fills the
// chip in whole rounds; 2 (128 x 128) for the others.
template <int FORM>
hipError_t launch_form(const GemmArgs& g, hipStream_t s) {
    constexpr int WN = FORM == FORM_FP32 ? 4 : 2, BN = 64 * WN;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((dft_gemm_kernel<FORM, WN>), dim3((unsigned)(nm * nn)), dim3(NT), 0, s, g);
    return hipGetLastError();
}

// Raw-operand GEMM: wide tiles when K is a whole number of their K tiles (a
// tile's byte range fits the 32-bit buffer offsets), else 128 x 128 tiles.
template <int FORM>
hipError_t launch_raw(const GemmArgs& g, hipStream_t s) {
    using G = WideGeom<FORM>;
    const int64_t eb = FT<FORM>::EB;
    if (g.K % G::BK == 0 && g.lda == g.K && (int64_t)G::BM * g.lda * eb < (1ll << 31) &&
        (int64_t)G::BN * g.K * eb < (1ll << 31)) {
        const int64_t nm = (g.F + G::BM - 1) / G::BM, nn = (g.N + G::BN - 1) / G::BN;
        hipLaunchKernelGGL((dft_gemm_wide_kernel<FORM>), dim3((unsigned)(nm * nn)), dim3(G::NTH), 0, s, g);
        return hipGetLastError();
    }
    constexpr int WN = 2, BN = 64 * WN;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    hipLaunchKernelGGL((dft_gemm_raw_kernel<FORM, WN>), dim3((unsigned)(nm * nn)), dim3(NT), 0, s, g);
    return hipGetLastError();
}

}  // namespace

bool gemm_raw_form(int form) { return form != FORM_FP32; }

bool gemm_batch_wide_tile(int form, int K, int& bm, int& bn) {
    auto geom = [&](auto tag) {
        using G = WideGeom<decltype(tag)::value>;
        bm = G::BM;
        bn = G::BN;
        return K % G::BK == 0 && (int64_t)G::BM * K * FT<decltype(tag)::value>::EB < (1ll << 31) &&
               (int64_t)G::BN * K * FT<decltype(tag)::value>::EB < (1ll << 31);
    };
    switch (form) {
        case FORM_BF16: return geom(std::integral_constant<int, FORM_BF16>{});
        case FORM_BF16X3: return geom(std::integral_constant<int, FORM_BF16X3>{});
        case FORM_FP16: return geom(std::integral_constant<int, FORM_FP16>{});
        case FORM_FP16X3: return geom(std::integral_constant<int, FORM_FP16X3>{});
        case FORM_FP8: return geom(std::integral_constant<int, FORM_FP8>{});
        case FORM_MXFP8: return geom(std::integral_constant<int, FORM_MXFP8>{});
        default: return false;
    }
}

hipError_t launch_gemm_batch(const BatchTable* t, int form, bool raw, int tile_n, int grid, hipStream_t s,
                             bool wide) {
    if (wide) {
        if (!raw) return hipErrorInvalidValue;
        auto go = [&](auto tag) {
            constexpr int F = decltype(tag)::value;
            hipLaunchKernelGGL((dft_gemm_batch_wide_kernel<F>), dim3(grid), dim3(WideGeom<F>::NTH), 0, s, t);
            return hipGetLastError();
        };
        switch (form) {
            case FORM_BF16: return go(std::integral_constant<int, FORM_BF16>{});
            case FORM_BF16X3: return go(std::integral_constant<int, FORM_BF16X3>{});
            case FORM_FP16: return go(std::integral_constant<int, FORM_FP16>{});
            case FORM_FP16X3: return go(std::integral_constant<int, FORM_FP16X3>{});
            case FORM_FP8: return go(std::integral_constant<int, FORM_FP8>{});
            case FORM_MXFP8: return go(std::integral_constant<int, FORM_MXFP8>{});
            default: return hipErrorInvalidValue;
        }
    }
    const dim3 gd(grid), bd(NT);
    if (tile_n == 2 * kGemmBN) {
        if (raw || form != FORM_FP32) return hipErrorInvalidValue;
        hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_FP32, false, 2 * kGemmBN / 64>), gd, bd, 0, s, t);
        return hipGetLastError();
    }
    if (tile_n != kGemmBN) return hipErrorInvalidValue;
    if (raw) {
        switch (form) {
            case FORM_BF16: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_BF16, true>), gd, bd, 0, s, t); break;
            case FORM_BF16X3: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_BF16X3, true>), gd, bd, 0, s, t); break;
            case FORM_MXFP8: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_MXFP8, true>), gd, bd, 0, s, t); break;
            case FORM_FP8: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_FP8, true>), gd, bd, 0, s, t); break;
            case FORM_FP16: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_FP16, true>), gd, bd, 0, s, t); break;
            case FORM_FP16X3: hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_FP16X3, true>), gd, bd, 0, s, t); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (form != FORM_FP32) return hipErrorInvalidValue;  // the other forms take A in operand form
    hipLaunchKernelGGL((dft_gemm_batch_kernel<FORM_FP32, false>), gd, bd, 0, s, t);
    return hipGetLastError();
}

bool fused_supported(const FirArgs& x, int form) {
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    return form == FORM_FP32 && x.M >= 1 && x.M <= 16 && x.W % 32 == 0 && x.plen % 4 == 0 && al16(x.chunk) &&
           (x.prefix == nullptr || al16(x.prefix));
}

hipError_t launch_dft_fused(const GemmArgs& g, const FirArgs& x, hipStream_t s) {
    if (g.F <= 0) return hipSuccess;
    if (!fused_supported(x, g.form)) return hipErrorInvalidValue;
    FusedArgs fa;
    fa.g = g;
    fa.x = x;
    constexpr int WN = 4, BN = 64 * WN;
    const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
    const dim3 grid((unsigned)(nm * nn)), block(NT);
    auto go = [&](auto mt_tag) {
        constexpr int MT = decltype(mt_tag)::value;
        if (x.M == MT) hipLaunchKernelGGL((dft_gemm_fused_kernel<WN, MT, true>), grid, block, 0, s, fa);
        else hipLaunchKernelGGL((dft_gemm_fused_kernel<WN, MT, false>), grid, block, 0, s, fa);
        return hipGetLastError();
    };
    if (x.M <= 4) return go(std::integral_constant<int, 4>{});
    if (x.M <= 8) return go(std::integral_constant<int, 8>{});
    return go(std::integral_constant<int, 16>{});
}

hipError_t launch_dft_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.F <= 0) return hipSuccess;
    if (g.Aq) {  // A in operand form
        switch (g.form) {
            case FORM_BF16: return launch_raw<FORM_BF16>(g, s);
            case FORM_BF16X3: return g.Aq1 ? launch_raw<FORM_BF16X3>(g, s) : hipErrorInvalidValue;
            case FORM_MXFP8: return (g.K % 128 == 0 && g.Aqs) ? launch_raw<FORM_MXFP8>(g, s) : hipErrorInvalidValue;
            case FORM_FP8: return g.fexp ? launch_raw<FORM_FP8>(g, s) : hipErrorInvalidValue;
            case FORM_FP16: return g.fexp ? launch_raw<FORM_FP16>(g, s) : hipErrorInvalidValue;
            case FORM_FP16X3: return (g.fexp && g.Aq1) ? launch_raw<FORM_FP16X3>(g, s) : hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    if (g.tw) {  // FP32, operand from the twiddle table
        if (g.form != FORM_FP32 || g.compensated) return hipErrorInvalidValue;
        constexpr int WN = 4, BN = 64 * WN;
        const int P = g.real_pack ? g.K : g.K / 2;
        const size_t lds = kTableTileBytes + 8 * (size_t)P;
        static bool attr = false;
        if (!attr) {  // up to P = 8192 (64 KiB of table)
            hipError_t e = hipFuncSetAttribute((const void*)dft_gemm_table_kernel<WN>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)(kTableTileBytes + 8 * 8192));
            if (e != hipSuccess) return e;
            attr = true;
        }
        const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
        hipLaunchKernelGGL((dft_gemm_table_kernel<WN>), dim3((unsigned)(nm * nn)), dim3(NT), lds, s, g, P);
        return hipGetLastError();
    }
    if (g.compensated) {
        if (g.form != FORM_FP32) return hipErrorInvalidValue;
        constexpr int WN = 2, BN = 64 * WN;
        const int64_t nm = (g.F + BM - 1) / BM, nn = (g.N + BN - 1) / BN;
        hipLaunchKernelGGL((dft_gemm_comp_kernel<WN>), dim3((unsigned)(nm * nn)), dim3(NT), 0, s, g);
        return hipGetLastError();
    }
    switch (g.form) {
        case FORM_FP32: return launch_form<FORM_FP32>(g, s);
        case FORM_BF16: return launch_form<FORM_BF16>(g, s);
        case FORM_BF16X3: return launch_form<FORM_BF16X3>(g, s);
        default: return hipErrorInvalidValue;  // the others take A in operand form
    }
}

}  // namespace tina
