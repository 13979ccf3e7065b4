// Polyphase FIR kernels and their launch templates, shared by the
// translation units that instantiate them (one per output mode, so that the
// many unrolled variants compile in parallel).  Not part of the ABI.
#pragma once
#include "internal.h"

#include <stdio.h>
#include <stdlib.h>

#include <type_traits>

namespace tina {

// Output modes of the FIR: FP32 rows, block-scaled FP8 codes and scales,
// bf16 pieces, per-frame partial maxima alone, per-frame scaled FP8 or fp16
// pieces.
enum FirOut : int {
    FIR_OUT_F32 = 0, FIR_OUT_MX = 2, FIR_OUT_BF16 = 3, FIR_OUT_BF16X2 = 4,
    FIR_OUT_AMAXONLY = 5, FIR_OUT_FP8F = 6, FIR_OUT_FP16F = 7, FIR_OUT_FP16FX2 = 8
};
// Operand-form output of the FIR (FirArgs::qmode): none (FP32 y), block-scaled
// FP8 codes and scales, bf16 (RNE), bf16 hi + lo (lo = RNE(y - hi)); with
// the frame's scale 2^-fexp[f] applied: FP8 E4M3 (saturated at 448), fp16,
// fp16 hi + lo (lo = RNE((x - hi) 2^11)); or only the partial maxima.
enum QMode : int {
    QM_NONE = 0, QM_MX = 1, QM_BF16 = 2, QM_BF16X2 = 3, QM_FP8F = 4, QM_FP16F = 5, QM_FP16FX2 = 6, QM_AMAXONLY = 7
};
constexpr int mode_qm(int mode) {
    return mode == FIR_OUT_MX ? QM_MX
         : mode == FIR_OUT_BF16 ? QM_BF16
         : mode == FIR_OUT_BF16X2 ? QM_BF16X2
         : mode == FIR_OUT_FP8F ? QM_FP8F
         : mode == FIR_OUT_FP16F ? QM_FP16F
         : mode == FIR_OUT_FP16FX2 ? QM_FP16FX2
         : mode == FIR_OUT_AMAXONLY ? QM_AMAXONLY : QM_NONE;
}
// Bytes per operand element and whether a second piece is written.
constexpr int qm_bytes(int qm) { return (qm == QM_MX || qm == QM_FP8F) ? 1 : 2; }
constexpr bool qm_two_pieces(int qm) { return qm == QM_BF16X2 || qm == QM_FP16FX2; }
constexpr bool qm_stores(int qm) { return qm != QM_NONE && qm != QM_AMAXONLY; }

// Launch-shape override for tuning sweeps: TINA_FIR_TUNE="vec,tf,nt"
// (vec 0 and tf 0 keep the defaults, vec 1/2/4 forces the vector width where
// the register ring allows it; nt 0 turns non-temporal access off, FP32
// output mode only).
struct FirTune { int vec = 0, tf = 0, nt = -1; };
FirTune fir_tune();
// Vector width (floats per thread) for these arguments.
int pick_vec(const FirArgs& a);

// Single-pass FIR for the per-frame scaled forms (fir_frame.hip): whole frame
// rows per block, so the frame's maximum, exponent and codes come from one
// read of the input.  fir_frame_vec: the floats per thread it would use, or 0
// when the arguments need the three-launch path (frames wider than 4096
// floats, more taps than its register ring holds, misaligned buffers).
int fir_frame_vec(const FirArgs& a);
hipError_t launch_fir_frame(const FirArgs& a, hipStream_t s);
// Batched form: the items flagged fir_single (fir_frame_batch_vec != 0),
// runs of each item's fir_tf frames as units of the table's frame stage.
// grid: a multiple of 8 (one range per XCD).
hipError_t launch_fir_frame_batch(const BatchTable* t, int qmode, int grid, hipStream_t s);

// Per-mode entry points (fir_out_*.hip).
hipError_t launch_fir_mode_f32(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_mx(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_bf16(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_bf16x2(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_amaxonly(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_fp8f(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_fp16f(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_mode_fp16fx2(FirArgs& a, int vec, hipStream_t s);
hipError_t launch_fir_batch_mode_f32(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_mx(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_bf16(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_bf16x2(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_amaxonly(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_fp8f(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_fp16f(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);
hipError_t launch_fir_batch_mode_fp16fx2(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s);

namespace {

typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <int VEC> struct VecT;
template <> struct VecT<1> { using T = float; };
template <> struct VecT<2> { using T = fvec2; };
template <> struct VecT<4> { using T = fvec4; };

template <int VEC>
__device__ inline float vget(const typename VecT<VEC>::T& v, int i) {
    if constexpr (VEC == 1) return v;
    else return v[i];
}
template <int VEC>
__device__ inline void vset(typename VecT<VEC>::T& v, int i, float x) {
    if constexpr (VEC == 1) v = x;
    else v[i] = x;
}

template <bool NTL, class V>
__device__ inline V ld(const V* p) {
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NTS, class V>
__device__ inline void st(V* p, const V& v) {
    if constexpr (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __attribute__((aligned(16))) float kZeros[4] = {0.f, 0.f, 0.f, 0.f};

// Input floats j0..j0+VEC-1 of frame g (g >= -(M-1)); ext = prefix ++ chunk,
// frame g starting at ext float (g + M - 1) * W.  The VEC floats never
// straddle the prefix/chunk boundary (plen is a multiple of VEC).  The source
// is chosen by a pointer select, not a branch, so that the loads of a block of
// frames can all be in flight together.
template <int VEC, bool NTL>
__device__ inline typename VecT<VEC>::T load_frame(const FirArgs& a, int64_t g, int j0) {
    using V = typename VecT<VEC>::T;
    const int64_t e = (g + a.M - 1) * (int64_t)a.W + j0;
    const float* hist = a.prefix ? a.prefix + e : kZeros;
    const float* p = e >= a.plen ? a.chunk + (e - a.plen) : hist;
    return ld<NTL>(reinterpret_cast<const V*>(p));
}

// Taps of the VEC columns j0.. for tap m: h[(M-1-m)*P + (j0+v)/cf].
template <int VEC>
__device__ inline typename VecT<VEC>::T load_taps(const FirArgs& a, int M, int m, int j0) {
    using V = typename VecT<VEC>::T;
    const float* base = a.taps + (int64_t)(M - 1 - m) * a.P;
    if (a.cf == 1) return *reinterpret_cast<const V*>(base + j0);
    V t;
    if constexpr (VEC == 4) {
        const fvec2 v = *reinterpret_cast<const fvec2*>(base + (j0 >> 1));
        t[0] = v[0]; t[1] = v[0]; t[2] = v[1]; t[3] = v[1];
    } else if constexpr (VEC == 2) {
        const float v = base[j0 >> 1];
        t[0] = v; t[1] = v;
    } else {
        t = base[j0 >> 1];
    }
    return t;
}

// One output frame from ring slot u (the newest frame) and the MT-1 before it.
template <int VEC, int MT, bool EXACT>
__device__ __forceinline__ typename VecT<VEC>::T fir_point(const typename VecT<VEC>::T (&tp)[MT],
                                                           const typename VecT<VEC>::T (&win)[MT], int u, int M) {
    typename VecT<VEC>::T acc = tp[0] * win[u];
#pragma unroll
    for (int m = 1; m < MT; ++m) {
        if (EXACT || m < M) acc = __builtin_elementwise_fma(tp[m], win[(u - m + MT) % MT], acc);
    }
    return acc;
}


// Smallest e in [-127, 127] with amax <= 448 * 2^e (0 for a zero or
// non-finite amax): the block scale of the block-scaled FP8 output.  With
// amax = m 2^E, m in [0.5, 1), and 448 = 0.875 * 2^9, that is E - 9 when
// m <= 0.875 and E - 8 otherwise (no division, no search).
__device__ inline int mx_exponent(float amax) {
    if (!(amax > 0.0f) || !isfinite(amax)) return 0;
    int E;
    const float m = frexpf(amax, &E);
    const int e = E - 9 + (m > 0.875f ? 1 : 0);
    return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// v from the lane a DPP pattern names (row-local; lanes the pattern leaves
// out read 0).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_read(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}
// Maximum over aligned groups of G lanes (1 to 32) of |x|, on the bit
// patterns: for non-negative floats the unsigned order is the float order,
// and 0 (what an absent lane reads) is the identity.  lane ^ 1, lane ^ 2
// (quad permutes), the mirror within 8 lanes and within a 16-lane row, then
// lane ^ 16 through the swizzle unit.
template <int G>
__device__ __forceinline__ float group_absmax(float x) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group of 1 to 32 lanes");
    uint32_t v = __builtin_bit_cast(uint32_t, fabsf(x));
    if constexpr (G >= 2) v = max(v, dpp_read<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    if constexpr (G >= 4) v = max(v, dpp_read<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    if constexpr (G >= 8) v = max(v, dpp_read<0x141>(v));  // row_half_mirror
    if constexpr (G >= 16) v = max(v, dpp_read<0x140>(v));  // row_mirror
    if constexpr (G >= 32)  // ds_swizzle bit mode: and 0x1f, or 0, xor 0x10
        v = max(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
    return __builtin_bit_cast(float, v);
}

// Where one block of frames goes.  PtrSink: plain pointers, row u of the
// block at base + u * stride.  BufSink: buffer resources whose base is the
// block's first row (wave-uniform); a lane's column offset stays in one VGPR
// and the row offset u * stride is an SGPR, so no per-row address registers
// are kept.  Out-of-range buffer stores are dropped by the hardware.
template <int VEC, bool NT>
struct PtrSink {
    using V = typename VecT<VEC>::T;
    float* yb;
    uint8_t* qb[2];   // operand pieces, at this lane's position
    uint8_t* sb;
    int64_t ldy, ldq, nsc;  // ldq in bytes
    __device__ __forceinline__ void y(int u, const V& v) const { st<NT>(reinterpret_cast<V*>(yb + u * ldy), v); }
    template <class T>
    __device__ __forceinline__ void q(int piece, int u, T w) const {
        st<NT>(reinterpret_cast<T*>(qb[piece] + u * ldq), w);
    }
    __device__ __forceinline__ void s8(int u, uint8_t b) const { sb[u * nsc] = b; }
};

constexpr int kBufWord3 = 0x00020000;  // raw (untyped) buffer access
constexpr int kNtAux = 2;              // non-temporal cache policy bit of buffer loads and stores

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
    const uint32_t n = bytes <= 0 ? 0u : (bytes >= 0xffffffffLL ? 0xffffffffu : (uint32_t)bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, kBufWord3);
}

template <int VEC, bool NT>
struct BufSink {
    using V = typename VecT<VEC>::T;
    __amdgpu_buffer_rsrc_t ry, rq[2], rs;
    uint32_t vy, vq, vs;  // lane offsets (bytes)
    int32_t ldy4, ldq, nsc;  // row strides (bytes)
    __device__ __forceinline__ void y(int u, const V& v) const {
        constexpr int aux = NT ? kNtAux : 0;
        if constexpr (VEC == 4)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t, v),
                                                   ry, vy, u * ldy4, aux);
        else if constexpr (VEC == 2)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v),
                                                  ry, vy, u * ldy4, aux);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), ry, vy, u * ldy4, aux);
    }
    template <class T>
    __device__ __forceinline__ void q(int piece, int u, T w) const {
        constexpr int aux = NT ? kNtAux : 0;
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, w),
                                                  rq[piece], vq, u * ldq, aux);
        else if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)w, rq[piece], vq, u * ldq, aux);
        else
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)w, rq[piece], vq, u * ldq, aux);
    }
    __device__ __forceinline__ void s8(int u, uint8_t b) const { __builtin_amdgcn_raw_buffer_store_b8(b, rs, vs, u * nsc, 0); }
};

// Load of the VEC floats at byte offset voff + row * stride4 of a buffer.
template <int VEC, bool NT>
__device__ __forceinline__ typename VecT<VEC>::T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, int32_t soff) {
    using V = typename VecT<VEC>::T;
    constexpr int aux = NT ? kNtAux : 0;
    if constexpr (VEC == 4) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, aux));
    else if constexpr (VEC == 2) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, aux));
    else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, aux));
}

// Per-frame partial maxima of |y| for the per-frame scaled forms: the gw
// lanes (a power of two up to 32) that hold one part of a frame row reduce
// their maxima with group_absmax, and the part's first lane stores it.
template <int VEC>
__device__ __forceinline__ void fir_amax(const FirArgs& a, const typename VecT<VEC>::T& acc, int64_t f, int col,
                                         int gw) {
    float mx = 0.0f;
#pragma unroll
    for (int v = 0; v < VEC; ++v) mx = fmaxf(mx, fabsf(vget<VEC>(acc, v)));
    switch (gw) {
        case 32: mx = group_absmax<32>(mx); break;
        case 16: mx = group_absmax<16>(mx); break;
        case 8: mx = group_absmax<8>(mx); break;
        case 4: mx = group_absmax<4>(mx); break;
        case 2: mx = group_absmax<2>(mx); break;
        default: break;
    }
    if ((col & (gw - 1)) == 0) a.amax[f * a.nparts + col / gw] = mx;
}

__device__ __forceinline__ uint32_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// Row u of a block in a per-frame scaled operand form, the frame's values
// times 2^-e: FP8 E4M3 codes saturated at 448 (packed as the block-scaled
// codes are), fp16, or fp16 hi + lo with lo = RNE((x - hi) 2^11).
template <int VEC, int QM, class Sink>
__device__ __forceinline__ void fir_store_frame(const typename VecT<VEC>::T& acc, int e, int col, const Sink& out,
                                                int u) {
    const float sc = ldexpf(1.0f, -e);
    if constexpr (QM == QM_FP8F) {
        float x[4];
#pragma unroll
        for (int v = 0; v < VEC; ++v) x[v] = fminf(fmaxf(vget<VEC>(acc, v) * sc, -448.0f), 448.0f);
        if constexpr (VEC == 4) {
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], w, true);
            out.q(0, u, (uint32_t)w);
        } else if constexpr (VEC == 2) {
            const uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false) & 0xffffu;
            const uint32_t w1 = dpp_read<0xF5>(w);
            if ((col & 1) == 0) out.q(0, u, w | (w1 << 16));
        } else {
            const uint32_t c = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[0], 0, false) & 0xffu;
            const uint32_t c1 = dpp_read<0x55>(c), c2 = dpp_read<0xAA>(c), c3 = dpp_read<0xFF>(c);
            if ((col & 3) == 0) out.q(0, u, c | (c1 << 8) | (c2 << 16) | (c3 << 24));
        }
    } else {
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const float x = vget<VEC>(acc, v) * sc;
            const _Float16 h = (_Float16)x;
            hi[v] = __builtin_bit_cast(uint16_t, h);
            lo[v] = __builtin_bit_cast(uint16_t, (_Float16)((x - (float)h) * 2048.0f));
        }
        auto put = [&](int piece, const uint32_t (&h)[4]) {
            if constexpr (VEC == 4) out.q(piece, u, (uint64_t)(h[0] | (h[1] << 16)) | ((uint64_t)(h[2] | (h[3] << 16)) << 32));
            else if constexpr (VEC == 2) out.q(piece, u, h[0] | (h[1] << 16));
            else out.q(piece, u, (uint16_t)h[0]);
        };
        put(0, hi);
        if constexpr (QM == QM_FP16FX2) put(1, lo);
    }
}

// Store row u of a block: FP32, the frame row's partial maxima only,
// or an operand form (QM):
//  - QM_MX, block-scaled FP8: the 32/VEC lanes that hold one 32-float block
//    of the frame share its maximum (group_absmax), every lane converts its
//    VEC floats scaled by 2^-e to E4M3 codes, 4 codes are gathered into one
//    lane for a 4-byte store, and the block's first lane writes the E8M0
//    scale byte e + 127;
//  - QM_BF16 / QM_BF16X2: bf16 hi = RNE(y) (and lo = RNE(y - hi)), VEC
//    values per lane.
// f = the frame of row u.
template <int VEC, int QM, class Sink>
__device__ __forceinline__ void fir_store(const FirArgs& a, const typename VecT<VEC>::T& acc, int64_t f, int col,
                                          int gw, const Sink& out, int u) {
    if constexpr (QM == QM_MX) {
        constexpr int GL = 32 / VEC;  // lanes per 32-float block
        float mx = 0.0f;
#pragma unroll
        for (int v = 0; v < VEC; ++v) mx = fmaxf(mx, fabsf(vget<VEC>(acc, v)));
        mx = group_absmax<GL>(mx);
        const int e = mx_exponent(mx);
        const float sc = ldexpf(1.0f, -e);
        float x[4];
#pragma unroll
        for (int v = 0; v < VEC; ++v) x[v] = fminf(fmaxf(vget<VEC>(acc, v) * sc, -448.0f), 448.0f);
        if constexpr (VEC == 4) {
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], w, true);
            out.q(0, u, (uint32_t)w);
        } else if constexpr (VEC == 2) {  // lane pairs: the even lane stores both
            const uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false) & 0xffffu;
            const uint32_t w1 = dpp_read<0xF5>(w);  // quad_perm [1, 1, 3, 3]
            if ((col & 1) == 0) out.q(0, u, w | (w1 << 16));
        } else {  // lane quads: the first lane stores all four
            const uint32_t c = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[0], 0, false) & 0xffu;
            const uint32_t c1 = dpp_read<0x55>(c), c2 = dpp_read<0xAA>(c), c3 = dpp_read<0xFF>(c);  // lanes 1, 2, 3
            if ((col & 3) == 0) out.q(0, u, c | (c1 << 8) | (c2 << 16) | (c3 << 24));
        }
        if ((col & (GL - 1)) == 0) out.s8(u, (uint8_t)(e + 127));
    } else if constexpr (QM == QM_FP8F || QM == QM_FP16F || QM == QM_FP16FX2) {
        fir_store_frame<VEC, QM>(acc, a.fexp[f], col, out, u);
    } else if constexpr (QM == QM_AMAXONLY) {
        fir_amax<VEC>(a, acc, f, col, gw);
    } else if constexpr (QM == QM_BF16 || QM == QM_BF16X2) {
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const float x = vget<VEC>(acc, v);
            hi[v] = bf16_bits(x);
            lo[v] = bf16_bits(x - __builtin_bit_cast(float, hi[v] << 16));
        }
        auto put = [&](int piece, const uint32_t (&h)[4]) {
            if constexpr (VEC == 4) out.q(piece, u, (uint64_t)(h[0] | (h[1] << 16)) | ((uint64_t)(h[2] | (h[3] << 16)) << 32));
            else if constexpr (VEC == 2) out.q(piece, u, h[0] | (h[1] << 16));
            else out.q(piece, u, (uint16_t)h[0]);
        };
        put(0, hi);
        if constexpr (QM == QM_BF16X2) put(1, lo);
    } else {
        out.y(u, acc);
    }
}

// MT: ring length (unroll); EXACT: M == MT (no per-tap predicate);
// NT: non-temporal input loads and output stores (streaming cache policy);
// QM: operand-form output (a.q, a.q1, a.qs; QMode) instead of FP32 (a.y).
// One 256-thread unit of work: logical block `blk` of the (column, run) grid.
template <int VEC, int MT, bool EXACT, bool NT, int QM>
__device__ __forceinline__ void fir_unit(const FirArgs& a, int TF, int64_t blk) {
    using V = typename VecT<VEC>::T;
    const int ct = a.W / VEC;                    // threads per frame row (power of two)
    const int64_t gid = blk * 256 + threadIdx.x;
    const int col = (int)(gid & (ct - 1));
    const int64_t run = gid / ct;
    const int64_t f_begin = run * TF;
    if (f_begin >= a.F) return;                  // whole groups of `ct` lanes leave together
    const int64_t f_end = min(a.F, f_begin + TF);
    const int j0 = col * VEC;
    const int M = EXACT ? MT : a.M;
    const int gw = ct < 32 ? ct : 32;            // lanes sharing one partial maximum of a frame row

    V tp[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) tp[m] = (EXACT || m < M) ? load_taps<VEC>(a, M, m, j0) : V(0.0f);

    // Ring of the last MT input frames of this thread's columns: frame g of a
    // block starting at fb sits in slot (g - fb) mod MT.  Frames fb - d
    // (d = 1..M-1) must be there when a block starts.
    V win[MT];
    auto load_ring = [&](int64_t fb) {
#pragma unroll
        for (int d = 1; d < MT; ++d)
            win[MT - d] = (EXACT || d < M) ? load_frame<VEC, false>(a, a.g0 + fb - d, j0) : V(0.0f);
    };
    // One output frame straight from its M input frames (no ring): used for
    // blocks that straddle the prefix/chunk boundary and for the tail, so that
    // these rare cases need no statically unrolled copy of the block.
    auto direct = [&](int64_t f) {
        V acc = V(0.0f);
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (EXACT || m < M) acc = __builtin_elementwise_fma(tp[m], load_frame<VEC, NT>(a, a.g0 + f - m, j0), acc);
        return acc;
    };

    // Full blocks of MT frames, loaded SB frames at a time: the SB loads of a
    // sub-block issue before its first FMA.  When a wave's lanes all work on
    // the same frames (ct >= 64) and the block's first frame row lies in the
    // chunk (so the whole block does), loads and stores go through buffer
    // resources based at the block (BufSink) and the ring carries the input
    // frames from block to block.  Other blocks go through pointers, choosing
    // between prefix and chunk per load.  The choice is uniform over a frame
    // row, so the lanes that share a block maximum of the block-scaled output
    // take the same path.
    constexpr int SB = (VEC == 4 ? 8 : 16) < MT ? (VEC == 4 ? 8 : 16) : MT;
    const int64_t nsc = a.W / 32;
    constexpr int QB = qm_bytes(QM);  // bytes per operand element
    auto sink_ptr = [&](int64_t fb) {
        PtrSink<VEC, NT> o;
        o.yb = QM ? nullptr : a.y + fb * a.ldy + j0;
        o.qb[0] = qm_stores(QM) ? a.q + (fb * a.ldq + j0) * QB : nullptr;
        o.qb[1] = qm_two_pieces(QM) ? a.q1 + (fb * a.ldq + j0) * QB : nullptr;
        o.sb = QM == QM_MX ? a.qs + fb * nsc + j0 / 32 : nullptr;
        o.ldy = a.ldy;
        o.ldq = a.ldq * QB;
        o.nsc = nsc;
        return o;
    };
    bool ring_ok = false;
    int64_t fb = f_begin;
    for (; fb + MT <= f_end; fb += MT) {
        const int64_t e_row = (a.g0 + fb + a.M - 1) * (int64_t)a.W - a.plen;  // block's first float in the chunk
        if (ct >= 64 && e_row >= 0) {
            if (!ring_ok) load_ring(fb);
            ring_ok = true;
            const int64_t fu = (int64_t)uniform64((uint64_t)fb);
            const int64_t eu = (a.g0 + fu + a.M - 1) * (int64_t)a.W - a.plen;
            const __amdgpu_buffer_rsrc_t rin = make_rsrc(a.chunk + eu, (a.nchunk - eu) * 4);
            const uint32_t vin = (uint32_t)j0 * 4u;
            const int32_t w4 = a.W * 4;
            BufSink<VEC, NT> o;
            if constexpr (QM == QM_AMAXONLY) {
                // partial maxima only: nothing is stored through the sink
            } else if constexpr (QM != QM_NONE) {
                o.rq[0] = make_rsrc(a.q + fu * a.ldq * QB, (a.F - fu) * a.ldq * QB);
                if constexpr (qm_two_pieces(QM)) o.rq[1] = make_rsrc(a.q1 + fu * a.ldq * QB, (a.F - fu) * a.ldq * QB);
                if constexpr (QM == QM_MX) o.rs = make_rsrc(a.qs + fu * nsc, (a.F - fu) * nsc);
                o.vq = (uint32_t)(j0 * QB);
                o.vs = (uint32_t)(j0 / 32);
                o.ldq = (int32_t)(a.ldq * QB);
                o.nsc = (int32_t)nsc;
            } else {
                o.ry = make_rsrc(a.y + fu * a.ldy, (a.F - fu) * a.ldy * 4);
                o.vy = (uint32_t)j0 * 4u;
                o.ldy4 = (int32_t)(a.ldy * 4);
            }
#pragma unroll
            for (int sb = 0; sb < MT; sb += SB) {
                V in[SB];
#pragma unroll
                for (int i = 0; i < SB; ++i) in[i] = buf_load<VEC, NT>(rin, vin, (sb + i) * w4);
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    const int u = sb + i;
                    win[u] = in[i];
                    const V acc = fir_point<VEC, MT, EXACT>(tp, win, u, M);
                    fir_store<VEC, QM>(a, acc, fb + u, col, gw, o, u);
                }
            }
        } else {
            ring_ok = false;
            const PtrSink<VEC, NT> o = sink_ptr(fb);
            for (int u = 0; u < MT; ++u) fir_store<VEC, QM>(a, direct(fb + u), fb + u, col, gw, o, u);
        }
    }
    // Tail block.
    const PtrSink<VEC, NT> o = sink_ptr(fb);
    for (int u = 0; u < MT && fb + u < f_end; ++u) fir_store<VEC, QM>(a, direct(fb + u), fb + u, col, gw, o, u);
}

template <int VEC, int MT, bool EXACT, bool NT, int QM>
__global__ __launch_bounds__(256) void fir_kernel(FirArgs a, int TF) {
    fir_unit<VEC, MT, EXACT, NT, QM>(a, TF, xcd_logical_block(blockIdx.x, gridDim.x));
}

// One unit with the ring and tap loop unrolled for the item's own tap count
// M0 (searched from M0 up to MT): the run-time predicated form of fir_unit
// needs 2.5x the registers and runs 2-4x slower.  Same FMA order, same bits.
template <int M0, int MT, int QM>
__device__ __forceinline__ void fir_unit_own_m(const FirArgs& a, int TF, int64_t blk) {
    if constexpr (M0 <= MT) {
        if (a.M == M0) fir_unit<1, M0, true, true, QM>(a, TF, blk);
        else fir_unit_own_m<M0 + 1, MT, QM>(a, TF, blk);
    }
}

// Persistent batched FIR: each block walks its XCD's contiguous, cost-balanced
// range of units (see BatchTable); a unit is one 256-thread block of one item.
// Batches whose largest tap count is at most 16 with mixed tap counts run
// every item's units with the ring unrolled for its own M.
template <int MT, bool EXACT, int QM>
__global__ __launch_bounds__(256) void fir_batch_kernel(const BatchTable* __restrict__ t) {
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const int64_t end = t->fir_bounds[x + 1];
    for (int64_t u = t->fir_bounds[x] + i; u < end; u += nbx) {
        const int it = batch_find(t->items, t->n_items, u, /*stage=*/0);
        const BatchItem& b = t->items[it];
        // A private copy of the item's arguments: read through the table, every
        // field would be reloaded after each output store (they might alias).
        const FirArgs fa = b.fir;
        if constexpr (!EXACT && MT <= 16) fir_unit_own_m<1, MT, QM>(fa, b.fir_tf, u - b.fir_unit0);
        else fir_unit<1, MT, EXACT, true, QM>(fa, b.fir_tf, u - b.fir_unit0);
    }
}

template <int VEC, int MT, bool EXACT, int MODE>
hipError_t launch_one(FirArgs& a, hipStream_t s) {
    constexpr int QM = mode_qm(MODE);
    const int ct = a.W / VEC;
    // Frames per thread (a multiple of MT).  Measured on MI355X: 2*MT (at
    // least 16) keeps the halo re-reads in L2 while leaving enough waves to
    // hide HBM latency.
    // A multiple of MT, so that every run is whole ring blocks (tap counts
    // that are not powers of two included).
    int TF = 2 * MT < 16 ? ((16 + MT - 1) / MT) * MT : 2 * MT;
    const FirTune tune = fir_tune();
    if (tune.tf > 0) TF = ((tune.tf + MT - 1) / MT) * MT;
    const int64_t runs = (a.F + TF - 1) / TF;
    const int64_t threads = runs * ct;
    const int64_t blocks = (threads + 255) / 256;
    // Non-temporal loads and stores (streaming data, measured faster); the
    // FP32 mode can turn them off for tuning sweeps.
    if constexpr (MODE == FIR_OUT_F32) {
        if (tune.nt == 0) {
            hipLaunchKernelGGL((fir_kernel<VEC, MT, EXACT, false, QM_NONE>), dim3((unsigned)blocks), dim3(256), 0, s,
                               a, TF);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((fir_kernel<VEC, MT, EXACT, true, QM>), dim3((unsigned)blocks), dim3(256), 0, s, a, TF);
    return hipGetLastError();
}

template <int VEC, int MT, int MODE>
hipError_t launch_mt(FirArgs& a, hipStream_t s) {
    if (a.M == MT) return launch_one<VEC, MT, true, MODE>(a, s);
    // 9..15 taps at 1 or 2 floats per thread: the ring unrolled for the
    // exact count (the run-time predicated form takes 2.5x the registers);
    // at 4 floats per thread the 8-frame load groups need MT % 8 == 0.
    if constexpr (MT == 16 && VEC <= 2) {
        switch (a.M) {
            case 9: return launch_one<VEC, 9, true, MODE>(a, s);
            case 10: return launch_one<VEC, 10, true, MODE>(a, s);
            case 11: return launch_one<VEC, 11, true, MODE>(a, s);
            case 12: return launch_one<VEC, 12, true, MODE>(a, s);
            case 13: return launch_one<VEC, 13, true, MODE>(a, s);
            case 14: return launch_one<VEC, 14, true, MODE>(a, s);
            case 15: return launch_one<VEC, 15, true, MODE>(a, s);
            default: break;
        }
    }
    if constexpr (MT == 8) {  // 5..7 taps (8-frame load groups hold the whole ring at any width)
        switch (a.M) {
            case 5: return launch_one<VEC, 5, true, MODE>(a, s);
            case 6: return launch_one<VEC, 6, true, MODE>(a, s);
            case 7: return launch_one<VEC, 7, true, MODE>(a, s);
            default: break;
        }
    }
    if constexpr (MT == 4) {
        if (a.M == 3) return launch_one<VEC, 3, true, MODE>(a, s);
    }
    return launch_one<VEC, MT, false, MODE>(a, s);
}

template <int VEC, int MODE>
hipError_t launch_vec(FirArgs& a, hipStream_t s) {
    if (a.M <= 1) return launch_mt<VEC, 1, MODE>(a, s);
    if (a.M <= 2) return launch_mt<VEC, 2, MODE>(a, s);
    if (a.M <= 4) return launch_mt<VEC, 4, MODE>(a, s);
    if (a.M <= 8) return launch_mt<VEC, 8, MODE>(a, s);
    if (a.M <= 16) return launch_mt<VEC, 16, MODE>(a, s);
    if constexpr (VEC <= 2) {
        if (a.M <= 32) return launch_mt<VEC, 32, MODE>(a, s);
    }
    if constexpr (VEC == 1) {
        if (a.M <= 64) return launch_mt<VEC, 64, MODE>(a, s);
    }
    return hipErrorInvalidValue;
}

template <int MODE>
hipError_t launch_mode(FirArgs& a, int vec, hipStream_t s) {
    switch (vec) {
        case 4: return launch_vec<4, MODE>(a, s);
        case 2: return launch_vec<2, MODE>(a, s);
        default: return launch_vec<1, MODE>(a, s);
    }
}

template <int MODE>
hipError_t launch_batch_mode(const BatchTable* t, int max_m, bool all_exact, int grid, hipStream_t s) {
    constexpr int QM = mode_qm(MODE);
    auto go = [&](auto mt_tag) -> hipError_t {
        constexpr int MT = decltype(mt_tag)::value;
        if (all_exact) hipLaunchKernelGGL((fir_batch_kernel<MT, true, QM>), dim3(grid), dim3(256), 0, s, t);
        else hipLaunchKernelGGL((fir_batch_kernel<MT, false, QM>), dim3(grid), dim3(256), 0, s, t);
        return hipGetLastError();
    };
    if (max_m <= 1) return go(std::integral_constant<int, 1>{});
    if (max_m <= 2) return go(std::integral_constant<int, 2>{});
    if (max_m <= 4) return go(std::integral_constant<int, 4>{});
    if (max_m <= 8) return go(std::integral_constant<int, 8>{});
    if (max_m <= 16) return go(std::integral_constant<int, 16>{});
    if (max_m <= 32) return go(std::integral_constant<int, 32>{});
    if (max_m <= 64) return go(std::integral_constant<int, 64>{});
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace tina
