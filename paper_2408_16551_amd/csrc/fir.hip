// Polyphase FIR (Sec. 5.2, Eq. (20)): y_p(f) = sum_{m<M} h[(M-1-m)P + p] x_p(f - m),
// with branch p of frame f at stream sample f*P + p.  A complex sample is two
// floats filtered independently by the same real taps, so the kernel works on
// float columns j of a frame (W = P*cf floats) with branch p = j / cf.
//
// HBM-bound streaming kernel: each thread owns VEC adjacent float columns and
// walks TF consecutive frames, keeping the last MT input frames of its
// columns in registers (a ring indexed statically by unrolling the frame loop
// by MT), so every input float is read once from HBM plus a (M-1)/TF halo,
// and every output float is written once.  Lanes of a wave cover adjacent
// columns, so each load and store of a frame row is contiguous across the wave.
#include "internal.h"

#include <stdio.h>
#include <stdlib.h>

#include <type_traits>

namespace tina {
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

template <int VEC, bool AMAX>
__device__ __forceinline__ void fir_amax(const FirArgs& a, const typename VecT<VEC>::T& acc, int64_t f, int col,
                                         int gw) {
    if constexpr (AMAX) {
        float mx = 0.0f;
#pragma unroll
        for (int v = 0; v < VEC; ++v) mx = fmaxf(mx, fabsf(vget<VEC>(acc, v)));
        for (int off = gw >> 1; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, gw));
        if ((col & (gw - 1)) == 0) a.amax[f * a.nparts + col / gw] = mx;
    }
}

// MT: ring length (unroll); EXACT: M == MT (no per-tap predicate);
// NT: non-temporal input loads and output stores (streaming cache policy).
// One 256-thread unit of work: logical block `blk` of the (column, run) grid.
template <int VEC, int MT, bool EXACT, bool AMAX, bool NT>
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
    const int gw = ct < 64 ? ct : 64;            // lanes sharing one frame row in a wave

    V tp[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) tp[m] = (EXACT || m < M) ? load_taps<VEC>(a, M, m, j0) : V(0.0f);

    V win[MT];
    // Frames f_begin - d (d = 1..M-1) go to ring slot MT - d (f_begin is a multiple of MT).
#pragma unroll
    for (int d = 1; d < MT; ++d) {
        win[MT - d] = (EXACT || d < M) ? load_frame<VEC, false>(a, a.g0 + f_begin - d, j0) : V(0.0f);
    }
    win[0] = V(0.0f);

    // Full blocks of MT frames, loaded SB frames at a time: the SB loads of a
    // sub-block issue before its first FMA.
    constexpr int SB = (VEC == 4 ? 8 : 16) < MT ? (VEC == 4 ? 8 : 16) : MT;
    int64_t fb = f_begin;
    for (; fb + MT <= f_end; fb += MT) {
#pragma unroll
        for (int sb = 0; sb < MT; sb += SB) {
            V in[SB];
#pragma unroll
            for (int i = 0; i < SB; ++i) in[i] = load_frame<VEC, NT>(a, a.g0 + fb + sb + i, j0);
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int u = sb + i;
                win[u] = in[i];
                const V acc = fir_point<VEC, MT, EXACT>(tp, win, u, M);
                st<NT>(reinterpret_cast<V*>(a.y + (fb + u) * a.ldy + j0), acc);
                fir_amax<VEC, AMAX>(a, acc, fb + u, col, gw);
            }
        }
    }
    // Tail block.
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        if (fb + u < f_end) {
            win[u] = load_frame<VEC, NT>(a, a.g0 + fb + u, j0);
            const V acc = fir_point<VEC, MT, EXACT>(tp, win, u, M);
            st<NT>(reinterpret_cast<V*>(a.y + (fb + u) * a.ldy + j0), acc);
            fir_amax<VEC, AMAX>(a, acc, fb + u, col, gw);
        }
    }
}

template <int VEC, int MT, bool EXACT, bool AMAX, bool NT>
__global__ __launch_bounds__(256) void fir_kernel(FirArgs a, int TF) {
    fir_unit<VEC, MT, EXACT, AMAX, NT>(a, TF, xcd_logical_block(blockIdx.x, gridDim.x));
}

// Persistent batched FIR: each block walks its XCD's contiguous, cost-balanced
// range of units (see BatchTable); a unit is one 256-thread block of one item.
template <int MT, bool EXACT, bool AMAX>
__global__ __launch_bounds__(256) void fir_batch_kernel(const BatchTable* __restrict__ t) {
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const int64_t end = t->fir_bounds[x + 1];
    for (int64_t u = t->fir_bounds[x] + i; u < end; u += nbx) {
        const int it = batch_find(t->items, t->n_items, u, /*stage=*/0);
        const BatchItem& b = t->items[it];
        fir_unit<1, MT, EXACT, AMAX, true>(b.fir, b.fir_tf, u - b.fir_unit0);
    }
}

// Launch-shape override for tuning sweeps: TINA_FIR_TUNE="vec,tf,nt"
// (vec 0 and tf 0 keep the defaults; nt 0 turns non-temporal access off).
struct FirTune { int vec = 0, tf = 0, nt = -1; };
FirTune fir_tune() {
    static FirTune t = [] {
        FirTune r;
        if (const char* e = getenv("TINA_FIR_TUNE")) {
            int v = 0, f = 0, n = -1;
            if (sscanf(e, "%d,%d,%d", &v, &f, &n) >= 1) { r.vec = v; r.tf = f; r.nt = n; }
        }
        return r;
    }();
    return t;
}

template <int VEC, int MT, bool EXACT, bool AMAX>
hipError_t launch_one(FirArgs& a, hipStream_t s) {
    const int ct = a.W / VEC;
    // Frames per thread (a multiple of MT).  Measured on MI355X: 2*MT (at
    // least 16) keeps the halo re-reads in L2 while leaving enough waves to
    // hide HBM latency.
    int TF = 2 * MT < 16 ? 16 : 2 * MT;
    const FirTune tune = fir_tune();
    if (tune.tf > 0) TF = ((tune.tf + MT - 1) / MT) * MT;
    const int64_t runs = (a.F + TF - 1) / TF;
    const int64_t threads = runs * ct;
    const int64_t blocks = (threads + 255) / 256;
    // Non-temporal loads and stores by default (streaming data, measured faster).
    if (tune.nt != 0)
        hipLaunchKernelGGL((fir_kernel<VEC, MT, EXACT, AMAX, true>), dim3((unsigned)blocks), dim3(256), 0, s, a, TF);
    else
        hipLaunchKernelGGL((fir_kernel<VEC, MT, EXACT, AMAX, false>), dim3((unsigned)blocks), dim3(256), 0, s, a, TF);
    return hipGetLastError();
}

template <int VEC, int MT>
hipError_t launch_mt(FirArgs& a, hipStream_t s) {
    const bool exact = (a.M == MT);
    if (a.amax) return exact ? launch_one<VEC, MT, true, true>(a, s) : launch_one<VEC, MT, false, true>(a, s);
    return exact ? launch_one<VEC, MT, true, false>(a, s) : launch_one<VEC, MT, false, false>(a, s);
}

template <int VEC>
hipError_t launch_vec(FirArgs& a, hipStream_t s) {
    if (a.M <= 1) return launch_mt<VEC, 1>(a, s);
    if (a.M <= 2) return launch_mt<VEC, 2>(a, s);
    if (a.M <= 4) return launch_mt<VEC, 4>(a, s);
    if (a.M <= 8) return launch_mt<VEC, 8>(a, s);
    if (a.M <= 16) return launch_mt<VEC, 16>(a, s);
    if constexpr (VEC <= 2) {
        if (a.M <= 32) return launch_mt<VEC, 32>(a, s);
    }
    if constexpr (VEC == 1) {
        if (a.M <= 64) return launch_mt<VEC, 64>(a, s);
    }
    return hipErrorInvalidValue;
}

int pick_vec(const FirArgs& a) {
    auto aligned = [](const void* p, int bytes) { return ((uintptr_t)p % bytes) == 0; };
    // Vector width by register budget (taps, ring and prefetch each take
    // MT*VEC registers): 4 floats for up to 8 taps, else 1 (measured best).
    int vec = a.M <= 8 ? 4 : 1;
    const FirTune tune = fir_tune();
    if (tune.vec == 1 || tune.vec == 2 || tune.vec == 4) vec = tune.vec < vec ? tune.vec : vec;
    while (vec > 1 && !(a.plen % vec == 0 && aligned(a.chunk, 4 * vec) && aligned(a.y, 4 * vec) &&
                        (a.prefix == nullptr || aligned(a.prefix, 4 * vec)) && a.ldy % vec == 0))
        vec >>= 1;
    return vec;
}

__global__ void gather_ext_kernel(const float* prefix, int64_t plen, const float* chunk, float* dst,
                                  int64_t start, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t e = start + i;
    dst[i] = e < plen ? (prefix ? prefix[e] : 0.0f) : chunk[e - plen];
}

// Batched state update: for every item with a state, dst[i] = ext[start + i].
__global__ void gather_batch_kernel(const BatchTable* __restrict__ t) {
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const int64_t end = t->st_bounds[x + 1];
    for (int64_t u = t->st_bounds[x] + i; u < end; u += nbx) {
        const int it = batch_find(t->items, t->n_items, u, /*stage=*/2);
        const BatchItem& b = t->items[it];
        const int64_t k = (u - b.st_unit0) * 256 + threadIdx.x;
        if (k < b.st_count) {
            const int64_t e = b.st_start + k;
            b.st_dst[k] = e < b.fir.plen ? (b.fir.prefix ? b.fir.prefix[e] : 0.0f) : b.fir.chunk[e - b.fir.plen];
        }
    }
}

}  // namespace

hipError_t launch_gather_batch(const BatchTable* t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(gather_batch_kernel, dim3(grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

int fir_amax_parts(const FirArgs& a) {
    const int ct = a.W / pick_vec(a);
    const int gw = ct < 64 ? ct : 64;
    return ct / gw;
}

hipError_t launch_fir(FirArgs& a, hipStream_t s) {
    if (a.F <= 0) return hipSuccess;
    const int vec = pick_vec(a);
    {
        const int ct = a.W / vec;
        const int gw = ct < 64 ? ct : 64;
        a.nparts = ct / gw;
    }
    switch (vec) {
        case 4: return launch_vec<4>(a, s);
        case 2: return launch_vec<2>(a, s);
        default: return launch_vec<1>(a, s);
    }
}

hipError_t launch_fir_batch(const BatchTable* t, int max_m, bool all_exact, bool amax, int grid, hipStream_t s) {
    auto go = [&](auto mt_tag) -> hipError_t {
        constexpr int MT = decltype(mt_tag)::value;
        if (amax) {
            if (all_exact) hipLaunchKernelGGL((fir_batch_kernel<MT, true, true>), dim3(grid), dim3(256), 0, s, t);
            else hipLaunchKernelGGL((fir_batch_kernel<MT, false, true>), dim3(grid), dim3(256), 0, s, t);
        } else {
            if (all_exact) hipLaunchKernelGGL((fir_batch_kernel<MT, true, false>), dim3(grid), dim3(256), 0, s, t);
            else hipLaunchKernelGGL((fir_batch_kernel<MT, false, false>), dim3(grid), dim3(256), 0, s, t);
        }
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

hipError_t launch_gather_ext(const float* prefix, int64_t plen, const float* chunk, int64_t nchunk,
                             float* dst, int64_t start, int64_t count, hipStream_t s) {
    (void)nchunk;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_ext_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, prefix, plen,
                       chunk, dst, start, count);
    return hipGetLastError();
}

}  // namespace tina
