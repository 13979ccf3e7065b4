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

namespace tina {
namespace {

template <int VEC> struct VecT;
template <> struct VecT<1> { using T = float; };
template <> struct VecT<2> { using T = float2; };
template <> struct VecT<4> { using T = float4; };

template <int VEC>
__device__ inline float vget(const typename VecT<VEC>::T& v, int i) {
    if constexpr (VEC == 1) return v;
    else if constexpr (VEC == 2) return i == 0 ? v.x : v.y;
    else return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
template <int VEC>
__device__ inline void vset(typename VecT<VEC>::T& v, int i, float x) {
    if constexpr (VEC == 1) v = x;
    else if constexpr (VEC == 2) { if (i == 0) v.x = x; else v.y = x; }
    else { if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x; }
}

// Input floats j0..j0+VEC-1 of frame g (g >= -(M-1)); ext = prefix ++ chunk,
// frame g starting at ext float (g + M - 1) * W.  The VEC floats never
// straddle the prefix/chunk boundary (plen is a multiple of VEC).
template <int VEC>
__device__ inline typename VecT<VEC>::T load_frame(const FirArgs& a, int64_t g, int j0) {
    using V = typename VecT<VEC>::T;
    const int64_t e = (g + a.M - 1) * (int64_t)a.W + j0;
    if (e >= a.plen) return *reinterpret_cast<const V*>(a.chunk + (e - a.plen));
    if (a.prefix) return *reinterpret_cast<const V*>(a.prefix + e);
    V z;
#pragma unroll
    for (int i = 0; i < VEC; ++i) vset<VEC>(z, i, 0.0f);
    return z;
}

// MT: ring length (unroll); EXACT: M == MT (no per-tap predicate).
template <int VEC, int MT, bool EXACT, bool AMAX>
__global__ __launch_bounds__(256) void fir_kernel(FirArgs a, int TF) {
    using V = typename VecT<VEC>::T;
    const int ct = a.W / VEC;                    // threads per frame row (power of two)
    const int64_t nb = gridDim.x;
    const int64_t blk = xcd_logical_block(blockIdx.x, nb);
    const int64_t gid = blk * blockDim.x + threadIdx.x;
    const int col = (int)(gid & (ct - 1));
    const int64_t run = gid / ct;
    const int64_t f_begin = run * TF;
    if (f_begin >= a.F) return;                  // whole groups of `ct` lanes leave together
    const int64_t f_end = min(a.F, f_begin + TF);
    const int j0 = col * VEC;
    const int M = EXACT ? MT : a.M;

    float tp[MT][VEC];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            tp[m][v] = (EXACT || m < M) ? a.taps[(int64_t)(M - 1 - m) * a.P + (j0 + v) / a.cf] : 0.0f;

    V win[MT];
    // Frames f_begin - d (d = 1..M-1) go to ring slot MT - d (f_begin is a multiple of MT).
#pragma unroll
    for (int d = 1; d < MT; ++d) {
        if (EXACT || d < M) win[MT - d] = load_frame<VEC>(a, a.g0 + f_begin - d, j0);
    }

    const int gw = ct < 64 ? ct : 64;            // lanes sharing one frame row in a wave
    for (int64_t fb = f_begin; fb < f_end; fb += MT) {
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int64_t f = fb + u;
            if (f < f_end) {
                win[u] = load_frame<VEC>(a, a.g0 + f, j0);
                V acc;
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    float s = 0.0f;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (EXACT || m < M) s = fmaf(tp[m][v], vget<VEC>(win[(u - m + MT) % MT], v), s);
                    }
                    vset<VEC>(acc, v, s);
                }
                *reinterpret_cast<V*>(a.y + f * a.ldy + j0) = acc;
                if constexpr (AMAX) {
                    float mx = 0.0f;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) mx = fmaxf(mx, fabsf(vget<VEC>(acc, v)));
                    for (int off = gw >> 1; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, gw));
                    if ((col & (gw - 1)) == 0) a.amax[f * a.nparts + col / gw] = mx;
                }
            }
        }
    }
}

template <int VEC, int MT, bool EXACT, bool AMAX>
hipError_t launch_one(FirArgs& a, hipStream_t s) {
    const int ct = a.W / VEC;
    // Frames per thread: a multiple of MT; long enough that the (M-1)-frame
    // halo is a small fraction, short enough to leave many waves in flight.
    int TF = MT;
    while (TF < 32) TF += MT;
    int64_t runs = (a.F + TF - 1) / TF;
    while (TF < 128 && runs * ct > 256 * 1024) {
        TF += MT;
        runs = (a.F + TF - 1) / TF;
    }
    const int64_t threads = runs * ct;
    const int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL((fir_kernel<VEC, MT, EXACT, AMAX>), dim3((unsigned)blocks), dim3(256), 0, s, a, TF);
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
    int vec = a.M <= 16 ? 4 : (a.M <= 32 ? 2 : 1);
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

}  // namespace

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

hipError_t launch_gather_ext(const float* prefix, int64_t plen, const float* chunk, int64_t nchunk,
                             float* dst, int64_t start, int64_t count, hipStream_t s) {
    (void)nchunk;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_ext_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, prefix, plen,
                       chunk, dst, start, count);
    return hipGetLastError();
}

}  // namespace tina
