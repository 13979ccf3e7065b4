// Single-pass polyphase FIR for the per-frame scaled operand forms (FP8 E4M3,
// fp16, fp16 hi + lo), for frames of at most 1024 threads' columns.  A
// per-frame scale needs the whole frame's largest |y| before its first code,
// so here one block holds whole frame rows: W / VEC threads, each with VEC
// adjacent columns, walk a run of frames through the same register ring as
// the streaming FIR.  For every ring block of MT frames the block computes
// the outputs and each frame's maximum over the lanes of each wave; then one
// lane per frame reduces the waves' maxima (through LDS) and derives the
// frame's exponent, and every thread writes its scaled codes.
// The input is read once, instead of once for the maxima and again for the
// codes.  Outputs, maxima, exponents and codes are those of the three-launch
// path (same FMA order; the maximum of a set of floats does not depend on the
// order it is taken in), so both paths give the same bits.
#include "fir_kernels.h"

namespace tina {
namespace {

constexpr int kFrameMaxThreads = 1024;

// One block's run of frames [run * TF, ...) of a, with blockDim.x = W / VEC.
// smax: [wave][frame of the ring block] (stride MT), sexp: the ring block's
// frame exponents.  Every thread of the block takes the same barriers.
template <int VEC, int MT, bool EXACT, int QM>
__device__ __forceinline__ void frame_unit(const FirArgs& a, int TF, int64_t run, float* smax, int* sexp) {
    using V = typename VecT<VEC>::T;
    const int col = threadIdx.x, j0 = col * VEC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int64_t f_begin = run * TF;
    const int64_t f_end = min(a.F, f_begin + TF);
    const int M = EXACT ? MT : a.M;
    const float limit = QM == QM_FP8F ? 448.0f : 32768.0f;
    constexpr int QB = qm_bytes(QM);

    V tp[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) tp[m] = (EXACT || m < M) ? load_taps<VEC>(a, M, m, j0) : V(0.0f);
    // Ring slot u holds frame fb + u of the block starting at fb; the frames
    // before the run's first block come first.
    V win[MT];
#pragma unroll
    for (int d = 1; d < MT; ++d)
        win[MT - d] = (EXACT || d < M) ? load_frame<VEC, false>(a, a.g0 + f_begin - d, j0) : V(0.0f);

    for (int64_t fb = f_begin; fb < f_end; fb += MT) {  // uniform over the block
        const int nu = f_end - fb < MT ? (int)(f_end - fb) : MT;
        // Frames enter the ring SB at a time: their loads issue together, and
        // slot u is overwritten only once the outputs before it are done with
        // the frame it held.  Past the last frame the slots take zeros (the
        // run ends with this block).
        constexpr int SB = (VEC == 4 ? 8 : 16) < MT ? (VEC == 4 ? 8 : 16) : MT;
        V ys[MT];
#pragma unroll
        for (int sb = 0; sb < MT; sb += SB) {
            V in[SB];
#pragma unroll
            for (int i = 0; i < SB; ++i)
                in[i] = sb + i < nu ? load_frame<VEC, true>(a, a.g0 + fb + sb + i, j0) : V(0.0f);
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int u = sb + i;
                win[u] = in[i];
                ys[u] = fir_point<VEC, MT, EXACT>(tp, win, u, M);
                // The frame's maximum of |y| as the three-launch path takes
                // it: fmaxf over the lane's values (NaN dropped), then the
                // bit-pattern maximum over lanes and waves.
                float mx = 0.0f;
#pragma unroll
                for (int v = 0; v < VEC; ++v) mx = fmaxf(mx, fabsf(vget<VEC>(ys[u], v)));
                mx = group_absmax<32>(mx);
                mx = fmaxf(mx, __shfl_xor(mx, 32));
                if (lane == 0) smax[wave * MT + u] = mx;
            }
        }
        __syncthreads();  // smax complete
        // Lane u of the first wave reduces frame u over the waves and derives
        // its exponent once for the block.
        if (threadIdx.x < MT && (int)threadIdx.x < nu) {
            float fm = 0.0f;
            for (int w = 0; w < nwaves; ++w) fm = fmaxf(fm, smax[w * MT + threadIdx.x]);
            const int e = frame_exponent(fm, limit);
            sexp[threadIdx.x] = e;
            a.fexp[fb + threadIdx.x] = e;
        }
        __syncthreads();  // sexp complete; smax free for the next ring block
        PtrSink<VEC, true> o;
        o.yb = nullptr;
        o.qb[0] = a.q + (fb * a.ldq + j0) * QB;
        o.qb[1] = qm_two_pieces(QM) ? a.q1 + (fb * a.ldq + j0) * QB : nullptr;
        o.sb = nullptr;
        o.ldy = 0;
        o.ldq = a.ldq * QB;
        o.nsc = 0;
#pragma unroll
        for (int u = 0; u < MT; ++u)
            if (u < nu) fir_store_frame<VEC, QM>(ys[u], sexp[u], col, o, u);
        // The next block writes smax only after this block's reads of it
        // (the barrier above) and sexp only after its first barrier, which
        // every thread reaches once done with these stores.
    }
}

template <int VEC, int MT, bool EXACT, int QM>
__global__ __launch_bounds__(kFrameMaxThreads) void fir_frame_kernel(FirArgs a, int TF) {
    __shared__ float smax[kFrameMaxThreads / 64 * MT];
    __shared__ int sexp[MT];
    frame_unit<VEC, MT, EXACT, QM>(a, TF, blockIdx.x, smax, sexp);
}

// Batched: every item whose frame row is exactly 1024 threads of VEC floats
// (W = 1024, 2048 or 4096) and whose tap count has an exact ring here
// (fir_frame_batch_vec) runs its frame runs as units of this persistent
// kernel, each XCD's blocks walking that XCD's cost-balanced range; the
// other items of a per-frame scaled batch take the three launches.  The ring
// is unrolled for the item's own M, as in the streaming batched FIR.
template <int VEC, int M0, int MMAX, int QM>
__device__ __forceinline__ void frame_unit_own_m(const FirArgs& a, int TF, int64_t run, float* smax, int* sexp) {
    if constexpr (M0 <= MMAX) {
        if (a.M == M0) frame_unit<VEC, M0, true, QM>(a, TF, run, smax, sexp);
        else frame_unit_own_m<VEC, M0 + 1, MMAX, QM>(a, TF, run, smax, sexp);
    }
}

template <int QM>
__global__ __launch_bounds__(kFrameMaxThreads) void fir_frame_batch_kernel(const BatchTable* __restrict__ t) {
    __shared__ float smax[kFrameMaxThreads / 64 * 16];
    __shared__ int sexp[16];
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const int64_t end = t->frame_bounds[x + 1];
    for (int64_t u = t->frame_bounds[x] + i; u < end; u += nbx) {
        const int it = batch_find(t->items, t->n_items, u, /*stage=*/3);
        const BatchItem& b = t->items[it];
        const FirArgs fa = b.fir;  // a private copy (see fir_batch_kernel)
        const int64_t run = u - b.frame_unit0;
        switch (fa.W) {  // uniform over the block: one item per unit
            case 1024: frame_unit_own_m<1, 1, 16, QM>(fa, b.fir_tf, run, smax, sexp); break;
            case 2048: frame_unit_own_m<2, 1, 16, QM>(fa, b.fir_tf, run, smax, sexp); break;
            default: frame_unit_own_m<4, 1, 8, QM>(fa, b.fir_tf, run, smax, sexp); break;
        }
    }
}

template <int VEC, int MT, bool EXACT, int QM>
hipError_t launch_frame_one(const FirArgs& a, hipStream_t s) {
    const int TF = MT * ((128 + MT - 1) / MT);  // whole ring blocks, at least 128 frames per block
    const int64_t blocks = (a.F + TF - 1) / TF;
    hipLaunchKernelGGL((fir_frame_kernel<VEC, MT, EXACT, QM>), dim3((unsigned)blocks), dim3(a.W / VEC), 0, s, a, TF);
    return hipGetLastError();
}

template <int VEC, int QM>
hipError_t launch_frame_vec(const FirArgs& a, hipStream_t s) {
    // The ring unrolled for the exact tap count up to 16 (8 at four floats per
    // thread); more taps take the 32-frame ring with the taps beyond M off.
    switch (a.M) {
#define TINA_FRAME_M(m) case m: return launch_frame_one<VEC, m, true, QM>(a, s);
        TINA_FRAME_M(1) TINA_FRAME_M(2) TINA_FRAME_M(3) TINA_FRAME_M(4)
        TINA_FRAME_M(5) TINA_FRAME_M(6) TINA_FRAME_M(7) TINA_FRAME_M(8)
#undef TINA_FRAME_M
        default: break;
    }
    if constexpr (VEC <= 2) {
        switch (a.M) {
#define TINA_FRAME_M(m) case m: return launch_frame_one<VEC, m, true, QM>(a, s);
            TINA_FRAME_M(9) TINA_FRAME_M(10) TINA_FRAME_M(11) TINA_FRAME_M(12)
            TINA_FRAME_M(13) TINA_FRAME_M(14) TINA_FRAME_M(15) TINA_FRAME_M(16)
#undef TINA_FRAME_M
            default: break;
        }
    }
    if constexpr (VEC == 1) {
        if (a.M <= 32) return launch_frame_one<1, 32, false, QM>(a, s);
    }
    return hipErrorInvalidValue;
}

template <int QM>
hipError_t launch_frame_qm(const FirArgs& a, int vec, hipStream_t s) {
    switch (vec) {
        case 4: return launch_frame_vec<4, QM>(a, s);
        case 2: return launch_frame_vec<2, QM>(a, s);
        default: return launch_frame_vec<1, QM>(a, s);
    }
}

}  // namespace

int fir_frame_vec(const FirArgs& a) {
    if (!qmode_frame_scaled(a.qmode) || !a.fexp || !a.q || (a.qmode == QM_FP16FX2 && !a.q1)) return 0;
    auto aligned = [](const void* p, int bytes) { return ((uintptr_t)p % bytes) == 0; };
    // The widest vector (fewest per-frame reduction steps per float) whose
    // ring fits the register budget of 1024 threads: 4 floats up to 8 taps,
    // 2 up to 16, 1 up to 32; at least one whole wave per frame row and at
    // most 1024 threads.
    int vec = a.M <= 8 ? 4 : (a.M <= 16 ? 2 : (a.M <= 32 ? 1 : 0));
    while (vec > 1 && a.W % (64 * vec) != 0) vec /= 2;
    if (vec == 0 || a.W % (64 * vec) != 0 || a.W / vec > kFrameMaxThreads) return 0;
    if (a.plen % vec != 0 || !aligned(a.chunk, 4 * vec) || (a.prefix && !aligned(a.prefix, 4 * vec))) return 0;
    if (a.qmode == QM_FP8F) {
        if (!aligned(a.q, 4) || a.ldq % 4 != 0) return 0;  // 4 codes per store
    } else if (!aligned(a.q, 2 * vec) || (a.q1 && !aligned(a.q1, 2 * vec)) || a.ldq % vec != 0) {
        return 0;
    }
    return vec;
}

int fir_frame_batch_vec(const FirArgs& a) {
    if (!qmode_frame_scaled(a.qmode)) return 0;
    const int vec = a.W == 1024 ? 1 : (a.W == 2048 ? 2 : (a.W == 4096 ? 4 : 0));
    if (vec == 0 || a.M < 1 || a.M > (vec == 4 ? 8 : 16)) return 0;
    auto aligned = [](const void* p, int bytes) { return ((uintptr_t)p % bytes) == 0; };
    if (a.plen % vec != 0 || !aligned(a.chunk, 4 * vec) || (a.prefix && !aligned(a.prefix, 4 * vec))) return 0;
    if (a.qmode == QM_FP8F) {
        if (!aligned(a.q, 4) || a.ldq % 4 != 0) return 0;
    } else if (!aligned(a.q, 2 * vec) || (a.q1 && !aligned(a.q1, 2 * vec)) || a.ldq % vec != 0) {
        return 0;
    }
    return vec;
}


hipError_t launch_fir_frame_batch(const BatchTable* t, int qmode, int grid, hipStream_t s) {
    switch (qmode) {
        case QM_FP8F: hipLaunchKernelGGL(fir_frame_batch_kernel<QM_FP8F>, dim3(grid), dim3(kFrameMaxThreads), 0, s, t); break;
        case QM_FP16F: hipLaunchKernelGGL(fir_frame_batch_kernel<QM_FP16F>, dim3(grid), dim3(kFrameMaxThreads), 0, s, t); break;
        case QM_FP16FX2: hipLaunchKernelGGL(fir_frame_batch_kernel<QM_FP16FX2>, dim3(grid), dim3(kFrameMaxThreads), 0, s, t); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fir_frame(const FirArgs& a, hipStream_t s) {
    const int vec = fir_frame_vec(a);
    if (vec == 0) return hipErrorInvalidValue;
    switch (a.qmode) {
        case QM_FP8F: return launch_frame_qm<QM_FP8F>(a, vec, s);
        case QM_FP16F: return launch_frame_qm<QM_FP16F>(a, vec, s);
        case QM_FP16FX2: return launch_frame_qm<QM_FP16FX2>(a, vec, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tina
