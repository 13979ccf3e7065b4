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
//
// This file: host-side launch choices and the state-gather kernels; the FIR
// kernels themselves are in fir_kernels.h, instantiated per output mode in
// fir_out_*.hip.
#include "fir_kernels.h"

namespace tina {

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

int pick_vec(const FirArgs& a) {
    auto aligned = [](const void* p, int bytes) { return ((uintptr_t)p % bytes) == 0; };
    // Vector width by register budget (taps, ring and prefetch each take
    // MT*VEC registers): 4 floats for up to 8 taps, else 1 (measured best).
    int vec = a.M <= 8 ? 4 : 1;
    // Block-scaled output: 4 floats per thread up to 16 taps (the per-block
    // maximum is then shared among 8 lanes, and a lane's 4 codes leave in one
    // store; measured faster than 1 or 2 at 16 taps).
    // (9..15 taps take 2, whose ring can be unrolled for the exact count.)
    if ((a.qmode == QM_MX || a.qmode == QM_FP8F) && a.M <= 16) vec = (a.M <= 8 || a.M == 16) ? 4 : 2;
    const FirTune tune = fir_tune();
    if (tune.vec == 1 || tune.vec == 2 || tune.vec == 4) vec = tune.vec;
    if (vec == 4 && a.M > 16) vec = 2;  // widest ring per vector width: 16 taps (VEC 4), 32 (VEC 2), 64 (VEC 1)
    if (vec == 2 && a.M > 32) vec = 1;
    auto out_ok = [&](int v) {
        if (a.qmode == QM_AMAXONLY) return true;  // nothing but the partial maxima
        if (a.qmode == QM_MX || a.qmode == QM_FP8F) return aligned(a.q, 4) && a.ldq % 4 == 0;  // 4-byte code stores
        if (a.qmode != QM_NONE)  // bf16 / fp16: 2 v bytes per store
            return aligned(a.q, 2 * v) && (a.q1 == nullptr || aligned(a.q1, 2 * v)) && a.ldq % v == 0;
        return aligned(a.y, 4 * v) && a.ldy % v == 0;
    };
    while (vec > 1 && !(a.plen % vec == 0 && aligned(a.chunk, 4 * vec) && out_ok(vec) &&
                        (a.prefix == nullptr || aligned(a.prefix, 4 * vec))))
        vec >>= 1;
    return vec;
}

namespace {

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

// Largest value over a wave (all 64 lanes take part).
__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// e_f = frame_exponent(largest partial maximum of frame f, limit): one wave
// per frame, its lanes reading the frame's partial maxima side by side.
__device__ inline void frame_exponent_wave(const float* __restrict__ amax, int nparts, int64_t f, float limit,
                                           int32_t* __restrict__ fexp) {
    const int lane = threadIdx.x & 63;
    float m = 0.0f;
    for (int q = lane; q < nparts; q += 64) m = fmaxf(m, amax[f * nparts + q]);
    m = wave_max(m);
    if (lane == 0) fexp[f] = frame_exponent(m, limit);
}

__global__ __launch_bounds__(256) void frame_exponent_kernel(const float* __restrict__ amax, int nparts, int64_t F,
                                                             float limit, int32_t* __restrict__ fexp) {
    const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (f < F) frame_exponent_wave(amax, nparts, f, limit, fexp);  // wave-uniform
}

// The same for every item of a batch that takes the three launches (items
// of the single-pass frame stage derive their exponents themselves): the
// grid's waves share each item's frames, item after item.
__global__ __launch_bounds__(256) void frame_exponent_batch_kernel(const BatchTable* __restrict__ t, float limit) {
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    for (int it = 0; it < t->n_items; ++it) {
        if (t->items[it].fir_single) continue;
        const FirArgs& a = t->items[it].fir;
        for (int64_t f = w; f < a.F; f += nw) frame_exponent_wave(a.amax, a.nparts, f, limit, a.fexp);
    }
}

}  // namespace

hipError_t launch_gather_batch(const BatchTable* t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(gather_batch_kernel, dim3(grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

int fir_amax_parts(const FirArgs& a) {
    const int ct = a.W / pick_vec(a);
    const int gw = ct < 32 ? ct : 32;
    return ct / gw;
}

hipError_t launch_fir(FirArgs& a, hipStream_t s) {
    if (a.F <= 0) return hipSuccess;
    const int vec = pick_vec(a);
    {
        const int ct = a.W / vec;
        const int gw = ct < 32 ? ct : 32;
        a.nparts = ct / gw;
    }
    if (qmode_frame_scaled(a.qmode)) {
        // Per-frame scaled codes: the frame's maximum must be known before its
        // first code is written.  Frames of at most 4096 floats: one block
        // holds whole frame rows and does it in one pass over the input.
        // Wider frames span many blocks: pass 1 finds the partial maxima, a
        // small kernel the exponents, and pass 2 recomputes the FIR (reading
        // the input again is cheaper than writing and reading FP32 rows) and
        // writes the scaled codes.
        if (fir_frame_vec(a) != 0) return launch_fir_frame(a, s);
        if (!a.amax || !a.fexp || !a.q || (a.qmode == QM_FP16FX2 && !a.q1)) return hipErrorInvalidValue;
        FirArgs p1 = a;
        p1.qmode = QM_AMAXONLY;
        p1.y = nullptr;
        p1.q = p1.q1 = p1.qs = nullptr;
        const int v1 = pick_vec(p1);
        {
            const int ct = a.W / v1;
            p1.nparts = ct / (ct < 32 ? ct : 32);
        }
        hipError_t e = launch_fir_mode_amaxonly(p1, v1, s);
        if (e != hipSuccess) return e;
        const float limit = a.qmode == QM_FP8F ? 448.0f : 32768.0f;
        hipLaunchKernelGGL(frame_exponent_kernel, dim3((unsigned)((a.F + 3) / 4)), dim3(256), 0, s, p1.amax,
                           p1.nparts, a.F, limit, a.fexp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        a.nparts = p1.nparts;
        switch (a.qmode) {
            case QM_FP8F: return launch_fir_mode_fp8f(a, vec, s);
            case QM_FP16F: return launch_fir_mode_fp16f(a, vec, s);
            default: return launch_fir_mode_fp16fx2(a, vec, s);
        }
    }
    if (a.qmode == QM_MX) return launch_fir_mode_mx(a, vec, s);
    if (a.qmode == QM_BF16) return launch_fir_mode_bf16(a, vec, s);
    if (a.qmode == QM_BF16X2) return launch_fir_mode_bf16x2(a, vec, s);
    return launch_fir_mode_f32(a, vec, s);
}

hipError_t launch_fir_batch(const BatchTable* t, int max_m, bool all_exact, int qmode, int grid, hipStream_t s,
                            bool frame_stage) {
    if (qmode_frame_scaled(qmode)) {
        // Items with whole frame rows of 1024 threads: one pass (frame stage);
        // the others as in launch_fir: maxima, exponents, codes.
        hipError_t e = hipSuccess;
        if (frame_stage) e = launch_fir_frame_batch(t, qmode, grid / 4, s);  // one 1024-thread block per CU
        if (e != hipSuccess) return e;
        e = launch_fir_batch_mode_amaxonly(t, max_m, all_exact, grid, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(frame_exponent_batch_kernel, dim3(grid), dim3(256), 0, s, t,
                           qmode == QM_FP8F ? 448.0f : 32768.0f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        switch (qmode) {
            case QM_FP8F: return launch_fir_batch_mode_fp8f(t, max_m, all_exact, grid, s);
            case QM_FP16F: return launch_fir_batch_mode_fp16f(t, max_m, all_exact, grid, s);
            default: return launch_fir_batch_mode_fp16fx2(t, max_m, all_exact, grid, s);
        }
    }
    if (qmode == QM_MX) return launch_fir_batch_mode_mx(t, max_m, all_exact, grid, s);
    if (qmode == QM_BF16) return launch_fir_batch_mode_bf16(t, max_m, all_exact, grid, s);
    if (qmode == QM_BF16X2) return launch_fir_batch_mode_bf16x2(t, max_m, all_exact, grid, s);
    return launch_fir_batch_mode_f32(t, max_m, all_exact, grid, s);
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

