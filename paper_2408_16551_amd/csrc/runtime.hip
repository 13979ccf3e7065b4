// C ABI: plans, per-stream state and the execute call of the filter bank.
//
// Execute enqueues, on the caller's stream:
//   1. the polyphase FIR (fir.hip) over history ++ residue ++ new samples,
//      into the caller's output (FIR-only plans) or into the plan's FP32
//      workspace, with per-frame |y| maxima for the scaled forms;
//   2. the DFT-across-branches GEMM (gemm.hip) from the workspace into the
//      caller's complex64 output;
//   3. with a state: the new history and residue gathered into the state's
//      other buffer (ping-pong, so the FIR of this call still reads the old one).
// Inputs larger than the workspace run as consecutive frame pieces.
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "runtime_types.h"

using namespace tina;

thread_local std::string g_err;

tina_status tina_fail(tina_status s, const std::string& msg) {
    g_err = msg;
    return s;
}


extern "C" {

const char* tina_last_error(void) { return g_err.c_str(); }

const char* tina_version(void) { return "tina_pfb 0.1 (gfx950)"; }

tina_status tina_pfb_plan(const tina_pfb_desc* d, tina_pfb_plan_t* out) {
    if (!d || !out) return fail(TINA_ERR_INVALID_ARGUMENT, "plan: NULL descriptor or output handle");
    *out = nullptr;
    if (d->struct_size < offsetof(tina_pfb_desc, workspace_bytes))
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: struct_size too small");
    const int64_t ws_req = d->struct_size >= offsetof(tina_pfb_desc, dft_algorithm) ? d->workspace_bytes : 0;
    const int dft_alg = d->struct_size >= offsetof(tina_pfb_desc, reserved_) ? d->dft_algorithm : TINA_DFT_DENSE;
    if (dft_alg != TINA_DFT_DENSE && dft_alg != TINA_DFT_FACTORED && dft_alg != TINA_DFT_FUSED &&
        dft_alg != TINA_DFT_COMPENSATED && dft_alg != TINA_DFT_TABLE)
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: unknown dft_algorithm");
    if (d->sample_type != TINA_SAMPLE_R32 && d->sample_type != TINA_SAMPLE_C64)
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: unknown sample_type");
    if (d->window < TINA_WINDOW_RECT || d->window > TINA_WINDOW_CUSTOM)
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: unknown window");
    if (d->output != TINA_OUT_PFB && d->output != TINA_OUT_FIR_ONLY && d->output != TINA_OUT_INVERSE)
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: unknown output");
    if (d->output != TINA_OUT_FIR_ONLY && (d->precision < TINA_PREC_FP32 || d->precision > TINA_PREC_MXFP8))
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: unknown precision");
    if (d->window == TINA_WINDOW_CUSTOM && !d->custom_taps)
        return fail(TINA_ERR_INVALID_ARGUMENT, "plan: CUSTOM window without custom_taps");
    if (d->channels <= 0 || d->taps <= 0) return fail(TINA_ERR_INVALID_ARGUMENT, "plan: channels and taps must be positive");
    if (!is_pow2(d->channels) || d->channels < 16 || d->channels > 8192)
        return fail(TINA_ERR_UNSUPPORTED, "plan: channels must be a power of two in [16, 8192]");
    if (d->taps > 64) return fail(TINA_ERR_UNSUPPORTED, "plan: taps must be in [1, 64]");
    if (d->output == TINA_OUT_INVERSE &&
        (d->sample_type != TINA_SAMPLE_C64 || dft_alg != TINA_DFT_DENSE ||
         !(d->precision == TINA_PREC_FP32 || d->precision == TINA_PREC_BF16 || d->precision == TINA_PREC_BF16X3)))
        return fail(TINA_ERR_UNSUPPORTED, "plan: the synthesis bank needs complex64, the dense DFT and FP32, BF16 or BF16X3");
    if (d->output == TINA_OUT_PFB && d->precision == TINA_PREC_MXFP8 &&
        (int64_t)d->channels * (d->sample_type == TINA_SAMPLE_C64 ? 2 : 1) % 128 != 0)
        return fail(TINA_ERR_UNSUPPORTED, "plan: MXFP8 needs 128 | channels (real) or 64 | channels (complex)");
    if (dft_alg == TINA_DFT_FUSED && d->output == TINA_OUT_PFB &&
        (d->precision != TINA_PREC_FP32 || d->taps > 16 || (int64_t)d->channels * (d->sample_type == TINA_SAMPLE_C64 ? 2 : 1) % 32 != 0))
        return fail(TINA_ERR_UNSUPPORTED, "plan: the fused FIR + DFT needs FP32, taps <= 16 and 32 | channels * floats per sample");
    if (dft_alg == TINA_DFT_FACTORED && d->output == TINA_OUT_PFB &&
        (d->precision != TINA_PREC_FP32 || !fft_supported(d->channels)))
        return fail(TINA_ERR_UNSUPPORTED, "plan: the factored DFT needs FP32 and 256 <= channels <= 4096");
    if (dft_alg == TINA_DFT_COMPENSATED && d->output == TINA_OUT_PFB && d->precision != TINA_PREC_FP32)
        return fail(TINA_ERR_UNSUPPORTED, "plan: compensated accumulation needs FP32");
    if (dft_alg == TINA_DFT_TABLE && d->output == TINA_OUT_PFB && d->precision != TINA_PREC_FP32)
        return fail(TINA_ERR_UNSUPPORTED, "plan: the twiddle-table operand needs FP32");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(TINA_ERR_DEVICE, "plan: no HIP device");
    if (d->device < 0 || d->device >= ndev) return fail(TINA_ERR_INVALID_ARGUMENT, "plan: bad device ordinal");

    DeviceScope ds(d->device);
    if (ds.err != hipSuccess) return fail(TINA_ERR_DEVICE, "plan: hipSetDevice failed");

    tina_pfb_plan_s* p = new (std::nothrow) tina_pfb_plan_s();
    if (!p) return fail(TINA_ERR_OUT_OF_MEMORY, "plan: host allocation");
    p->device = d->device;
    p->P = d->channels;
    p->M = d->taps;
    p->sample_type = d->sample_type;
    p->cf = d->sample_type == TINA_SAMPLE_C64 ? 2 : 1;
    p->W = p->P * p->cf;
    p->window = d->window;
    p->precision = d->output != TINA_OUT_FIR_ONLY ? d->precision : TINA_PREC_FP32;
    p->output = d->output;
    p->dft_algorithm = d->output == TINA_OUT_PFB ? dft_alg : TINA_DFT_DENSE;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, d->device) == hipSuccess && prop.multiProcessorCount > 0)
            p->cus = prop.multiProcessorCount;
    }
    p->K = p->W;
    p->N = p->W;
    p->kout = d->output != TINA_OUT_PFB ? p->P : (p->cf == 2 ? p->P : p->P / 2 + 1);

    auto bail = [&](tina_status st, const std::string& m) {
        p->release();
        delete p;
        return fail(st, m);
    };
    const int64_t L = (int64_t)p->P * p->M;
    if (hipMalloc(&p->h64, L * sizeof(double)) != hipSuccess || hipMalloc(&p->h32, L * sizeof(float)) != hipSuccess)
        return bail(TINA_ERR_OUT_OF_MEMORY, "plan: taps allocation");
    hipError_t e;
    if (d->window == TINA_WINDOW_CUSTOM) {
        e = hipMemcpy(p->h64, d->custom_taps, L * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_taps_to_f32(p->h64, p->h32, L, nullptr);
    } else {
        e = launch_window(p->h64, p->h32, p->P, p->M, d->window, nullptr);
    }
    if (e != hipSuccess) return bail(TINA_ERR_DEVICE, std::string("plan: taps: ") + hipGetErrorString(e));

    if (p->output != TINA_OUT_FIR_ONLY) {
        const int form = p->precision;
        if (p->output == TINA_OUT_INVERSE) {
            const int64_t nbytes = (int64_t)p->N * p->K * form_elem_bytes(form);
            for (int i = 0; i < form_pieces(form); ++i)
                if (hipMalloc(&p->B[i], nbytes) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "plan: IDFT operand allocation");
            if (hipMalloc(&p->g32, L * sizeof(float)) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "plan: synthesis taps");
            for (int i = 0; i < 2; ++i)
                if (hipMalloc(&p->hist[i], std::max<int64_t>(1, (int64_t)(p->M - 1) * p->W) * sizeof(float)) != hipSuccess)
                    return bail(TINA_ERR_OUT_OF_MEMORY, "plan: synthesis history");
            e = launch_dft_operand(p->B[0], p->B[1], p->P, 1, form, nullptr, /*inverse=*/1);
            if (e == hipSuccess) e = launch_synthesis_taps(p->h64, p->g32, p->P, p->M, nullptr);
        } else if (p->dft_algorithm == TINA_DFT_FACTORED) {
            int P1, P2;
            fft_factors(p->P, P1, P2);
            if (hipMalloc(&p->fft_mat1, sizeof(float) * 4 * P1 * P1) != hipSuccess ||
                (P1 != P2 && hipMalloc(&p->fft_mat3, sizeof(float) * 4 * P2 * P2) != hipSuccess) ||
                hipMalloc(&p->fft_tw, sizeof(float) * 2 * p->P) != hipSuccess)
                return bail(TINA_ERR_OUT_OF_MEMORY, "plan: factored DFT tables");
            e = launch_fft_tables(p->fft_mat1, p->fft_mat3, p->fft_tw, p->P, nullptr);
        } else if (p->dft_algorithm == TINA_DFT_TABLE) {  // no N x K operand: P twiddles
            if (hipMalloc(&p->fft_tw, sizeof(float) * 2 * p->P) != hipSuccess)
                return bail(TINA_ERR_OUT_OF_MEMORY, "plan: twiddle table");
            e = launch_twiddle_table(p->fft_tw, p->P, nullptr);
        } else if (form_mx(form)) {
            if (hipMalloc(&p->B[0], mx_codes_bytes(p->N, p->K)) != hipSuccess ||
                hipMalloc(&p->B[1], (int64_t)p->N * (p->K / 32)) != hipSuccess)
                return bail(TINA_ERR_OUT_OF_MEMORY, "plan: DFT operand allocation");
            e = launch_dft_operand(p->B[0], p->B[1], p->P, p->cf == 2, form, nullptr);
        } else {
            const int64_t nbytes = (int64_t)p->N * p->K * form_elem_bytes(form);
            for (int i = 0; i < form_pieces(form); ++i)
                if (hipMalloc(&p->B[i], nbytes) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "plan: DFT operand allocation");
            e = launch_dft_operand(p->B[0], p->B[1], p->P, p->cf == 2, form, nullptr);
        }
        if (e != hipSuccess) return bail(TINA_ERR_DEVICE, std::string("plan: DFT operand: ") + hipGetErrorString(e));
        const int64_t ws_bytes = ws_req == 0 ? kWorkspaceBytes : ws_req;
        p->ch_frames = ws_bytes > 0 ? ws_bytes / ((int64_t)p->W * 4) : 0;
        p->ch_frames = p->ch_frames >= 128 ? (p->ch_frames / 128) * 128 : p->ch_frames;
        if (ws_bytes > 0 && p->ch_frames < 1) p->ch_frames = 1;
        if (p->ch_frames > 0 && hipMalloc(&p->ws, p->ch_frames * p->W * sizeof(float)) != hipSuccess)
            return bail(TINA_ERR_OUT_OF_MEMORY, "plan: workspace allocation");
        if (p->ch_frames > 0 && form_scaled(form)) {
            p->amax_parts_cap = p->W / 32 > 1 ? p->W / 32 : 1;  // the most parts: one per 32 lanes at VEC = 1
            if (hipMalloc(&p->amax, p->ch_frames * p->amax_parts_cap * sizeof(float)) != hipSuccess ||
                hipMalloc(&p->fexp, p->ch_frames * sizeof(int32_t)) != hipSuccess)
                return bail(TINA_ERR_OUT_OF_MEMORY, "plan: scale workspace allocation");
        }
    }
    // The tables above were generated on the null stream: wait for it alone,
    // so that a plan made while other work runs on non-blocking streams (a
    // server's steps) does not wait for that work.
    e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return bail(TINA_ERR_DEVICE, std::string("plan: ") + hipGetErrorString(e));
    *out = p;
    return TINA_OK;
}

tina_status tina_pfb_plan_destroy(tina_pfb_plan_t p) {
    if (!p) return TINA_OK;
    DeviceScope ds(p->device);
    (void)hipDeviceSynchronize();
    p->release();
    delete p;
    return TINA_OK;
}

tina_status tina_pfb_channels_out(tina_pfb_plan_t p, int64_t* ch) {
    if (!p || !ch) return fail(TINA_ERR_INVALID_ARGUMENT, "channels_out: NULL argument");
    *ch = p->kout;
    return TINA_OK;
}

tina_status tina_pfb_plan_taps(tina_pfb_plan_t p, double* host) {
    if (!p || !host) return fail(TINA_ERR_INVALID_ARGUMENT, "plan_taps: NULL argument");
    DeviceScope ds(p->device);
    HIP_TRY(hipMemcpy(host, p->h64, (size_t)p->P * p->M * sizeof(double), hipMemcpyDeviceToHost));
    return TINA_OK;
}

tina_status tina_pfb_output_frames(tina_pfb_plan_t p, tina_pfb_state_t st, int64_t n, int64_t* frames) {
    if (!p || !frames) return fail(TINA_ERR_INVALID_ARGUMENT, "output_frames: NULL argument");
    if (n < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "output_frames: negative sample count");
    if (st && st->plan != p) return fail(TINA_ERR_INVALID_ARGUMENT, "output_frames: state belongs to another plan");
    const int64_t r = st ? st->residue : 0;
    *frames = (r + n) / p->P;
    return TINA_OK;
}

}  // extern "C"

namespace {

// Device memory one execute call works in between the FIR and the DFT: the
// FIR output (or the GEMM operand codes), per-frame partial maxima and frame
// exponents, sized for pieces of ch_frames frames.
struct ExecWorkspace {
    float* ws = nullptr;
    float* amax = nullptr;
    int32_t* fexp = nullptr;
    int64_t ch_frames = 0;
    bool use_plan = true;  // the plan's own workspace: calls are ordered across streams and may be timed
};

tina_status execute_with(tina_pfb_plan_s* p, const void* d_in, int64_t n, void* d_out, int64_t cap,
                         tina_pfb_state_t st, int64_t* frames_written, void* stream, const ExecWorkspace& w,
                         const char* who) {
    const std::string name(who);
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": NULL plan");
    if (n < 0) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": negative sample count");
    if (n > 0 && !d_in) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": NULL input");
    if (st && st->plan != p) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": state belongs to another plan");
    const size_t sbytes = p->cf * sizeof(float);
    if ((uintptr_t)d_in % sbytes) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": input not aligned to its sample size");
    const int64_t r = st ? st->residue : 0;
    const int64_t F = (r + n) / p->P;
    if (F > 0 && !d_out) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": NULL output");
    const size_t obytes = p->output == TINA_OUT_PFB ? 8 : sbytes;
    if ((uintptr_t)d_out % obytes) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": output misaligned");
    if (F > cap) return fail(TINA_ERR_INVALID_ARGUMENT, name + ": output capacity (" + std::to_string(cap) +
                                                         " frames) below frame count " + std::to_string(F));
    if (p->output == TINA_OUT_INVERSE)
        return fail(TINA_ERR_INVALID_ARGUMENT, name + ": synthesis plans run through tina_pfb_synthesize");
    if (p->output == TINA_OUT_PFB && w.ch_frames == 0)
        return fail(TINA_ERR_UNSUPPORTED, name + ": plan was created without a workspace (batch/server use only)");
    if (!w.use_plan && p->output == TINA_OUT_PFB && F > w.ch_frames)
        return fail(TINA_ERR_TOO_LARGE, name + ": " + std::to_string(F) + " frames exceed the " +
                                            std::to_string(w.ch_frames) + " frames per call that the " +
                                            std::to_string(kStaticScratchBytes >> 20) +
                                            " MiB static scratch holds for this plan");
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return fail(TINA_ERR_DEVICE, name + ": hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    if (w.use_plan) HIP_TRY(p->order.begin(s));
    if (st) st->plan_ordered = false;  // until this call's work is covered by the order event

    FirArgs fa{};
    fa.prefix = st ? st->buf[st->cur] : nullptr;
    fa.plen = (int64_t)(p->M - 1) * p->W + r * p->cf;
    fa.chunk = (const float*)d_in;
    fa.nchunk = n * p->cf;
    fa.taps = p->h32;
    fa.W = p->W;
    fa.P = p->P;
    fa.M = p->M;
    fa.cf = p->cf;

    // Records a HIP event pair around one stage launch when profiling.
    auto timed = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& list, auto&& launch) -> hipError_t {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (p->profiling && w.use_plan) {
            e0 = p->next_event();
            e1 = p->next_event();
            if (e0 && e1) (void)hipEventRecord(e0, s);
        }
        hipError_t e = launch();
        if (e == hipSuccess && e0 && e1) {
            e = hipEventRecord(e1, s);
            list.emplace_back(e0, e1);
        }
        return e;
    };

    if (p->output == TINA_OUT_FIR_ONLY) {
        fa.y = (float*)d_out;
        fa.ldy = p->W;
        fa.g0 = 0;
        fa.F = F;
        fa.amax = nullptr;
        if (F > 0) HIP_TRY(timed(p->ev_fir, [&] { return launch_fir(fa, s); }));
    } else {
        const int form = p->precision;
        const int64_t ldo = p->cf == 2 ? 2 * (int64_t)p->P : (int64_t)p->P + 2;
        for (int64_t c0 = 0; c0 < F; c0 += w.ch_frames) {
            const int64_t Fc = F - c0 < w.ch_frames ? F - c0 : w.ch_frames;
            fa.y = w.ws;
            fa.ldy = p->W;
            fa.g0 = c0;
            fa.F = Fc;
            fa.amax = form_scaled(form) ? w.amax : nullptr;
            // Operand-form FIR output in the FP32 workspace (4 bytes per float):
            // E4M3 codes (then the block scales), or the 16-bit piece(s) one
            // after the other; per-frame scaled forms also keep the frames'
            // exponents beside their partial maxima.
            fa.qmode = form_fir_qmode(form);
            if (fa.qmode != 0) {
                fa.y = nullptr;
                fa.q = (uint8_t*)w.ws;
                fa.ldq = p->W;
                if (form_mx(form)) fa.qs = (uint8_t*)w.ws + mx_codes_bytes(w.ch_frames, p->W);
                if (form == TINA_PREC_BF16X3 || form == TINA_PREC_FP16X3)
                    fa.q1 = (uint8_t*)w.ws + (int64_t)w.ch_frames * p->W * 2;
                if (form_scaled(form)) fa.fexp = w.fexp;
            }
            if (p->dft_algorithm == TINA_DFT_FUSED && fused_supported(fa, form)) {
                GemmArgs ga{};
                ga.B0 = p->B[0];
                ga.out = (float*)d_out + c0 * ldo;
                ga.ldo = ldo;
                ga.F = Fc;
                ga.K = p->K;
                ga.N = p->N;
                ga.real_pack = p->cf == 1;
                ga.form = form;
                HIP_TRY(timed(p->ev_dft, [&] { return launch_dft_fused(ga, fa, s); }));
                continue;
            }
            HIP_TRY(timed(p->ev_fir, [&] { return launch_fir(fa, s); }));
            if (p->dft_algorithm == TINA_DFT_FACTORED) {
                FftArgs xa{};
                xa.y = w.ws;
                xa.ldy = p->W;
                xa.F = Fc;
                xa.mat1 = p->fft_mat1;
                xa.mat3 = p->fft_mat3;
                xa.tw = p->fft_tw;
                xa.out = (float*)d_out + c0 * ldo;
                xa.ldo = ldo;
                xa.P = p->P;
                xa.cplx = p->cf == 2;
                xa.cus = p->cus;
                HIP_TRY(timed(p->ev_dft, [&] { return launch_fft_dft(xa, s); }));
                continue;
            }
            GemmArgs ga{};
            ga.A = w.ws;
            ga.lda = p->W;
            ga.B0 = p->B[0];
            ga.B1 = p->B[1];
            ga.out = (float*)d_out + c0 * ldo;
            ga.ldo = ldo;
            ga.F = Fc;
            ga.K = p->K;
            ga.N = p->N;
            ga.real_pack = p->cf == 1;
            ga.form = form;
            ga.Aq = fa.q;
            ga.Aq1 = fa.q1;
            ga.Aqs = fa.qs;
            ga.fexp = fa.fexp;
            ga.compensated = p->dft_algorithm == TINA_DFT_COMPENSATED;
            ga.tw = p->dft_algorithm == TINA_DFT_TABLE ? p->fft_tw : nullptr;
            HIP_TRY(timed(p->ev_dft, [&] { return launch_dft_gemm(ga, s); }));
        }
    }
    if (st) {
        const int64_t r2 = (r + n) % p->P;
        const int64_t count = (int64_t)(p->M - 1) * p->W + r2 * p->cf;
        HIP_TRY(launch_gather_ext(fa.prefix, fa.plen, fa.chunk, fa.nchunk, st->buf[st->cur ^ 1], F * p->W, count, s));
        st->cur ^= 1;
        st->residue = r2;
    }
    if (w.use_plan) HIP_TRY(p->order.end(s));
    if (st) st->plan_ordered = w.use_plan && p->order.valid;
    if (frames_written) *frames_written = F;
    return TINA_OK;
}

// Static scratch of the allocation-free execute: one per device, at a
// device address that hipGetSymbolAddress reports once per device (the host
// name of the array is not a device address).
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The scratch's device address on the current device `dev` (set up on the
// first call there); nullptr with the HIP error in *e on failure.
void* scratch_address(int dev, hipError_t* e) {
    *e = hipSuccess;
    if (dev < 0 || dev >= kMaxDevices) {
        *e = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        *e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*e != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

// Frames per call that the scratch holds for plan p, and the workspace laid
// out in it at base (FIR output or operand codes, then per-frame partial
// maxima and exponents, each 256-byte aligned).
ExecWorkspace scratch_workspace(const tina_pfb_plan_s* p, uint8_t* base) {
    ExecWorkspace w;
    w.use_plan = false;
    const bool scaled = form_scaled(p->precision) && p->output == TINA_OUT_PFB;
    const int64_t parts = p->W / 32 > 1 ? p->W / 32 : 1;  // the most partial maxima per frame (as at plan time)
    const int64_t per_frame = (int64_t)p->W * 4 + (scaled ? parts * 4 + 4 : 0);
    int64_t ch = (kStaticScratchBytes - (scaled ? 512 : 0)) / per_frame;  // 512: alignment of maxima, exponents
    if (ch >= 128) ch = ch / 128 * 128;
    w.ch_frames = ch;
    w.ws = (float*)base;
    if (scaled) {
        const int64_t amax_off = align256(ch * p->W * 4);
        const int64_t fexp_off = align256(amax_off + ch * parts * 4);
        w.amax = (float*)(base + amax_off);
        w.fexp = (int32_t*)(base + fexp_off);
    }
    return w;
}

}  // namespace

extern "C" {

tina_status tina_pfb_execute(tina_pfb_plan_t p, const void* d_in, int64_t n, void* d_out, int64_t cap,
                             tina_pfb_state_t st, int64_t* frames_written, void* stream) {
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "execute: NULL plan");
    ExecWorkspace w;
    w.ws = p->ws;
    w.amax = p->amax;
    w.fexp = p->fexp;
    w.ch_frames = p->ch_frames;
    return execute_with(p, d_in, n, d_out, cap, st, frames_written, stream, w, "execute");
}

tina_status tina_pfb_execute_noalloc(tina_pfb_plan_t p, const void* d_in, int64_t n, void* d_out, int64_t cap,
                                     tina_pfb_state_t st, int64_t* frames_written, void* stream) {
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "execute_noalloc: NULL plan");
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return fail(TINA_ERR_DEVICE, "execute_noalloc: hipSetDevice failed");
    hipError_t e;
    void* base = scratch_address(p->device, &e);
    if (!base) return fail(TINA_ERR_DEVICE, std::string("execute_noalloc: scratch address: ") + hipGetErrorString(e));
    return execute_with(p, d_in, n, d_out, cap, st, frames_written, stream,
                        scratch_workspace(p, (uint8_t*)base), "execute_noalloc");
}

tina_status tina_pfb_profile_enable(tina_pfb_plan_t p, int enable) {
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "profile_enable: NULL plan");
    DeviceScope ds(p->device);
    HIP_TRY(hipDeviceSynchronize());
    p->clear_events();
    p->profiling = enable != 0;
    return TINA_OK;
}

tina_status tina_pfb_profile_read(tina_pfb_plan_t p, double* fir_ms, int64_t* fir_n, double* dft_ms, int64_t* dft_n) {
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "profile_read: NULL plan");
    DeviceScope ds(p->device);
    auto sum = [&](const std::vector<std::pair<hipEvent_t, hipEvent_t>>& list, double* ms, int64_t* n) -> tina_status {
        double t = 0.0;
        for (const auto& pr : list) {
            HIP_TRY(hipEventSynchronize(pr.second));
            float x = 0.0f;
            HIP_TRY(hipEventElapsedTime(&x, pr.first, pr.second));
            t += x;
        }
        if (ms) *ms = t;
        if (n) *n = (int64_t)list.size();
        return TINA_OK;
    };
    tina_status st = sum(p->ev_fir, fir_ms, fir_n);
    if (st != TINA_OK) return st;
    return sum(p->ev_dft, dft_ms, dft_n);
}

tina_status tina_pfb_synthesize(tina_pfb_plan_t p, const void* d_X, int64_t F, void* d_out, int64_t cap,
                                tina_pfb_state_t st, int64_t* written, void* stream) {
    if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: NULL plan");
    if (p->output != TINA_OUT_INVERSE) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: not a synthesis plan");
    if (F < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: negative frame count");
    if (F > 0 && (!d_X || !d_out)) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: NULL buffer");
    if (st && st->plan != p) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: state belongs to another plan");
    if ((uintptr_t)d_X % 16 || (uintptr_t)d_out % 8)
        return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: d_X must be 16-byte and d_out 8-byte aligned");
    if (F * p->P > cap) return fail(TINA_ERR_INVALID_ARGUMENT, "synthesize: output capacity below frames * P samples");
    if (p->ch_frames == 0) return fail(TINA_ERR_UNSUPPORTED, "synthesize: plan was created without a workspace");
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return fail(TINA_ERR_DEVICE, "synthesize: hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(p->order.begin(s));
    if (st && F > 0) st->plan_ordered = false;  // until this call's work is covered by the order event
    const int64_t hist_floats = (int64_t)(p->M - 1) * p->W;
    const float* prefix = st ? st->buf[st->cur] : nullptr;
    int scratch = 0;
    for (int64_t c0 = 0; c0 < F; c0 += p->ch_frames) {
        const int64_t Fc = F - c0 < p->ch_frames ? F - c0 : p->ch_frames;
        GemmArgs ga{};  // inverse DFT of the frames into the workspace
        ga.A = (const float*)d_X + c0 * p->W;
        ga.lda = p->W;
        ga.B0 = p->B[0];
        ga.B1 = p->B[1];
        ga.out = p->ws;
        ga.ldo = p->W;
        ga.F = Fc;
        ga.K = p->K;
        ga.N = p->N;
        ga.real_pack = 0;
        ga.form = p->precision;
        HIP_TRY(launch_dft_gemm(ga, s));
        FirArgs fa{};  // synthesis FIR across frames
        fa.prefix = prefix;
        fa.plen = hist_floats;
        fa.chunk = p->ws;
        fa.nchunk = Fc * p->W;
        fa.taps = p->g32;
        fa.y = (float*)d_out + c0 * p->W;
        fa.ldy = p->W;
        fa.g0 = 0;
        fa.F = Fc;
        fa.W = p->W;
        fa.P = p->P;
        fa.M = p->M;
        fa.cf = p->cf;
        HIP_TRY(launch_fir(fa, s));
        // History for the next piece (or the state): the last M-1 frames of prefix ++ workspace.
        const bool last = c0 + Fc >= F;
        if (last && !st) break;
        float* dst = last ? st->buf[st->cur ^ 1] : p->hist[scratch];
        HIP_TRY(launch_gather_ext(prefix, hist_floats, p->ws, Fc * p->W, dst, Fc * p->W, hist_floats, s));
        prefix = dst;
        scratch ^= 1;
    }
    if (st && F > 0) st->cur ^= 1;
    HIP_TRY(p->order.end(s));
    if (st && F > 0) st->plan_ordered = p->order.valid;
    if (written) *written = F * p->P;
    return TINA_OK;
}

tina_status tina_pfb_state_create(tina_pfb_plan_t p, tina_pfb_state_t* out) {
    if (!p || !out) return fail(TINA_ERR_INVALID_ARGUMENT, "state_create: NULL argument");
    *out = nullptr;
    DeviceScope ds(p->device);
    tina_pfb_state_s* st = new (std::nothrow) tina_pfb_state_s();
    if (!st) return fail(TINA_ERR_OUT_OF_MEMORY, "state_create: host allocation");
    st->plan = p;
    st->cap_floats = (int64_t)p->M * p->W;  // (M-1)*W history + up to W residue floats
    for (int i = 0; i < 2; ++i) {
        if (hipMalloc(&st->buf[i], st->cap_floats * sizeof(float)) != hipSuccess ||
            hipMemset(st->buf[i], 0, st->cap_floats * sizeof(float)) != hipSuccess) {
            for (float* b : st->buf)
                if (b) (void)hipFree(b);
            delete st;
            return fail(TINA_ERR_OUT_OF_MEMORY, "state_create: device allocation");
        }
    }
    *out = st;
    return TINA_OK;
}

// Waits until no enqueued work reads or writes the state's buffers.  Calls
// of one plan are ordered across streams (each starts after the previous one
// ends), so after an update by a plan call that the plan's stream-order event
// covers, the plan's latest event is enough; otherwise (batch, allocation-free
// or captured calls, or none yet) the whole device is waited for.
static hipError_t wait_for_state(const tina_pfb_state_s* st) {
    const tina_pfb_plan_s* p = st->plan;
    if (st->plan_ordered && p->order.valid) return hipEventSynchronize(p->order.ev);
    return hipDeviceSynchronize();
}

tina_status tina_pfb_state_destroy(tina_pfb_state_t st) {
    if (!st) return TINA_OK;
    DeviceScope ds(st->plan->device);
    (void)hipDeviceSynchronize();
    for (float* b : st->buf)
        if (b) (void)hipFree(b);
    delete st;
    return TINA_OK;
}

tina_status tina_pfb_state_reset(tina_pfb_state_t st) {
    if (!st) return fail(TINA_ERR_INVALID_ARGUMENT, "state_reset: NULL state");
    DeviceScope ds(st->plan->device);
    HIP_TRY(wait_for_state(st));
    for (float* b : st->buf) HIP_TRY(hipMemset(b, 0, st->cap_floats * sizeof(float)));
    st->cur = 0;
    st->residue = 0;
    return TINA_OK;
}

tina_status tina_pfb_state_size(tina_pfb_state_t st, int64_t* n, int64_t* residue) {
    if (!st) return fail(TINA_ERR_INVALID_ARGUMENT, "state_size: NULL state");
    const tina_pfb_plan_s* p = st->plan;
    if (n) *n = (int64_t)(p->M - 1) * p->P + st->residue;
    if (residue) *residue = st->residue;
    return TINA_OK;
}

tina_status tina_pfb_state_export(tina_pfb_state_t st, void* host, int64_t capacity, int64_t* n_samples) {
    if (!st || !host) return fail(TINA_ERR_INVALID_ARGUMENT, "state_export: NULL argument");
    const tina_pfb_plan_s* p = st->plan;
    const int64_t n = (int64_t)(p->M - 1) * p->P + st->residue;
    if (capacity < n) return fail(TINA_ERR_INVALID_ARGUMENT, "state_export: host buffer too small");
    DeviceScope ds(p->device);
    HIP_TRY(wait_for_state(st));
    if (n > 0) HIP_TRY(hipMemcpy(host, st->buf[st->cur], n * p->cf * sizeof(float), hipMemcpyDeviceToHost));
    if (n_samples) *n_samples = n;
    return TINA_OK;
}

tina_status tina_pfb_state_import(tina_pfb_state_t st, const void* host, int64_t n) {
    if (!st || (!host && n > 0)) return fail(TINA_ERR_INVALID_ARGUMENT, "state_import: NULL argument");
    const tina_pfb_plan_s* p = st->plan;
    const int64_t hist = (int64_t)(p->M - 1) * p->P;
    if (n < hist || n - hist >= p->P) return fail(TINA_ERR_INVALID_ARGUMENT, "state_import: sample count must be (M-1)*P + residue, residue < P");
    DeviceScope ds(p->device);
    HIP_TRY(wait_for_state(st));
    if (n > 0) HIP_TRY(hipMemcpy(st->buf[0], host, n * p->cf * sizeof(float), hipMemcpyHostToDevice));
    st->cur = 0;
    st->residue = n - hist;
    return TINA_OK;
}

}  // extern "C"
