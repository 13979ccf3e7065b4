/*
 * tina_pfb.h -- C ABI of the MI355X (gfx950) polyphase filter bank channelizer.
 *
 * The filter bank follows the TINA paper (arXiv 2408.16551), Sec. 5.2,
 * Eq. (20): an input stream x(n) is split into P branches x_p(n'), each branch
 * is filtered by its share h_p of the prototype filter taps,
 *     y_p(n') = sum_{m=0}^{M-1} h_p(m) x_p(n'-m),
 * and each frame of branch outputs goes through a DFT across the P branches
 * (Sec. 4.1, Eq. (12): Z = X F, F the Fourier matrix).  Readings used where
 * the paper is silent:
 *   - branch p of frame f is sample f*P + p of the stream;
 *   - h_p(m) = h[(M-1-m)*P + p] for a prototype h of length L = P*M;
 *   - the DFT is forward and unnormalised, X[k] = sum_p y[p] exp(-2 pi i p k/P);
 *   - a real stream yields channels k = 0..P/2, a complex stream k = 0..P-1.
 *
 * Conventions for every call:
 *   - The return value is a tina_status; TINA_OK is 0.  On failure a message
 *     is available from tina_last_error() (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   - Arguments are validated before any work is enqueued, so a call that
 *     fails validation has not written to any output.
 *   - "Device pointer" means memory the caller allocated on the plan's HIP
 *     device (hipMalloc, or a torch tensor's data_ptr()).  The library never
 *     frees caller memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Device work is asynchronous on that stream unless stated otherwise.
 *   - Sizes are int64_t counts of samples or frames, never bytes, unless the
 *     name says _bytes.
 *   - A plan (and a batch context) owns device scratch that every call of it
 *     uses: the workspace between the FIR and the DFT, per-frame scales,
 *     argument tables.  Calls of one plan on different streams are therefore
 *     ordered by the library: a call on another stream than the previous
 *     call's first waits (hipStreamWaitEvent) for that call's work.  Calls
 *     captured into a graph are not ordered this way; the capturing caller
 *     orders the graph's launches.  Plans, states and batch contexts are
 *     thread-compatible, not thread-safe: one host thread calls an object at
 *     a time.
 */
#ifndef TINA_PFB_H
#define TINA_PFB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tina_status {
    TINA_OK = 0,
    TINA_ERR_INVALID_ARGUMENT = 1, /* a NULL handle/pointer, a bad size or alignment */
    TINA_ERR_UNSUPPORTED = 2,      /* valid request the library does not implement */
    TINA_ERR_OUT_OF_MEMORY = 3,    /* a device or host allocation failed */
    TINA_ERR_DEVICE = 4,           /* a HIP runtime call failed */
    TINA_ERR_BUSY = 5,             /* a queue is full; retry later */
    TINA_ERR_NOT_READY = 6,        /* the result is not complete yet */
    TINA_ERR_TOO_LARGE = 7,        /* the request can never fit the configured budget */
    TINA_ERR_TIMEOUT = 8,          /* a wait ran out of time */
    TINA_ERR_CANCELLED = 9         /* the request was cancelled or its server stopped */
} tina_status;

typedef enum tina_sample_type {
    TINA_SAMPLE_R32 = 0, /* real float32 samples */
    TINA_SAMPLE_C64 = 1  /* complex64 samples: interleaved float32 re, im */
} tina_sample_type;

/* Prototype window.  The prototype is h[n] = sinc((n - (L-1)/2) / P) * w[n],
 * n = 0..L-1, L = P*M, sinc(t) = sin(pi t)/(pi t), with a symmetric window w
 * over L points: rect 1; Hann 0.5 - 0.5 cos(2 pi n/(L-1));
 * Hamming 0.54 - 0.46 cos(2 pi n/(L-1));
 * Blackman 0.42 - 0.5 cos(2 pi n/(L-1)) + 0.08 cos(4 pi n/(L-1)).
 * No normalisation.  CUSTOM takes h from the descriptor instead. */
typedef enum tina_window {
    TINA_WINDOW_RECT = 0,
    TINA_WINDOW_HANN = 1,
    TINA_WINDOW_HAMMING = 2,
    TINA_WINDOW_BLACKMAN = 3,
    TINA_WINDOW_CUSTOM = 4
} tina_window;

/* Arithmetic of the DFT stage (a matrix product on the MFMA units, FP32
 * accumulation).  The FIR stage computes in FP32 in every form.
 *   FP32       plain FP32 operands.
 *   BF16       operands rounded to bfloat16.
 *   BF16X3     operands split into bfloat16 hi + lo pieces, three products
 *              (hi*hi + hi*lo + lo*hi).
 *   FP16       operands rounded to float16, each frame scaled by a power of
 *              two so that its largest branch output fits the format.
 *   FP16X3     float16 hi + lo pieces (lo scaled by 2^11), three products,
 *              same per-frame power-of-two scale.
 *   FP8_FRAME  operands in FP8 E4M3 (OCP), each frame scaled by a power of two
 *              so that its largest branch output maps to at most 448.
 *   MXFP8      block-scaled FP8 (quantisation, Sec. 1): operands in E4M3 with
 *              one power-of-two scale per 32 consecutive entries along the
 *              summed axis (a frame's branch values, re/im interleaved for
 *              complex input; a DFT coefficient row), the smallest with
 *              max|v| <= 448 * scale; rounding to nearest even.  The FIR
 *              writes this form directly (1 byte per value plus 1 per 32),
 *              and the matrix units apply the scales.  Needs channels a
 *              multiple of 128 (real) or 64 (complex). */
typedef enum tina_precision {
    TINA_PREC_FP32 = 0,
    TINA_PREC_BF16 = 1,
    TINA_PREC_BF16X3 = 2,
    TINA_PREC_FP16 = 3,
    TINA_PREC_FP16X3 = 4,
    TINA_PREC_FP8_FRAME = 5,
    TINA_PREC_MXFP8 = 6
} tina_precision;

typedef enum tina_output {
    TINA_OUT_PFB = 0,      /* channelizer output: frames x K complex64 */
    TINA_OUT_FIR_ONLY = 1, /* polyphase FIR output only: frames x P samples of the input type */
    TINA_OUT_INVERSE = 2   /* synthesis bank (tina_pfb_synthesize): channel frames -> samples;
                              complex64 only, precision FP32, BF16 or BF16X3, dense DFT */
} tina_output;

typedef struct tina_pfb_desc {
    uint32_t struct_size;      /* sizeof(tina_pfb_desc) */
    int32_t channels;          /* P: power of two, 16 <= P <= 8192 */
    int32_t taps;              /* M: taps per branch, 1 <= M <= 64 */
    int32_t sample_type;       /* tina_sample_type */
    int32_t window;            /* tina_window */
    int32_t precision;         /* tina_precision (ignored for TINA_OUT_FIR_ONLY) */
    int32_t output;            /* tina_output */
    int32_t device;            /* HIP device ordinal */
    const double* custom_taps; /* host, P*M doubles, read during tina_pfb_plan when
                                  window == TINA_WINDOW_CUSTOM; otherwise NULL */
    int64_t workspace_bytes;   /* FIR workspace of tina_pfb_execute: 0 = default (512 MiB),
                                  < 0 = none (the plan is used only through batches or a
                                  server, and tina_pfb_execute returns UNSUPPORTED).
                                  Descriptors whose struct_size ends before this field
                                  get the default. */
    int32_t dft_algorithm;     /* tina_dft_algorithm (descriptors ending before this field:
                                  TINA_DFT_DENSE) */
    int32_t reserved_;         /* must be 0 */
} tina_pfb_desc;

/* How the DFT across branches is computed (both give the DFT of Eq. (12)):
 *   TINA_DFT_DENSE     the dense matrix product X = Y F on the MFMA units, in the
 *                      plan's precision (the paper's pointwise-convolution mapping);
 *   TINA_DFT_FACTORED  a factored (four-step) DFT, P = P1 * P2: P2 DFTs of size
 *                      P1, twiddles, P1 DFTs of size P2, each size-P1/P2 DFT a
 *                      small matrix product on the MFMA units in FP32 -- 8 P (P1 + P2)
 *                      flops per frame instead of 8 P^2.  FP32 only; 256 <= P <= 4096.
 *                      Also in FP32 batches (one launch per channel count and
 *                      input type over those items' frames) and in an FP32
 *                      server created with this algorithm.
 *   TINA_DFT_FUSED     the dense product with the polyphase FIR fused into it:
 *                      each matrix-product tile forms its rows of FIR output
 *                      from the input stream in on-chip memory (a sliding
 *                      window over the frames staged in LDS), so the FIR output
 *                      never goes to HBM.  Results are bit for bit those of
 *                      TINA_DFT_DENSE.  FP32, taps <= 16, single-stream
 *                      execute; a call whose input is not 16-byte aligned (or
 *                      whose residue leaves the history a partial float4) runs
 *                      the two-kernel path instead.
 *   TINA_DFT_COMPENSATED the dense FP32 product with compensated accumulation
 *                      over K: each K tile of 32 products is summed on its
 *                      own, and the tile sums are added to the running sum
 *                      with an error-free two-sum whose rounding error is
 *                      carried into the next tile.  The error of a channel
 *                      then scales with the partial sums of one tile instead
 *                      of the whole row, which keeps channels far below the
 *                      frame's strongest one accurate (Eq. (12) at a wide
 *                      dynamic range).  FP32 only; single-stream execute.
 *   TINA_DFT_TABLE     the dense FP32 product with the operand F of Eq. (12)
 *                      never materialised: each matrix-product tile assembles
 *                      its operand rows in on-chip memory from a P-entry
 *                      twiddle table (cos, sin of 2 pi r / P, r = p k mod P),
 *                      8 P bytes instead of the N x K operand (256 MiB at
 *                      P = 4096 complex).  Same entries, so results are bit
 *                      for bit those of TINA_DFT_DENSE.  FP32 only;
 *                      single-stream execute. */
typedef enum tina_dft_algorithm {
    TINA_DFT_DENSE = 0,
    TINA_DFT_FACTORED = 1,
    TINA_DFT_FUSED = 2,
    TINA_DFT_COMPENSATED = 3,
    TINA_DFT_TABLE = 4
} tina_dft_algorithm;

typedef struct tina_pfb_plan_s* tina_pfb_plan_t;
typedef struct tina_pfb_state_s* tina_pfb_state_t;

/* Last error message of the calling thread ("" if none). */
const char* tina_last_error(void);

/* Library version string. */
const char* tina_version(void);

/*
 * Create a plan: designs the prototype window and the DFT operand (the
 * Fourier matrix of Sec. 4.1 in the operand form of the chosen precision) on
 * the device in FP64, then rounds them to the forms the kernels use.  The
 * plan owns all of its device memory, including an FP32 workspace for the
 * FIR output (desc->workspace_bytes, default 512 MiB; execute runs inputs
 * with more frames than it holds as consecutive pieces), and synchronises
 * once before returning.
 * Errors: INVALID_ARGUMENT (bad descriptor), UNSUPPORTED (P or M outside the
 * ranges above), OUT_OF_MEMORY, DEVICE.
 */
tina_status tina_pfb_plan(const tina_pfb_desc* desc, tina_pfb_plan_t* out_plan);

/* Release a plan and its device memory (synchronises its device first).
 * NULL is accepted. */
tina_status tina_pfb_plan_destroy(tina_pfb_plan_t plan);

/* Number of output channels per frame: P/2+1 (real input) or P (complex), or
 * P for TINA_OUT_FIR_ONLY. */
tina_status tina_pfb_channels_out(tina_pfb_plan_t plan, int64_t* channels);

/* Copy the plan's FP64 prototype taps h[0..P*M) to host memory (P*M
 * doubles).  Synchronous. */
tina_status tina_pfb_plan_taps(tina_pfb_plan_t plan, double* host_taps);

/* Frames that tina_pfb_execute will produce for n_samples new samples:
 * floor((r + n_samples)/P) where r is the state's residue (0 without state). */
tina_status tina_pfb_output_frames(tina_pfb_plan_t plan, tina_pfb_state_t state,
                                   int64_t n_samples, int64_t* frames);

/*
 * Run the filter bank on n_samples samples at d_in (device pointer; float32
 * or complex64 per the plan; 4-byte aligned for R32, 8-byte for C64).
 *
 * Without a state (state == NULL) the history before the first sample is
 * zero, frames = floor(n_samples / P), trailing samples that do not fill a
 * frame are ignored, and nothing is retained.  With a state, the stream's
 * last (M-1)*P samples and its partial-frame residue are prepended, the
 * frames completed by this chunk are produced, and the state is updated on
 * `stream` after them (the state must not be used concurrently on another
 * stream).
 *
 * Output at d_out (device pointer, 8-byte aligned), row-major:
 *   TINA_OUT_PFB:      frames x channels_out complex64 (interleaved float32);
 *   TINA_OUT_FIR_ONLY: frames x P samples of the input type.
 * out_capacity_frames is the number of frames d_out can hold; it must be at
 * least the frame count, else INVALID_ARGUMENT and nothing is enqueued.
 * *frames_written (may be NULL) receives the frame count.
 * The call enqueues work on `stream` and returns without synchronising; the
 * caller keeps d_in and d_out alive until that work is complete.
 */
tina_status tina_pfb_execute(tina_pfb_plan_t plan, const void* d_in, int64_t n_samples,
                             void* d_out, int64_t out_capacity_frames,
                             tina_pfb_state_t state, int64_t* frames_written, void* stream);

/*
 * Allocation-free execute, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, validation and results as tina_pfb_execute
 * (the same kernels run: outputs are bit for bit those of tina_pfb_execute),
 * but the FIR output / operand codes and the per-frame scales live in a
 * static 64 MiB device array of the library instead of the plan's workspace,
 * so the plan may be created with workspace_bytes < 0.  The call makes no
 * hipMalloc, hipFree or other allocating call; the array's device address is
 * looked up once per device on the first call there.
 * Limit: one call handles at most floor((64 MiB - s) / bytes_per_frame)
 * frames, rounded down to a multiple of 128 when at least 128, where W is the
 * floats per frame (P for R32, 2P for C64), bytes_per_frame = 4 W, and for
 * the per-frame scaled forms (FP16, FP16X3, FP8_FRAME) bytes_per_frame =
 * 4 W + 4 max(1, W/32) + 4 and s = 512 (else s = 0): 16384 frames for
 * P = 1024 real FP32.  More frames return TINA_ERR_TOO_LARGE before anything
 * is enqueued.  FIR-only plans use no scratch and have no limit.
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (on different streams, or from different threads) race
 * and corrupt each other's output.  Calls are not ordered against the plan's
 * tina_pfb_execute calls (they do not share memory), and are never timed by
 * tina_pfb_profile_*.
 */
tina_status tina_pfb_execute_noalloc(tina_pfb_plan_t plan, const void* d_in, int64_t n_samples,
                                     void* d_out, int64_t out_capacity_frames,
                                     tina_pfb_state_t state, int64_t* frames_written, void* stream);

/*
 * Synthesis (inverse) filter bank of a TINA_OUT_INVERSE plan: for n_frames
 * frames of P complex64 channel values at d_X (device, row-major, 16-byte
 * aligned), the
 * inverse DFT of each frame (Sec. 4.2, Eq. (14): angle +2 pi p k / P, scaled
 * by 1/P) as a matrix product on the MFMA units, then the polyphase FIR of
 * Eq. (20) across frames with synthesis taps g_p(m) = h[m P + p] (each
 * analysis branch filter reversed in time).  Output: n_frames * P complex64
 * samples at d_out (device); out_capacity_samples must be at least that.
 * With a state (created from this plan), the (M-1)*P inverse-DFT samples
 * of the previous call are the history, and the state is updated on
 * `stream`; without one the history is zero.  Asynchronous on `stream`.
 */
tina_status tina_pfb_synthesize(tina_pfb_plan_t plan, const void* d_X, int64_t n_frames, void* d_out,
                                int64_t out_capacity_samples, tina_pfb_state_t state, int64_t* samples_written,
                                void* stream);

/* Per-stream filter state: (M-1)*P history samples plus fewer than P
 * residue samples, in device memory owned by the state.  Created zeroed.
 * The state takes no stream, and calls that update it may have run on any,
 * so reset, export and import first wait for the work that last used it:
 * when that was tina_pfb_execute or tina_pfb_synthesize of its plan outside
 * stream capture, for that plan's latest call (a plan's calls run one after
 * another across streams); after a batch, allocation-free or captured call,
 * or before any call, for all work on the device.  destroy waits for all
 * work on the device. */
tina_status tina_pfb_state_create(tina_pfb_plan_t plan, tina_pfb_state_t* out_state);
tina_status tina_pfb_state_destroy(tina_pfb_state_t state);
/* Zero the history and drop the residue (synchronous). */
tina_status tina_pfb_state_reset(tina_pfb_state_t state);
/* Samples held: (M-1)*P + residue.  Sample size is 4 (R32) or 8 (C64) bytes. */
tina_status tina_pfb_state_size(tina_pfb_state_t state, int64_t* n_samples, int64_t* residue);
/* Copy the state to host memory: (M-1)*P history samples followed by the
 * residue, capacity in samples.  Synchronous. */
tina_status tina_pfb_state_export(tina_pfb_state_t state, void* host_buf, int64_t capacity,
                                  int64_t* n_samples);
/* Load a state exported by a plan with the same P, M and sample type:
 * n_samples = (M-1)*P + residue with 0 <= residue < P.  Synchronous. */
tina_status tina_pfb_state_import(tina_pfb_state_t state, const void* host_buf, int64_t n_samples);

/*
 * Stage timing.  While enabled, tina_pfb_execute records a HIP event before
 * and after each stage's kernel launch on the caller's stream (FIR stage;
 * DFT-GEMM stage).  tina_pfb_profile_read waits for the recorded events and
 * returns the summed kernel durations in milliseconds and the launch counts
 * since the last enable; enabling again clears them.  Timing adds two event
 * records per stage per execute; disable it for production runs.
 */
tina_status tina_pfb_profile_enable(tina_pfb_plan_t plan, int enable);
tina_status tina_pfb_profile_read(tina_pfb_plan_t plan, double* fir_ms, int64_t* fir_launches,
                                  double* dft_ms, int64_t* dft_launches);

#ifdef __cplusplus
}
#endif
#endif /* TINA_PFB_H */
