/*
 * tina_pfb_server.h -- continuous-batching channelizer server (C ABI).
 *
 * Serves filter-bank requests (TINA, arXiv 2408.16551, Sec. 5.2, Eq. (20))
 * on many logical streams.  Each logical stream has its own channel count,
 * taps, window and a device-resident filter state (the last (M-1)*P samples
 * and the partial-frame residue), so consecutive requests of a stream are
 * consecutive chunks of one signal: the concatenated outputs equal the
 * filter bank of the concatenated inputs.
 *
 * A server thread runs steps back to back, building and enqueuing the next
 * step while the previous one is still on the device.  Requests queue in arrival order
 * and are admitted while a slot is free and their device buffers (input and
 * output) fit the HBM budget.  A request holds its slot, and its stream's
 * turn, until its last samples are in a step: the stream's next request may
 * then take the following step while the earlier one waits for its steps to
 * complete.  A stream's chunks are processed, and its requests complete, in
 * order.  A step that fails ends its requests and every later admitted
 * request of their streams.
 * Each step gives every admitted request whose input has reached the device
 * up to `frames_per_step` frames of work (times max_active / ready requests,
 * rounded down, when fewer than max_active are ready: the step workspace is
 * shared) and runs them together as one
 * batched launch per stage (tina_pfb_batch.h), optionally replayed from a
 * captured HIP graph, so requests that arrive while others run join at the
 * next step and their work overlaps on the device.  Input copies to the
 * device and output copies back run on two more HIP streams, so both
 * directions of the host link are used at once, beside the compute.
 *
 * Same conventions as tina_pfb.h: tina_status results, tina_last_error(),
 * validation before anything is queued.  All calls are thread-safe.
 */
#ifndef TINA_PFB_SERVER_H
#define TINA_PFB_SERVER_H

#include <stdint.h>

#include "tina_pfb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tina_server_s* tina_server_t;

typedef struct tina_server_config {
    uint32_t struct_size;      /* sizeof(tina_server_config) */
    int32_t device;            /* HIP device ordinal */
    int32_t precision;         /* tina_precision of every stream's DFT */
    int32_t max_streams;       /* logical streams, >= 1 */
    int32_t max_active;        /* requests admitted at once (slots), >= 1 */
    int32_t max_queued;        /* requests waiting for admission; submit returns BUSY beyond */
    int64_t hbm_budget_bytes;  /* device arena for request input and output buffers */
    int64_t frames_per_step;   /* frames of work per request per step with every slot busy, >= 1 */
    int32_t use_graph;         /* nonzero: each step replays a captured HIP graph (every
                                  variant captured at creation); zero: plain launches (every
                                  kernel variant launched once at creation).  A replay leaves
                                  the device ~8 us longer idle between two steps; plain
                                  launches cost more host time per step, which overlaps the
                                  step in flight */
    int32_t max_channels;      /* largest P any stream will use (sizes the step workspace) */
    int32_t dft_algorithm;     /* tina_dft_algorithm of every stream: TINA_DFT_DENSE, or
                                  TINA_DFT_FACTORED with precision FP32 (stream P then in
                                  [256, 4096]; steps run as plain launches).  Configurations
                                  whose struct_size ends before this field: DENSE */
    int32_t reserved_;         /* must be 0 */
} tina_server_config;

/* Create a server and start its thread.  The server owns the arena
 * (hbm_budget_bytes), a batch context and its step workspace
 * (max_active * frames_per_step * 2 * max_channels floats), and three HIP
 * streams (compute, host-to-device copies, device-to-host copies), all at the
 * default priority.  Errors: INVALID_ARGUMENT, OUT_OF_MEMORY, DEVICE. */
tina_status tina_server_create(const tina_server_config* cfg, tina_server_t* out_server);

/* Stop the thread after the admitted requests finish, fail the queued ones
 * with TINA_ERR_CANCELLED, and release everything.  NULL is accepted. */
tina_status tina_server_destroy(tina_server_t server);

/* Register a logical stream with P channels (power of two, 16..max_channels),
 * M taps (1..64), a sample type and a window (not CUSTOM).  Plans are shared
 * between streams with the same parameters; each stream owns its state
 * (2 * M * P samples of device memory, outside the arena).  Returns its id. */
tina_status tina_server_stream_create(tina_server_t server, int32_t channels, int32_t taps, int32_t sample_type,
                                      int32_t window, int32_t* stream_id);

/* One request: the next n_samples samples of stream `stream_id`, read from
 * host_in (host memory; pinned memory makes the copy asynchronous), the
 * output rows written to host_out (host memory, room for
 * out_capacity_frames rows of the stream's output, layout as
 * tina_pfb_execute).  Both buffers are lent to the server until the request
 * is reported done.
 *
 * flags: TINA_REQ_DEVICE_BUFFERS -- host_in and host_out are device memory
 * on the server's device (the caller's; 4-byte aligned input, 8-byte aligned
 * output): the steps read and write them in place, no copy is made and the
 * arena (hbm_budget_bytes) is not used, so admission waits only for a slot.
 * The input may still be being written when submit is called: submit records
 * an event on ready_stream (a hipStream_t; NULL is the default stream), and
 * the request joins no step before the work enqueued there so far is done.
 * ready_stream is ignored for host buffers. */
#define TINA_REQ_DEVICE_BUFFERS 1
typedef struct tina_request {
    int32_t stream_id;
    int32_t flags;             /* 0 or TINA_REQ_DEVICE_BUFFERS */
    const void* host_in;
    int64_t n_samples;
    void* host_out;
    int64_t out_capacity_frames;
    void* ready_stream;        /* TINA_REQ_DEVICE_BUFFERS: stream that writes host_in */
} tina_request;

typedef struct tina_result {
    int32_t status;            /* TINA_OK, or the error that ended the request */
    int32_t pad_;
    int64_t frames;            /* output rows written to host_out */
    double t_submit_us;        /* server clock (microseconds since server creation) */
    double t_admit_us;         /* admitted: arena allocated, input copy queued */
    double t_first_step_us;    /* first step containing this request was launched */
    double t_done_us;          /* output copied back to host_out */
    int32_t steps;             /* steps the request took part in */
    int32_t pad2_;
} tina_result;

/* Queue a request.  Errors (nothing queued): INVALID_ARGUMENT (bad stream
 * id, NULL buffers, output capacity below the frame count this request
 * completes), TOO_LARGE (its buffers can never fit the budget), BUSY (the
 * queue is full), CANCELLED (the server is stopping). */
tina_status tina_pfb_submit(tina_server_t server, const tina_request* req, uint64_t* request_id);

/* Result of a request: TINA_ERR_NOT_READY while it runs; otherwise TINA_OK
 * with *result filled (the request is then forgotten; a later poll of the
 * same id returns INVALID_ARGUMENT). */
tina_status tina_pfb_poll(tina_server_t server, uint64_t request_id, tina_result* result);

/* As tina_pfb_poll, but waits up to timeout_us microseconds (negative:
 * forever); TINA_ERR_TIMEOUT when it runs out. */
tina_status tina_pfb_wait(tina_server_t server, uint64_t request_id, int64_t timeout_us, tina_result* result);

/* Cancel a request that has not been admitted yet (TINA_OK), or report
 * NOT_READY if it is already running (it then completes normally). */
tina_status tina_pfb_cancel(tina_server_t server, uint64_t request_id);

typedef struct tina_server_stats {
    int64_t steps;             /* steps launched */
    int64_t samples;           /* input samples processed */
    int64_t frames;            /* output frames produced */
    int64_t completed;         /* requests completed */
    int64_t admitted;          /* requests admitted */
    int64_t admission_waits;   /* times the queue head waited for arena memory */
    double device_busy_ms;     /* summed step durations (HIP events) */
    double now_us;             /* server clock */
    int64_t arena_in_use;      /* bytes currently allocated in the arena */
    int64_t arena_high_water;  /* largest arena use so far */
} tina_server_stats;

tina_status tina_server_get_stats(tina_server_t server, tina_server_stats* stats);

/* Host-only check of the server's arena allocator (first fit, 256-byte
 * granules, coalescing on release), exposed for tests; no device work.
 * ops[i] > 0 allocates ops[i] bytes: out[i] = offset, or -1 if it does not
 * fit.  ops[i] <= 0 releases the allocation made by operation -ops[i]:
 * out[i] = 1 if released, else 0.  *final_used = bytes allocated at the end. */
tina_status tina_server_arena_simulate(int64_t capacity, const int64_t* ops, int32_t n, int64_t* out,
                                       int64_t* final_used);

/* Host-only run of the server's scheduler on a scripted sequence of
 * operations, exposed for tests; no device work.  The decisions are those of
 * the running server: admission in arrival order while a slot is free and the
 * buffers fit the arena (a slot and the stream's turn are held until the
 * request's last samples are in a step; a request that does not fit blocks
 * the ones behind it), per-step quotas (frames_per_step
 * times max(1, max_active / ready requests) frames per request), cancellation
 * of the newest queued request of a stream, steps completing or failing in
 * order.  Requests are complex64 (8 bytes per sample and per output value).
 *
 * ops[i].kind and its fields:
 *   ADD_STREAM  arg = channels P                 -> event (ADD_STREAM, id = stream id, a = P)
 *   SUBMIT      arg = stream id, value = samples (negative: device buffers,
 *               -value samples, no arena)         -> event (SUBMIT, status, id (0 if refused),
 *                                                    a = samples, b = frames of the request)
 *   ADMIT       run admission                      -> one event (ADMIT, id, a = arena offset of
 *                                                    the input, b = of the output; -1 for device)
 *   READY       value = request id: its input copy completed (device-buffer
 *               requests are ready on admission)   -> event (READY, status)
 *   STEP        complete admitted empty requests, then build a step and put
 *               it in flight                       -> (COMPLETE ...) for empty requests, one
 *                                                    event (STEP, id, a = samples, b = frames)
 *                                                    per item, then (STEP, id = 0, a = items,
 *                                                    b = steps in flight)
 *   COMPLETE    arg = TINA_OK or the status the oldest in-flight step fails
 *               with                               -> (COMPLETE, status, id, a = frames done,
 *                                                    b = steps) for every request it ends
 *   CANCEL      value = request id                 -> event (CANCEL, status: OK, NOT_READY
 *                                                    (already admitted) or INVALID_ARGUMENT)
 * Up to `capacity` events are written; *n_events receives the number there
 * were (TOO_LARGE if more than capacity). */
enum {
    TINA_SCHED_ADD_STREAM = 1, TINA_SCHED_SUBMIT = 2, TINA_SCHED_ADMIT = 3, TINA_SCHED_READY = 4,
    TINA_SCHED_STEP = 5, TINA_SCHED_COMPLETE = 6, TINA_SCHED_CANCEL = 7
};
typedef struct tina_sched_op {
    int32_t kind;
    int32_t arg;
    int64_t value;
} tina_sched_op;
typedef struct tina_sched_event {
    int32_t kind;
    int32_t status;
    uint64_t id;
    int64_t a, b;
} tina_sched_event;
tina_status tina_server_schedule_simulate(int32_t max_active, int32_t max_queued, int64_t frames_per_step,
                                          int64_t arena_bytes, const tina_sched_op* ops, int32_t n_ops,
                                          tina_sched_event* events, int32_t capacity, int32_t* n_events);

#ifdef __cplusplus
}
#endif
#endif /* TINA_PFB_SERVER_H */
