/*
 * tina_pfb_batch.h -- batched filter-bank execution (C ABI).
 *
 * Runs the filter bank of Sec. 5.2, Eq. (20) of the TINA paper (arXiv
 * 2408.16551) on many independent stream chunks at once: each chunk has its
 * own plan (channels P, taps M, window, sample type; all plans in a batch use
 * the batch's DFT precision) and optionally its own per-stream state.  The
 * whole batch runs as one persistent launch per stage (FIR, DFT GEMM, state
 * update), reading a table of items uploaded to the device on the caller's
 * stream, so the work of short and long chunks, and of different channel
 * counts, is spread over all compute units in a single pass.
 *
 * The same conventions as tina_pfb.h hold: tina_status results, messages via
 * tina_last_error(), validation before any work is enqueued, device pointers
 * for sample data, asynchronous execution on `stream`.
 */
#ifndef TINA_PFB_BATCH_H
#define TINA_PFB_BATCH_H

#include <stdint.h>

#include "tina_pfb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tina_pfb_batch_s* tina_pfb_batch_t;

/* One stream chunk of a batch.  plan: a TINA_OUT_PFB plan on the batch's
 * device with the batch's precision, taking the dense DFT or (FP32) the
 * factored one: the factored items' DFTs run as one launch per channel
 * count and input type instead of the GEMM stage, and a batch may mix both
 * (fused or compensated plans: UNSUPPORTED).  state: NULL (zero history, nothing
 * retained) or a state of that plan; a state may appear only once per batch.
 * d_in: n_samples samples (device, aligned to the sample size).  d_out: room
 * for out_capacity_frames output rows (device, 8-byte aligned), row layout as
 * tina_pfb_execute.  frames_written is set when the call returns TINA_OK. */
typedef struct tina_pfb_work {
    tina_pfb_plan_t plan;
    tina_pfb_state_t state;
    const void* d_in;
    int64_t n_samples;
    void* d_out;
    int64_t out_capacity_frames;
    int64_t frames_written;
} tina_pfb_work;

/* Create a batch context on `device` for DFT precision `precision`
 * (tina_precision), holding up to max_items items per call and a device
 * workspace of workspace_bytes for the FIR output of the items (a call whose
 * items need more runs them as consecutive groups; one item that alone needs
 * more is rejected with TINA_ERR_TOO_LARGE).  The context owns the
 * workspace, a device item table and a pinned host copy of it. */
tina_status tina_pfb_batch_create(int device, int precision, int max_items, int64_t workspace_bytes,
                                  tina_pfb_batch_t* out_batch);

/* Release a batch context (synchronises its device first).  NULL is accepted. */
tina_status tina_pfb_batch_destroy(tina_pfb_batch_t batch);

/* Enqueue the filter bank of n items on `stream`.  Each item's result equals
 * tina_pfb_execute of that item alone (the same kernels and arithmetic per
 * output element).  States are updated as in tina_pfb_execute.  The call may
 * wait on the host for the previous call's table upload to finish before it
 * reuses the pinned table. */
tina_status tina_pfb_batch_execute(tina_pfb_batch_t batch, tina_pfb_work* items, int32_t n, void* stream);

/* Autotune the launch shapes (frames per FIR thread as a multiple of the tap
 * ring; GEMM tile columns, 128 or 256 -- 256 is tried for FP32) on this
 * batch's shape by timing each
 * candidate on the device, without writing any state; the choice is cached
 * under a signature of the shape (precision, total samples rounded to a
 * power of two, distinct (P, M, sample type)) for later
 * tina_pfb_batch_execute calls, and stored in the file named by the
 * TINA_TUNE_CACHE environment variable when it is set.  Writes the outputs of
 * the items (repeatedly).  Synchronous.  The chosen values are returned
 * through the two pointers when they are not NULL. */
tina_status tina_pfb_batch_tune(tina_pfb_batch_t batch, tina_pfb_work* items, int32_t n, void* stream,
                                int32_t* fir_tf_mult, int32_t* gemm_tile_n);

/* Host-only helper used to plan the persistent launches (exposed for
 * testing): split the units of one stage, given per item as units[i] units
 * of cost cost[i] each, into 8 contiguous ranges of about equal total cost,
 * one per XCD.  bounds9[x]..bounds9[x+1] is range x; bounds9[0] = 0 and
 * bounds9[8] = the total unit count.  No device work. */
tina_status tina_pfb_batch_split_units(const int64_t* units, const double* cost, int32_t n, int64_t* bounds9);

#ifdef __cplusplus
}
#endif
#endif /* TINA_PFB_BATCH_H */
