// Continuous-batching server for the filter bank (see tina_pfb_server.h).
//
// One server thread owns the device work:
//   admit   -- queued requests in arrival order, while a slot is free and the
//              request's device buffers fit the arena; a stream runs one
//              request at a time (its state orders the chunks);
//   copy in -- each admitted request's input goes to its arena buffer on the
//              host-to-device stream;
//   step    -- every admitted request whose input is on the device gets up
//              to frames_per_step frames; all of them run as one batched
//              launch per stage (batch.hip), optionally a graph replay;
//   copy out-- finished requests' output rows go back on the device-to-host
//              stream (the two directions overlap on the link), then their
//              arena buffers are freed and waiters are woken.
// Requests that arrive while a step runs are admitted before the next one.
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_types.h"
#include "scheduler.h"
#include "tina_pfb_batch.h"
#include "tina_pfb_server.h"

using namespace tina;

namespace {

// The server's side of a request: the caller's request and the events of its
// copies.  The scheduler's Request (sched::Request::user) points here.
struct ReqX {
    tina_request r{};
    int64_t sample_bytes = 0, row_bytes = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string fail_msg;  // why a step of this request failed
};

void destroy_reqx(ReqX* x) {
    if (!x) return;
    if (x->ev_in) (void)hipEventDestroy(x->ev_in);
    if (x->ev_out) (void)hipEventDestroy(x->ev_out);
    delete x;
}

ReqX* rx(sched::Request* q) { return static_cast<ReqX*>(q->user); }

// A step enqueued on the compute stream and not yet retired.  eb is recorded
// after its launches.  ea marks its start: recorded before them when the
// device had nothing else in flight, otherwise the previous step's eb (handed
// over when that step retires), so a loaded pipeline carries one marker per
// step instead of two (each costs the device a few microseconds between
// steps).
struct InFlight {
    std::vector<sched::StepItem> items;
    hipEvent_t ea = nullptr, eb = nullptr;
    bool start_at_prev = false;
};

constexpr int kMaxInFlight = 2;  // steps enqueued ahead of the device

}  // namespace

struct tina_server_s {
    tina_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;

    std::unique_ptr<sched::Scheduler> sch;  // every access under mu
    std::vector<tina_pfb_plan_s*> stream_plans;
    std::vector<tina_pfb_state_s*> stream_states;
    std::map<std::string, tina_pfb_plan_s*> plans;
    std::vector<sched::Request*> draining;  // output copies in flight

    uint8_t* arena_base = nullptr;
    tina_pfb_batch_s* batch = nullptr;
    hipStream_t s_comp = nullptr, s_h2d = nullptr, s_d2h = nullptr;  // copies in and out on their own streams
    std::vector<hipEvent_t> ev_pool;  // timing events of retired steps, for reuse
    std::deque<InFlight> inflight;    // loop thread only
    std::chrono::steady_clock::time_point t0;
    double device_busy_ms = 0.0;

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    void loop();
    bool retire(bool block);
    // Streams of requests that failed continue from the residue the scheduler
    // assumes (the whole request consumed); their history is not repaired.
    void resync(const std::vector<sched::Request*>& ended) {
        for (sched::Request* q : ended) stream_states[q->stream]->residue = sch->stream(q->stream).residue_issued;
    }
    void complete(const std::vector<sched::Request*>& done);
    void finish(sched::Request* q, int status) {
        sch->finish(q, status, now_us());
        cv_done.notify_all();
    }
};

// Requests whose samples have all been processed (lock held): device
// buffers are done; host buffers copy their output rows back first.
void tina_server_s::complete(const std::vector<sched::Request*>& done) {
    for (sched::Request* q : done) {
        ReqX* x = rx(q);
        if (q->device) {
            finish(q, TINA_OK);
            continue;
        }
        if (q->frames_done > 0)
            (void)hipMemcpyAsync(x->r.host_out, arena_base + q->off_out, q->frames_done * x->row_bytes,
                                 hipMemcpyDeviceToHost, s_d2h);
        (void)hipEventRecord(x->ev_out, s_d2h);
        draining.push_back(q);
    }
}

// Retires the oldest in-flight step if it has completed (or, with block,
// once it has): its timing, the progress of its requests, and the requests
// it completed.  Returns whether a step was retired.
bool tina_server_s::retire(bool block) {
    if (inflight.empty()) return false;
    InFlight& f = inflight.front();
    hipError_t e = block ? hipEventSynchronize(f.eb) : hipEventQuery(f.eb);
    if (e == hipErrorNotReady) return false;
    float ms = 0.f;
    if (e == hipSuccess && f.ea) (void)hipEventElapsedTime(&ms, f.ea, f.eb);
    std::unique_lock<std::mutex> lk(mu);
    device_busy_ms += ms;
    std::vector<sched::Request*> ended;
    complete(sch->step_done(f.items, e == hipSuccess, TINA_ERR_DEVICE, now_us(), &ended));
    for (sched::Request* q : ended) rx(q)->fail_msg = std::string("step failed on the device: ") + hipGetErrorString(e);
    resync(ended);
    if (f.ea) ev_pool.push_back(f.ea);
    if (inflight.size() > 1 && inflight[1].start_at_prev) inflight[1].ea = f.eb;  // the next step starts where this ended
    else ev_pool.push_back(f.eb);
    inflight.pop_front();
    cv_done.notify_all();
    return true;
}

void tina_server_s::loop() {
    (void)hipSetDevice(cfg.device);
    std::vector<tina_pfb_work> works;
    for (;;) {
        std::vector<sched::Request*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && sch->queued() == 0 && sch->active().empty() && draining.empty() && inflight.empty()) break;
            admitted = sch->admit(now_us());
        }
        for (sched::Request* q : admitted) {  // input copies, outside the lock
            ReqX* x = rx(q);
            if (q->device) continue;  // ev_in was recorded at submit
            if (q->in_bytes > 0 && q->n_samples > 0)
                (void)hipMemcpyAsync(arena_base + q->off_in, x->r.host_in, q->n_samples * x->sample_bytes,
                                     hipMemcpyHostToDevice, s_h2d);
            (void)hipEventRecord(x->ev_in, s_h2d);
        }
        while (retire(false)) {
        }

        // Build and enqueue the next step while up to kMaxInFlight - 1 others
        // are still on the device: the host's step turnaround (table fill,
        // launches) overlaps the device's work.
        bool built = false;
        if ((int)inflight.size() < kMaxInFlight) {
            std::vector<sched::StepItem> items;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (sched::Request* q : sch->active())
                    if (!q->in_ready) q->in_ready = hipEventQuery(rx(q)->ev_in) == hipSuccess;
                (void)hipGetLastError();  // a pending event's query is not an error
                complete(sch->take_empty());
                items = sch->build_step(now_us());
            }
            if (!items.empty()) {
                works.clear();
                for (const sched::StepItem& it : items) {
                    ReqX* x = rx(it.q);
                    const int s = it.q->stream;
                    tina_pfb_work w{};
                    w.plan = stream_plans[s];
                    w.state = stream_states[s];
                    const uint8_t* in0 = it.q->device ? (const uint8_t*)x->r.host_in : arena_base + it.q->off_in;
                    uint8_t* out0 = it.q->device ? (uint8_t*)x->r.host_out : arena_base + it.q->off_out;
                    w.d_in = in0 + it.sample0 * x->sample_bytes;
                    w.n_samples = it.n_samples;
                    w.d_out = out0 + it.frame0 * x->row_bytes;
                    w.out_capacity_frames = it.q->frames_total - it.frame0;
                    works.push_back(w);
                }
                InFlight f;
                f.items = std::move(items);
                f.start_at_prev = !inflight.empty();
                if (!f.start_at_prev) f.ea = take_event();
                f.eb = take_event();
                tina_status st = ((f.ea || f.start_at_prev) && f.eb) ? TINA_OK : TINA_ERR_DEVICE;
                if (st == TINA_OK && f.ea && hipEventRecord(f.ea, s_comp) != hipSuccess) st = TINA_ERR_DEVICE;
                // At most one step is in flight while this one is built, so the
                // step that last used the batch's other host table has retired:
                // its upload is done and no event is needed to reuse the table.
                if (st == TINA_OK)
                    st = batch_run_items(batch, works.data(), (int32_t)works.size(), s_comp, cfg.use_graph != 0);
                if (st == TINA_OK && hipEventRecord(f.eb, s_comp) != hipSuccess) st = TINA_ERR_DEVICE;
                if (st != TINA_OK) {  // nothing of this step may run: fail its requests
                    (void)hipStreamSynchronize(s_comp);
                    const std::string msg = tina_last_error();
                    std::unique_lock<std::mutex> lk(mu);
                    std::vector<sched::Request*> ended;
                    sch->step_done(f.items, false, st, now_us(), &ended);
                    for (sched::Request* q : ended) rx(q)->fail_msg = "step launch failed: " + msg;
                    resync(ended);
                    for (hipEvent_t e : {f.ea, f.eb})
                        if (e) ev_pool.push_back(e);
                    cv_done.notify_all();
                } else {
                    inflight.push_back(std::move(f));
                    built = true;
                }
            }
        }
        // Wait for the device when the pipeline is full, or when nothing new
        // could be built and a step is still running.
        if (!inflight.empty() && ((int)inflight.size() >= kMaxInFlight || !built)) retire(true);
        {
            std::unique_lock<std::mutex> lk(mu);
            for (auto it = draining.begin(); it != draining.end();) {
                sched::Request* q = *it;
                if (hipEventQuery(rx(q)->ev_out) != hipSuccess) { ++it; continue; }
                finish(q, TINA_OK);
                it = draining.erase(it);
            }
            if (!built && inflight.empty() && !stop) cv_work.wait_for(lk, std::chrono::microseconds(100));
        }
    }
}

extern "C" {

tina_status tina_server_create(const tina_server_config* c_in, tina_server_t* out) {
    if (!c_in || !out) return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: NULL argument");
    *out = nullptr;
    // Configurations that end before dft_algorithm take the dense DFT.
    if (c_in->struct_size < offsetof(tina_server_config, dft_algorithm))
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: struct_size too small");
    tina_server_config cfg{};
    memcpy(&cfg, c_in, std::min<size_t>(c_in->struct_size, sizeof(cfg)));
    cfg.struct_size = sizeof(cfg);
    const tina_server_config* c = &cfg;
    if (c->precision < TINA_PREC_FP32 || c->precision > TINA_PREC_MXFP8)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: unknown precision");
    if (c->dft_algorithm != TINA_DFT_DENSE && c->dft_algorithm != TINA_DFT_FACTORED)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: dft_algorithm must be DENSE or FACTORED");
    if (c->reserved_ != 0) return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: reserved_ must be 0");
    if (c->dft_algorithm == TINA_DFT_FACTORED && c->precision != TINA_PREC_FP32)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: the factored DFT is FP32 only");
    if (c->max_streams < 1 || c->max_active < 1 || c->max_queued < 1 || c->frames_per_step < 1 ||
        c->hbm_budget_bytes < 4096)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: max_streams, max_active, max_queued, frames_per_step "
                                               "must be >= 1 and the budget >= 4 KiB");
    if (!is_pow2(c->max_channels) || c->max_channels < 16 || c->max_channels > 8192)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: max_channels must be a power of two in [16, 8192]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: bad device");
    DeviceScope ds(c->device);
    tina_server_s* sv = new (std::nothrow) tina_server_s();
    if (!sv) return fail(TINA_ERR_OUT_OF_MEMORY, "server_create: host allocation");
    sv->cfg = *c;
    sv->t0 = std::chrono::steady_clock::now();
    sv->sch.reset(new (std::nothrow) sched::Scheduler(c->max_active, c->max_queued, c->frames_per_step, c->hbm_budget_bytes));
    auto bail = [&](tina_status st, const std::string& m) {
        if (sv->batch) tina_pfb_batch_destroy(sv->batch);
        if (sv->arena_base) (void)hipFree(sv->arena_base);
        for (hipStream_t s : {sv->s_comp, sv->s_h2d, sv->s_d2h})
            if (s) (void)hipStreamDestroy(s);
        delete sv;
        return fail(st, m);
    };
    if (!sv->sch) return bail(TINA_ERR_OUT_OF_MEMORY, "server_create: host allocation");
    if (hipMalloc(&sv->arena_base, c->hbm_budget_bytes) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "server_create: arena");
    const int64_t ws = (int64_t)c->max_active * c->frames_per_step * 2 * c->max_channels * 4;
    tina_status st = tina_pfb_batch_create(c->device, c->precision, c->max_active, std::max<int64_t>(ws, 1 << 20), &sv->batch);
    if (st != TINA_OK) return bail(st, std::string("server_create: ") + tina_last_error());
    batch_set_server_mode(sv->batch);
    // Largest GEMM tile count of a step: every slot with frames_per_step
    // frames of the widest stream (128 x 128 tiles, N = 2 * max_channels).
    batch_set_graph_bound(sv->batch, (int64_t)c->max_active * ((c->frames_per_step + kGemmBM - 1) / kGemmBM) *
                                         ((2 * (int64_t)c->max_channels + kGemmBN - 1) / kGemmBN));
    if (hipStreamCreateWithFlags(&sv->s_comp, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->s_h2d, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->s_d2h, hipStreamNonBlocking) != hipSuccess)
        return bail(TINA_ERR_DEVICE, "server_create: streams");
    for (int i = 0; i < 2 * kMaxInFlight; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return bail(TINA_ERR_DEVICE, "server_create: events");
        sv->ev_pool.push_back(e);
    }
    // Every step graph now, none while requests run; without graphs, every
    // kernel variant is launched once now.
    st = c->use_graph ? batch_prepare_graphs(sv->batch, sv->s_comp) : batch_warm_kernels(sv->batch, sv->s_comp);
    if (st == TINA_OK && hipStreamSynchronize(sv->s_comp) != hipSuccess) st = TINA_ERR_DEVICE;
    if (st != TINA_OK) return bail(st, std::string("server_create: ") + tina_last_error());
    sv->th = std::thread([sv] { sv->loop(); });
    *out = sv;
    return TINA_OK;
}

tina_status tina_server_destroy(tina_server_t sv) {
    if (!sv) return TINA_OK;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->sch->cancel_all_queued(sv->now_us());  // queued requests are cancelled
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    DeviceScope ds(sv->cfg.device);
    (void)hipDeviceSynchronize();
    for (uint64_t id : sv->sch->ids()) {  // every request the scheduler still holds
        destroy_reqx(rx(sv->sch->find(id)));
        sv->sch->erase(id);
    }
    for (tina_pfb_state_s* st : sv->stream_states) tina_pfb_state_destroy(st);
    for (auto& kv : sv->plans) tina_pfb_plan_destroy(kv.second);
    tina_pfb_batch_destroy(sv->batch);
    (void)hipFree(sv->arena_base);
    (void)hipStreamDestroy(sv->s_comp);
    (void)hipStreamDestroy(sv->s_h2d);
    (void)hipStreamDestroy(sv->s_d2h);
    for (hipEvent_t e : sv->ev_pool) (void)hipEventDestroy(e);
    delete sv;
    return TINA_OK;
}

tina_status tina_server_stream_create(tina_server_t sv, int32_t P, int32_t M, int32_t sample_type, int32_t window,
                                      int32_t* stream_id) {
    if (!sv || !stream_id) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: NULL argument");
    if (window == TINA_WINDOW_CUSTOM) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: custom taps are not supported here");
    if (P > sv->cfg.max_channels) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: channels above the server's max_channels");
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->sch->n_streams() >= sv->cfg.max_streams) return fail(TINA_ERR_BUSY, "stream_create: max_streams reached");
    const std::string key = std::to_string(P) + "/" + std::to_string(M) + "/" + std::to_string(sample_type) + "/" +
                            std::to_string(window);
    tina_pfb_plan_s* plan = nullptr;
    auto it = sv->plans.find(key);
    if (it != sv->plans.end()) {
        plan = it->second;
    } else {
        tina_pfb_desc d{};
        d.struct_size = sizeof(d);
        d.channels = P;
        d.taps = M;
        d.sample_type = sample_type;
        d.window = window;
        d.precision = sv->cfg.precision;
        d.output = TINA_OUT_PFB;
        d.device = sv->cfg.device;
        d.workspace_bytes = -1;  // used through the server's batch only
        d.dft_algorithm = sv->cfg.dft_algorithm;
        tina_status st = tina_pfb_plan(&d, &plan);
        if (st != TINA_OK) return st;
        sv->plans[key] = plan;
    }
    tina_pfb_state_s* state = nullptr;
    tina_status st = tina_pfb_state_create(plan, &state);
    if (st != TINA_OK) return st;
    sv->stream_plans.push_back(plan);
    sv->stream_states.push_back(state);
    *stream_id = sv->sch->add_stream(P);
    return TINA_OK;
}

tina_status tina_pfb_submit(tina_server_t sv, const tina_request* r, uint64_t* id) {
    if (!sv || !r || !id) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: NULL argument");
    const double t = sv->now_us();
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(TINA_ERR_CANCELLED, "submit: server is stopping");
    if (r->stream_id < 0 || r->stream_id >= sv->sch->n_streams()) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: bad stream id");
    if (r->n_samples < 0 || (r->n_samples > 0 && !r->host_in)) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: bad input");
    if (r->flags & ~TINA_REQ_DEVICE_BUFFERS) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: unknown flags");
    const bool dev = (r->flags & TINA_REQ_DEVICE_BUFFERS) != 0;
    if (dev && (((uintptr_t)r->host_in & 3) || ((uintptr_t)r->host_out & 7)))
        return fail(TINA_ERR_INVALID_ARGUMENT, "submit: device buffers misaligned");
    const tina_pfb_plan_s* p = sv->stream_plans[r->stream_id];
    const int64_t frames = sv->sch->frames_if_submitted(r->stream_id, r->n_samples);
    if (frames > 0 && !r->host_out) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: NULL output");
    if (frames > r->out_capacity_frames)
        return fail(TINA_ERR_INVALID_ARGUMENT, "submit: output capacity below the " + std::to_string(frames) + " frames of this request");
    ReqX* x = new (std::nothrow) ReqX();
    if (!x) return fail(TINA_ERR_OUT_OF_MEMORY, "submit: host allocation");
    x->r = *r;
    x->sample_bytes = p->cf * 4;
    x->row_bytes = p->kout * 8;
    if (hipEventCreateWithFlags(&x->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&x->ev_out, hipEventDisableTiming) != hipSuccess) {
        destroy_reqx(x);
        return fail(TINA_ERR_DEVICE, "submit: events");
    }
    if (dev && hipEventRecord(x->ev_in, (hipStream_t)r->ready_stream) != hipSuccess) {
        destroy_reqx(x);
        return fail(TINA_ERR_DEVICE, "submit: recording the input-ready event on ready_stream");
    }
    sched::Request* q = nullptr;
    switch (sv->sch->submit(r->stream_id, r->n_samples, dev, x->sample_bytes, x->row_bytes, t, &q)) {
        case sched::SUBMIT_OK: break;
        case sched::SUBMIT_TOO_LARGE:
            destroy_reqx(x);
            return fail(TINA_ERR_TOO_LARGE, "submit: request buffers exceed the HBM budget");
        case sched::SUBMIT_BUSY:
            destroy_reqx(x);
            return fail(TINA_ERR_BUSY, "submit: queue full");
        default:
            destroy_reqx(x);
            return fail(TINA_ERR_INVALID_ARGUMENT, "submit: bad stream id");
    }
    q->user = x;
    *id = q->id;
    sv->cv_work.notify_all();
    return TINA_OK;
}

static tina_status take_result(tina_server_s* sv, uint64_t id, tina_result* res, bool& ready) {
    sched::Request* q = sv->sch->find(id);
    if (!q) return fail(TINA_ERR_INVALID_ARGUMENT, "unknown request id");
    ready = q->phase == sched::DONE;
    if (!ready) return TINA_ERR_NOT_READY;
    if (res) {
        *res = tina_result{};
        res->status = q->status < 0 ? TINA_ERR_CANCELLED : q->status;
        res->frames = q->frames_done;
        res->t_submit_us = q->t_submit;
        res->t_admit_us = q->t_admit;
        res->t_first_step_us = q->t_first_step;
        res->t_done_us = q->t_done;
        res->steps = q->steps;
    }
    // A failed request's reason becomes the caller's tina_last_error().
    if (q->status > 0 && !rx(q)->fail_msg.empty()) (void)fail(TINA_OK, "request failed: " + rx(q)->fail_msg);
    destroy_reqx(rx(q));
    sv->sch->erase(id);
    return TINA_OK;
}

tina_status tina_pfb_poll(tina_server_t sv, uint64_t id, tina_result* res) {
    if (!sv) return fail(TINA_ERR_INVALID_ARGUMENT, "poll: NULL server");
    std::unique_lock<std::mutex> lk(sv->mu);
    bool ready = false;
    return take_result(sv, id, res, ready);
}

tina_status tina_pfb_wait(tina_server_t sv, uint64_t id, int64_t timeout_us, tina_result* res) {
    if (!sv) return fail(TINA_ERR_INVALID_ARGUMENT, "wait: NULL server");
    std::unique_lock<std::mutex> lk(sv->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us);
    for (;;) {
        bool ready = false;
        tina_status st = take_result(sv, id, res, ready);
        if (st != TINA_ERR_NOT_READY) return st;
        if (timeout_us < 0) sv->cv_done.wait(lk);
        else if (sv->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            st = take_result(sv, id, res, ready);
            return st == TINA_ERR_NOT_READY ? fail(TINA_ERR_TIMEOUT, "wait: timed out") : st;
        }
    }
}

tina_status tina_pfb_cancel(tina_server_t sv, uint64_t id) {
    if (!sv) return fail(TINA_ERR_INVALID_ARGUMENT, "cancel: NULL server");
    std::unique_lock<std::mutex> lk(sv->mu);
    if (!sv->sch->find(id)) return fail(TINA_ERR_INVALID_ARGUMENT, "cancel: unknown request id");
    const int c = sv->sch->cancel(id, sv->now_us());
    if (c == 0) return TINA_ERR_NOT_READY;
    if (c < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "cancel: only the newest queued request of a stream can be cancelled");
    sv->cv_done.notify_all();
    return TINA_OK;
}

tina_status tina_server_get_stats(tina_server_t sv, tina_server_stats* s) {
    if (!sv || !s) return fail(TINA_ERR_INVALID_ARGUMENT, "stats: NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    const sched::Stats& t = sv->sch->stats();
    *s = tina_server_stats{};
    s->steps = t.steps;
    s->samples = t.samples;
    s->frames = t.frames;
    s->completed = t.completed;
    s->admitted = t.admitted;
    s->admission_waits = t.admission_waits;
    s->device_busy_ms = sv->device_busy_ms;
    s->now_us = sv->now_us();
    s->arena_in_use = sv->sch->arena().used();
    s->arena_high_water = sv->sch->arena().high();
    return TINA_OK;
}

// Host-only check of the arena allocator (exposed for tests): op > 0
// allocates op bytes and stores the offset (or -1) in out[i]; op <= 0 releases
// the allocation made by operation -op and stores 1 (released) or 0.
tina_status tina_server_arena_simulate(int64_t capacity, const int64_t* ops, int32_t n, int64_t* out,
                                       int64_t* final_used) {
    if (!ops || !out || n < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "arena_simulate: NULL argument");
    sched::Arena a;
    a.init(capacity);
    for (int i = 0; i < n; ++i) {
        if (ops[i] > 0) out[i] = a.alloc(ops[i]);
        else {
            const int64_t j = -ops[i];
            out[i] = (j >= 0 && j < i && out[j] >= 0 && ops[j] > 0) ? (int64_t)a.release(out[j]) : 0;
        }
    }
    if (final_used) *final_used = a.used();
    return TINA_OK;
}

// Host-only run of the scheduler on a scripted sequence of operations (see
// tina_pfb_server.h): the same admission, quota, cancellation and
// completion decisions as the server, with steps that complete or fail when
// the script says so.
tina_status tina_server_schedule_simulate(int32_t max_active, int32_t max_queued, int64_t frames_per_step,
                                          int64_t arena_bytes, const tina_sched_op* ops, int32_t n_ops,
                                          tina_sched_event* events, int32_t capacity, int32_t* n_events) {
    if ((n_ops > 0 && !ops) || n_ops < 0 || !events || capacity < 0 || !n_events)
        return fail(TINA_ERR_INVALID_ARGUMENT, "schedule_simulate: NULL argument");
    if (max_active < 1 || max_queued < 1 || frames_per_step < 1 || arena_bytes < 0)
        return fail(TINA_ERR_INVALID_ARGUMENT, "schedule_simulate: bad configuration");
    sched::Scheduler sch(max_active, max_queued, frames_per_step, arena_bytes);
    std::deque<std::vector<sched::StepItem>> inflight;
    int32_t ne = 0;
    double t = 0.0;
    auto emit = [&](int32_t kind, int32_t status, uint64_t id, int64_t a, int64_t b) {
        if (ne < capacity) events[ne] = tina_sched_event{kind, status, id, a, b};
        ++ne;
    };
    auto done = [&](const std::vector<sched::Request*>& qs, int status) {
        for (sched::Request* q : qs) {
            if (q->phase != sched::DONE) sch.finish(q, status, t);
            emit(TINA_SCHED_COMPLETE, status, q->id, q->frames_done, q->steps);
        }
    };
    for (int32_t i = 0; i < n_ops; ++i, t += 1.0) {
        const tina_sched_op& op = ops[i];
        switch (op.kind) {
            case TINA_SCHED_ADD_STREAM:
                if (op.arg < 1) return fail(TINA_ERR_INVALID_ARGUMENT, "schedule_simulate: channels must be >= 1");
                emit(TINA_SCHED_ADD_STREAM, TINA_OK, (uint64_t)sch.add_stream(op.arg), op.arg, 0);
                break;
            case TINA_SCHED_SUBMIT: {
                const bool dev = op.value < 0;
                const int64_t n = dev ? -op.value : op.value;
                sched::Request* q = nullptr;
                const int P = op.arg >= 0 && op.arg < sch.n_streams() ? sch.stream(op.arg).P : 1;
                const sched::SubmitResult r = sch.submit(op.arg, n, dev, 8, 8 * (int64_t)P, t, &q);
                const int st = r == sched::SUBMIT_OK ? TINA_OK
                             : r == sched::SUBMIT_TOO_LARGE ? TINA_ERR_TOO_LARGE
                             : r == sched::SUBMIT_BUSY ? TINA_ERR_BUSY : TINA_ERR_INVALID_ARGUMENT;
                emit(TINA_SCHED_SUBMIT, st, q ? q->id : 0, n, q ? q->frames_total : 0);
                break;
            }
            case TINA_SCHED_ADMIT:
                for (sched::Request* q : sch.admit(t)) {
                    if (q->device) q->in_ready = true;  // device input: ready on admission
                    emit(TINA_SCHED_ADMIT, TINA_OK, q->id, q->off_in, q->off_out);
                }
                break;
            case TINA_SCHED_READY: {
                sched::Request* q = sch.find((uint64_t)op.value);
                if (q && q->phase == sched::ACTIVE) q->in_ready = true;
                emit(TINA_SCHED_READY, q && q->phase == sched::ACTIVE ? TINA_OK : TINA_ERR_INVALID_ARGUMENT,
                     (uint64_t)op.value, 0, 0);
                break;
            }
            case TINA_SCHED_STEP: {
                done(sch.take_empty(), TINA_OK);
                std::vector<sched::StepItem> items = sch.build_step(t);
                for (const sched::StepItem& it : items) emit(TINA_SCHED_STEP, TINA_OK, it.id, it.n_samples, it.frames);
                emit(TINA_SCHED_STEP, TINA_OK, 0, (int64_t)items.size(), (int64_t)inflight.size() + (items.empty() ? 0 : 1));
                if (!items.empty()) inflight.push_back(std::move(items));
                break;
            }
            case TINA_SCHED_COMPLETE: {
                if (inflight.empty()) {
                    emit(TINA_SCHED_COMPLETE, TINA_ERR_INVALID_ARGUMENT, 0, 0, 0);
                    break;
                }
                std::vector<sched::Request*> ended;
                const bool ok = op.arg == TINA_OK;
                std::vector<sched::Request*> complete = sch.step_done(inflight.front(), ok, op.arg, t, &ended);
                inflight.pop_front();
                done(complete, TINA_OK);
                done(ended, op.arg);
                break;
            }
            case TINA_SCHED_CANCEL: {
                const int c = sch.cancel((uint64_t)op.value, t);
                emit(TINA_SCHED_CANCEL, c > 0 ? TINA_OK : c == 0 ? TINA_ERR_NOT_READY : TINA_ERR_INVALID_ARGUMENT,
                     (uint64_t)op.value, 0, 0);
                break;
            }
            default:
                return fail(TINA_ERR_INVALID_ARGUMENT, "schedule_simulate: unknown operation kind " + std::to_string(op.kind));
        }
    }
    *n_events = ne;
    if (ne > capacity) return fail(TINA_ERR_TOO_LARGE, "schedule_simulate: more events than capacity");
    return TINA_OK;
}

}  // extern "C"
