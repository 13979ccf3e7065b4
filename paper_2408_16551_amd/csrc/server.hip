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

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_types.h"
#include "tina_pfb_batch.h"
#include "tina_pfb_server.h"

using namespace tina;

namespace {

// First-fit allocator over [0, capacity) in 256-byte units of alignment,
// coalescing neighbours on release.  Host-side bookkeeping only.
class Arena {
  public:
    void init(int64_t cap) {
        cap_ = cap;
        free_.clear();
        sizes_.clear();
        if (cap > 0) free_[0] = cap;
        used_ = high_ = 0;
    }
    static int64_t round(int64_t n) { return ((n + 255) / 256) * 256; }
    int64_t alloc(int64_t n) {
        n = round(n < 1 ? 1 : n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, rem = it->second - n;
                free_.erase(it);
                if (rem > 0) free_[off + n] = rem;
                sizes_[off] = n;
                used_ += n;
                high_ = std::max(high_, used_);
                return off;
            }
        }
        return -1;
    }
    bool release(int64_t off) {
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return false;
        int64_t n = s->second;
        sizes_.erase(s);
        used_ -= n;
        int64_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + n) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                n += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = n;
        return true;
    }
    int64_t used() const { return used_; }
    int64_t high() const { return high_; }
    int64_t capacity() const { return cap_; }

  private:
    int64_t cap_ = 0, used_ = 0, high_ = 0;
    std::map<int64_t, int64_t> free_;
    std::unordered_map<int64_t, int64_t> sizes_;
};

enum Phase { QUEUED, ACTIVE, DRAINING, DONE };

struct Req {
    uint64_t id = 0;
    tina_request r{};
    int64_t frames_total = 0;
    int64_t in_bytes = 0, out_bytes = 0, row_bytes = 0, sample_bytes = 0;
    int64_t off_in = -1, off_out = -1;
    int64_t samples_done = 0, frames_done = 0;
    bool in_ready = false;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    Phase phase = QUEUED;
    tina_result res{};
};

struct LStream {
    tina_pfb_plan_s* plan = nullptr;
    tina_pfb_state_s* state = nullptr;
    int64_t submitted_residue = 0;  // residue after every submitted request
    bool busy = false;              // a request of this stream is admitted
    std::vector<uint64_t> queued;   // its queued requests, oldest first
};

}  // namespace

struct tina_server_s {
    tina_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    bool failed = false;
    std::string fail_msg;

    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    std::vector<Req*> active, draining;
    std::vector<LStream> streams;
    std::map<std::string, tina_pfb_plan_s*> plans;
    uint64_t next_id = 1;

    Arena arena;
    uint8_t* arena_base = nullptr;
    tina_pfb_batch_s* batch = nullptr;
    hipStream_t s_comp = nullptr, s_h2d = nullptr, s_d2h = nullptr;  // copies in and out on their own streams
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    std::chrono::steady_clock::time_point t0;
    tina_server_stats stats{};

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    void finish(Req* q, int status);
};

namespace {

void destroy_req(Req* q) {
    if (q->ev_in) (void)hipEventDestroy(q->ev_in);
    if (q->ev_out) (void)hipEventDestroy(q->ev_out);
    delete q;
}

}  // namespace

// Marks q done with `status` (lock held), frees its arena buffers.
void tina_server_s::finish(Req* q, int status) {
    if (q->off_in >= 0) arena.release(q->off_in);
    if (q->off_out >= 0) arena.release(q->off_out);
    q->off_in = q->off_out = -1;
    q->res.status = status;
    q->res.frames = q->frames_done;
    q->res.t_done_us = now_us();
    q->phase = DONE;
    if (status == TINA_OK) ++stats.completed;
    cv_done.notify_all();
}

void tina_server_s::loop() {
    (void)hipSetDevice(cfg.device);
    std::vector<tina_pfb_work> items;
    std::vector<Req*> in_step;
    for (;;) {
        std::vector<Req*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && active.empty() && draining.empty()) break;
            // Admission in arrival order; a request of a busy stream waits, a
            // request that does not fit the arena blocks the ones behind it.
            for (auto it = queue.begin(); it != queue.end();) {
                Req* q = reqs[*it];
                LStream& ls = streams[q->r.stream_id];
                if (ls.busy || ls.queued.empty() || ls.queued.front() != q->id) { ++it; continue; }
                if ((int)active.size() >= cfg.max_active) break;
                if (!(q->r.flags & TINA_REQ_DEVICE_BUFFERS)) {
                    const int64_t oi = arena.alloc(q->in_bytes);
                    const int64_t oo = oi >= 0 ? arena.alloc(q->out_bytes) : -1;
                    if (oi < 0 || oo < 0) {
                        if (oi >= 0) arena.release(oi);
                        ++stats.admission_waits;
                        break;
                    }
                    q->off_in = oi;
                    q->off_out = oo;
                }
                q->phase = ACTIVE;
                q->res.t_admit_us = now_us();
                ls.busy = true;
                ls.queued.erase(ls.queued.begin());
                active.push_back(q);
                admitted.push_back(q);
                ++stats.admitted;
                it = queue.erase(it);
            }
            stats.arena_in_use = arena.used();
            stats.arena_high_water = arena.high();
        }
        for (Req* q : admitted) {  // input copies, outside the lock
            if (q->r.flags & TINA_REQ_DEVICE_BUFFERS) continue;  // ev_in was recorded at submit
            if (q->in_bytes > 0 && q->r.n_samples > 0)
                (void)hipMemcpyAsync(arena_base + q->off_in, q->r.host_in, q->r.n_samples * q->sample_bytes,
                                     hipMemcpyHostToDevice, s_h2d);
            (void)hipEventRecord(q->ev_in, s_h2d);
        }

        // Build the step: every active request whose input is on the device.
        // The workspace and the step graph's grid hold max_active requests of
        // frames_per_step frames each; when fewer are ready, each may take
        // proportionally more, so a lone long request does not crawl through
        // many small steps.
        items.clear();
        in_step.clear();
        std::vector<Req*> empty_done;
        {
            std::unique_lock<std::mutex> lk(mu);
            int64_t n_ready = 0;
            for (Req* q : active) {
                if (!q->in_ready) q->in_ready = hipEventQuery(q->ev_in) == hipSuccess;
                if (q->in_ready && q->r.n_samples > 0) ++n_ready;
            }
            const int64_t quota = cfg.frames_per_step * std::max<int64_t>(1, cfg.max_active / std::max<int64_t>(1, n_ready));
            for (Req* q : active) {
                if (!q->in_ready) continue;
                if (q->r.n_samples == 0) { empty_done.push_back(q); continue; }
                LStream& ls = streams[q->r.stream_id];
                const int64_t P = ls.plan->P;
                const int64_t r = ls.state->residue;
                const int64_t s = std::min(q->r.n_samples - q->samples_done, quota * P - r);
                tina_pfb_work w{};
                w.plan = ls.plan;
                w.state = ls.state;
                const bool dev = (q->r.flags & TINA_REQ_DEVICE_BUFFERS) != 0;
                const uint8_t* in0 = dev ? (const uint8_t*)q->r.host_in : arena_base + q->off_in;
                uint8_t* out0 = dev ? (uint8_t*)q->r.host_out : arena_base + q->off_out;
                w.d_in = in0 + q->samples_done * q->sample_bytes;
                w.n_samples = s;
                w.d_out = out0 + q->frames_done * q->row_bytes;
                w.out_capacity_frames = q->frames_total - q->frames_done;
                items.push_back(w);
                in_step.push_back(q);
            }
        }
        if (!items.empty()) {
            const double t_launch = now_us();
            (void)hipEventRecord(ev_a, s_comp);
            tina_status st = batch_run_items(batch, items.data(), (int32_t)items.size(), s_comp, cfg.use_graph != 0);
            (void)hipEventRecord(ev_b, s_comp);
            hipError_t e = hipEventSynchronize(ev_b);
            float ms = 0.f;
            if (e == hipSuccess) (void)hipEventElapsedTime(&ms, ev_a, ev_b);
            std::unique_lock<std::mutex> lk(mu);
            ++stats.steps;
            stats.device_busy_ms += ms;
            for (size_t i = 0; i < in_step.size(); ++i) {
                Req* q = in_step[i];
                if (q->res.steps == 0) q->res.t_first_step_us = t_launch;
                ++q->res.steps;
                if (st != TINA_OK || e != hipSuccess) continue;
                q->samples_done += items[i].n_samples;
                q->frames_done += items[i].frames_written;
                stats.samples += items[i].n_samples;
                stats.frames += items[i].frames_written;
            }
            if (st != TINA_OK || e != hipSuccess) {  // the step failed: fail its requests
                for (Req* q : in_step) {
                    streams[q->r.stream_id].busy = false;
                    active.erase(std::find(active.begin(), active.end(), q));
                    finish(q, st != TINA_OK ? st : TINA_ERR_DEVICE);
                }
                cv_work.notify_all();
                continue;
            }
        }
        // Requests whose samples are all processed: copy their output back.
        {
            std::unique_lock<std::mutex> lk(mu);
            for (auto it = active.begin(); it != active.end();) {
                Req* q = *it;
                const bool empty = std::find(empty_done.begin(), empty_done.end(), q) != empty_done.end();
                if (!empty && (q->samples_done < q->r.n_samples || !q->in_ready)) { ++it; continue; }
                // Device buffers: the step that wrote the last rows has been
                // waited for, so only host outputs need a copy.
                if (q->frames_done > 0 && !(q->r.flags & TINA_REQ_DEVICE_BUFFERS))
                    (void)hipMemcpyAsync(q->r.host_out, arena_base + q->off_out, q->frames_done * q->row_bytes,
                                         hipMemcpyDeviceToHost, s_d2h);
                (void)hipEventRecord(q->ev_out, s_d2h);
                q->phase = DRAINING;
                streams[q->r.stream_id].busy = false;
                draining.push_back(q);
                it = active.erase(it);
            }
            for (auto it = draining.begin(); it != draining.end();) {
                Req* q = *it;
                if (hipEventQuery(q->ev_out) != hipSuccess) { ++it; continue; }
                finish(q, TINA_OK);
                it = draining.erase(it);
            }
            const bool idle = items.empty();
            if (idle && !stop) cv_work.wait_for(lk, std::chrono::microseconds(100));
        }
    }
}

extern "C" {

tina_status tina_server_create(const tina_server_config* c, tina_server_t* out) {
    if (!c || !out) return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: NULL argument");
    *out = nullptr;
    if (c->struct_size < sizeof(tina_server_config)) return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: struct_size too small");
    if (c->precision < TINA_PREC_FP32 || c->precision > TINA_PREC_MXFP8)
        return fail(TINA_ERR_INVALID_ARGUMENT, "server_create: unknown precision");
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
    auto bail = [&](tina_status st, const std::string& m) {
        if (sv->batch) tina_pfb_batch_destroy(sv->batch);
        if (sv->arena_base) (void)hipFree(sv->arena_base);
        for (hipStream_t s : {sv->s_comp, sv->s_h2d, sv->s_d2h})
            if (s) (void)hipStreamDestroy(s);
        for (hipEvent_t e : {sv->ev_a, sv->ev_b})
            if (e) (void)hipEventDestroy(e);
        delete sv;
        return fail(st, m);
    };
    if (hipMalloc(&sv->arena_base, c->hbm_budget_bytes) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "server_create: arena");
    sv->arena.init(c->hbm_budget_bytes);
    const int64_t ws = (int64_t)c->max_active * c->frames_per_step * 2 * c->max_channels * 4;
    tina_status st = tina_pfb_batch_create(c->device, c->precision, c->max_active, std::max<int64_t>(ws, 1 << 20), &sv->batch);
    if (st != TINA_OK) return bail(st, std::string("server_create: ") + tina_last_error());
    // Largest GEMM tile count of a step: every slot with frames_per_step
    // frames of the widest stream (128 x 128 tiles, N = 2 * max_channels).
    batch_set_graph_bound(sv->batch, (int64_t)c->max_active * ((c->frames_per_step + kGemmBM - 1) / kGemmBM) *
                                         ((2 * (int64_t)c->max_channels + kGemmBN - 1) / kGemmBN));
    if (hipStreamCreateWithFlags(&sv->s_comp, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->s_h2d, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->s_d2h, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&sv->ev_a) != hipSuccess || hipEventCreate(&sv->ev_b) != hipSuccess)
        return bail(TINA_ERR_DEVICE, "server_create: streams/events");
    if (c->use_graph) {  // every step graph now, none while requests run
        st = batch_prepare_graphs(sv->batch, sv->s_comp);
        if (st == TINA_OK && hipStreamSynchronize(sv->s_comp) != hipSuccess) st = TINA_ERR_DEVICE;
        if (st != TINA_OK) return bail(st, std::string("server_create: ") + tina_last_error());
    }
    sv->th = std::thread([sv] { sv->loop(); });
    *out = sv;
    return TINA_OK;
}

tina_status tina_server_destroy(tina_server_t sv) {
    if (!sv) return TINA_OK;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (uint64_t id : sv->queue) {  // queued requests are cancelled
            Req* q = sv->reqs[id];
            q->res.status = TINA_ERR_CANCELLED;
            q->phase = DONE;
        }
        sv->queue.clear();
        sv->cv_work.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    DeviceScope ds(sv->cfg.device);
    (void)hipDeviceSynchronize();
    for (auto& kv : sv->reqs) destroy_req(kv.second);
    for (LStream& ls : sv->streams) tina_pfb_state_destroy(ls.state);
    for (auto& kv : sv->plans) tina_pfb_plan_destroy(kv.second);
    tina_pfb_batch_destroy(sv->batch);
    (void)hipFree(sv->arena_base);
    (void)hipStreamDestroy(sv->s_comp);
    (void)hipStreamDestroy(sv->s_h2d);
    (void)hipStreamDestroy(sv->s_d2h);
    (void)hipEventDestroy(sv->ev_a);
    (void)hipEventDestroy(sv->ev_b);
    delete sv;
    return TINA_OK;
}

tina_status tina_server_stream_create(tina_server_t sv, int32_t P, int32_t M, int32_t sample_type, int32_t window,
                                      int32_t* stream_id) {
    if (!sv || !stream_id) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: NULL argument");
    if (window == TINA_WINDOW_CUSTOM) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: custom taps are not supported here");
    if (P > sv->cfg.max_channels) return fail(TINA_ERR_INVALID_ARGUMENT, "stream_create: channels above the server's max_channels");
    std::unique_lock<std::mutex> lk(sv->mu);
    if ((int)sv->streams.size() >= sv->cfg.max_streams) return fail(TINA_ERR_BUSY, "stream_create: max_streams reached");
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
        tina_status st = tina_pfb_plan(&d, &plan);
        if (st != TINA_OK) return st;
        sv->plans[key] = plan;
    }
    LStream ls;
    ls.plan = plan;
    tina_status st = tina_pfb_state_create(plan, &ls.state);
    if (st != TINA_OK) return st;
    sv->streams.push_back(ls);
    *stream_id = (int32_t)sv->streams.size() - 1;
    return TINA_OK;
}

tina_status tina_pfb_submit(tina_server_t sv, const tina_request* r, uint64_t* id) {
    if (!sv || !r || !id) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: NULL argument");
    const double t = sv->now_us();
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(TINA_ERR_CANCELLED, "submit: server is stopping");
    if (r->stream_id < 0 || r->stream_id >= (int)sv->streams.size()) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: bad stream id");
    if (r->n_samples < 0 || (r->n_samples > 0 && !r->host_in)) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: bad input");
    if (r->flags & ~TINA_REQ_DEVICE_BUFFERS) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: unknown flags");
    const bool dev = (r->flags & TINA_REQ_DEVICE_BUFFERS) != 0;
    if (dev && (((uintptr_t)r->host_in & 3) || ((uintptr_t)r->host_out & 7)))
        return fail(TINA_ERR_INVALID_ARGUMENT, "submit: device buffers misaligned");
    LStream& ls = sv->streams[r->stream_id];
    const tina_pfb_plan_s* p = ls.plan;
    const int64_t frames = (ls.submitted_residue + r->n_samples) / p->P;
    if (frames > 0 && !r->host_out) return fail(TINA_ERR_INVALID_ARGUMENT, "submit: NULL output");
    if (frames > r->out_capacity_frames)
        return fail(TINA_ERR_INVALID_ARGUMENT, "submit: output capacity below the " + std::to_string(frames) + " frames of this request");
    Req* q = new (std::nothrow) Req();
    if (!q) return fail(TINA_ERR_OUT_OF_MEMORY, "submit: host allocation");
    q->r = *r;
    q->sample_bytes = p->cf * 4;
    q->row_bytes = p->kout * 8;
    q->frames_total = frames;
    q->in_bytes = dev ? 0 : r->n_samples * q->sample_bytes;  // arena bytes (none for device buffers)
    q->out_bytes = dev ? 0 : frames * q->row_bytes;
    if (Arena::round(q->in_bytes) + Arena::round(q->out_bytes) > sv->arena.capacity()) {
        delete q;
        return fail(TINA_ERR_TOO_LARGE, "submit: request buffers exceed the HBM budget");
    }
    if ((int)sv->queue.size() >= sv->cfg.max_queued) {
        delete q;
        return fail(TINA_ERR_BUSY, "submit: queue full");
    }
    if (hipEventCreateWithFlags(&q->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&q->ev_out, hipEventDisableTiming) != hipSuccess) {
        destroy_req(q);
        return fail(TINA_ERR_DEVICE, "submit: events");
    }
    if (dev && hipEventRecord(q->ev_in, (hipStream_t)r->ready_stream) != hipSuccess) {
        destroy_req(q);
        return fail(TINA_ERR_DEVICE, "submit: recording the input-ready event on ready_stream");
    }
    q->id = sv->next_id++;
    q->res.t_submit_us = t;
    ls.submitted_residue = (ls.submitted_residue + r->n_samples) % p->P;
    ls.queued.push_back(q->id);
    sv->reqs[q->id] = q;
    sv->queue.push_back(q->id);
    *id = q->id;
    sv->cv_work.notify_all();
    return TINA_OK;
}

static tina_status take_result(tina_server_s* sv, uint64_t id, tina_result* res, bool& ready) {
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(TINA_ERR_INVALID_ARGUMENT, "unknown request id");
    Req* q = it->second;
    ready = q->phase == DONE;
    if (!ready) return TINA_ERR_NOT_READY;
    if (res) *res = q->res;
    sv->reqs.erase(it);
    destroy_req(q);
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
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(TINA_ERR_INVALID_ARGUMENT, "cancel: unknown request id");
    Req* q = it->second;
    if (q->phase != QUEUED) return TINA_ERR_NOT_READY;
    LStream& ls = sv->streams[q->r.stream_id];
    if (ls.queued.empty() || ls.queued.back() != id)
        return fail(TINA_ERR_INVALID_ARGUMENT, "cancel: only the newest queued request of a stream can be cancelled");
    ls.queued.pop_back();
    ls.submitted_residue = ((ls.submitted_residue - q->r.n_samples) % ls.plan->P + ls.plan->P) % ls.plan->P;
    sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), id));
    q->res.status = TINA_ERR_CANCELLED;
    q->res.t_done_us = sv->now_us();
    q->phase = DONE;
    sv->cv_done.notify_all();
    return TINA_OK;
}

tina_status tina_server_get_stats(tina_server_t sv, tina_server_stats* s) {
    if (!sv || !s) return fail(TINA_ERR_INVALID_ARGUMENT, "stats: NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    *s = sv->stats;
    s->now_us = sv->now_us();
    s->arena_in_use = sv->arena.used();
    s->arena_high_water = sv->arena.high();
    return TINA_OK;
}

// Host-only check of the arena allocator (exposed for tests): op > 0
// allocates op bytes and stores the offset (or -1) in out[i]; op <= 0 releases
// the allocation made by operation -op and stores 1 (released) or 0.
tina_status tina_server_arena_simulate(int64_t capacity, const int64_t* ops, int32_t n, int64_t* out,
                                       int64_t* final_used) {
    if (!ops || !out || n < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "arena_simulate: NULL argument");
    Arena a;
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

}  // extern "C"
