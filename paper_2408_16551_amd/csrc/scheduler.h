// Host-side scheduling of the serving loop: admission, per-step frame quotas
// and request bookkeeping, with no device calls.  The server (server.hip)
// drives it with HIP work under its lock; tina_server_schedule_simulate drives
// it with a scripted executor on the CPU, so the same decisions can be tested
// without a GPU (and built with sanitizers).  Not part of the ABI.
//
// A request's samples are issued to steps in order: a step takes up to
// `quota` frames of it, quota = frames_per_step * max(1, max_active / ready)
// (the step workspace holds max_active requests of frames_per_step frames).
// Steps may be in flight while later ones are built; a request is complete
// when every step that took its samples has completed.  A slot and the
// stream's issue order are held only while a request has samples not yet
// given to a step: once its last samples are in a step, the stream's next
// request may be admitted and take the following step (steps run in order on
// one device stream, so its chunk still follows the previous one), while the
// finished request waits only for its steps to complete.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

namespace tina {
namespace sched {

// First-fit allocator over [0, capacity) in 256-byte granules, coalescing
// neighbours on release.  Bookkeeping only: offsets into the server's arena.
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

struct Request {
    uint64_t id = 0;
    int stream = 0;
    bool device = false;          // caller's device buffers: no arena
    int64_t n_samples = 0, frames_total = 0;
    int64_t in_bytes = 0, out_bytes = 0;  // arena bytes (0 for device buffers)
    int64_t off_in = -1, off_out = -1;
    int64_t samples_issued = 0, frames_issued = 0;  // given to steps so far
    int64_t samples_done = 0, frames_done = 0;      // of steps that completed
    int64_t residue0 = 0;         // the stream's residue before this request's samples
    bool in_ready = false;        // the input is on the device
    int steps = 0;
    Phase phase = QUEUED;
    int status = 0;
    double t_submit = 0, t_admit = 0, t_first_step = 0, t_done = 0;
    void* user = nullptr;         // the driver's per-request data
};

struct Stream {
    int P = 0;
    int64_t residue_submitted = 0;  // residue after every submitted request
    int64_t residue_issued = 0;     // residue after every sample given to a step
    uint64_t owner = 0;             // the admitted request whose samples are not all issued (0: none)
    uint64_t last_admitted = 0;     // the stream's most recently admitted request
    std::deque<uint64_t> queued;    // its queued requests, oldest first
};

struct StepItem {
    Request* q;                  // valid while the step is being built
    uint64_t id;                 // the request, looked up again when the step ends
    int64_t sample0, n_samples;  // the request's samples this step processes
    int64_t frame0, frames;      // the output rows they complete
};

struct Stats {
    int64_t admitted = 0, admission_waits = 0, completed = 0, steps = 0, samples = 0, frames = 0;
};

enum SubmitResult { SUBMIT_OK = 0, SUBMIT_BAD_STREAM, SUBMIT_TOO_LARGE, SUBMIT_BUSY };

class Scheduler {
  public:
    Scheduler(int max_active, int max_queued, int64_t frames_per_step, int64_t arena_bytes)
        : max_active_(max_active), max_queued_(max_queued), fps_(frames_per_step) {
        arena_.init(arena_bytes);
    }

    int add_stream(int P) {
        Stream s;
        s.P = P;
        streams_.push_back(s);
        return (int)streams_.size() - 1;
    }
    int n_streams() const { return (int)streams_.size(); }
    const Stream& stream(int i) const { return streams_[i]; }
    // Frames a request of n samples on stream s would complete if submitted now.
    int64_t frames_if_submitted(int s, int64_t n) const {
        return (streams_[s].residue_submitted + n) / streams_[s].P;
    }

    // Queue a request (arena bytes from its sample and row sizes unless device).
    SubmitResult submit(int s, int64_t n, bool device, int64_t sample_bytes, int64_t row_bytes, double t,
                        Request** out) {
        if (s < 0 || s >= (int)streams_.size()) return SUBMIT_BAD_STREAM;
        Stream& st = streams_[s];
        auto q = std::make_unique<Request>();
        q->stream = s;
        q->device = device;
        q->n_samples = n;
        q->frames_total = (st.residue_submitted + n) / st.P;
        q->in_bytes = device ? 0 : n * sample_bytes;
        q->out_bytes = device ? 0 : q->frames_total * row_bytes;
        if (Arena::round(q->in_bytes) + Arena::round(q->out_bytes) > arena_.capacity()) return SUBMIT_TOO_LARGE;
        if ((int)queue_.size() >= max_queued_) return SUBMIT_BUSY;
        q->id = next_id_++;
        q->t_submit = t;
        st.residue_submitted = (st.residue_submitted + n) % st.P;
        st.queued.push_back(q->id);
        queue_.push_back(q->id);
        *out = q.get();
        reqs_[q->id] = std::move(q);
        return SUBMIT_OK;
    }

    Request* find(uint64_t id) {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? nullptr : it->second.get();
    }
    // Forget a finished request (its result has been taken).
    void erase(uint64_t id) { reqs_.erase(id); }

    // Cancel: only a queued request that is the newest of its stream (the
    // residue of a later one would depend on it).  1 cancelled, 0 running
    // (not queued), -1 not the newest queued of its stream.
    int cancel(uint64_t id, double t) {
        Request* q = find(id);
        if (!q) return -1;
        if (q->phase != QUEUED) return 0;
        Stream& st = streams_[q->stream];
        if (st.queued.empty() || st.queued.back() != id) return -1;
        st.queued.pop_back();
        st.residue_submitted = ((st.residue_submitted - q->n_samples) % st.P + st.P) % st.P;
        queue_.erase(std::find(queue_.begin(), queue_.end(), id));
        q->status = -1;
        q->t_done = t;
        q->phase = DONE;
        return 1;
    }

    // Admission in arrival order while a slot is free (fewer than max_active
    // requests with samples to issue): a request whose stream still issues an
    // earlier request waits (its chunks run in order), a request whose
    // buffers do not fit the arena blocks the ones behind it (large requests
    // do not starve).
    std::vector<Request*> admit(double t) {
        std::vector<Request*> out;
        for (auto it = queue_.begin(); it != queue_.end();) {
            Request* q = find(*it);
            Stream& st = streams_[q->stream];
            if (st.owner != 0 || st.queued.empty() || st.queued.front() != q->id) { ++it; continue; }
            if (n_issuing_ >= max_active_) break;
            if (!q->device) {
                const int64_t oi = arena_.alloc(q->in_bytes);
                const int64_t oo = oi >= 0 ? arena_.alloc(q->out_bytes) : -1;
                if (oi < 0 || oo < 0) {
                    if (oi >= 0) arena_.release(oi);
                    ++stats_.admission_waits;
                    break;
                }
                q->off_in = oi;
                q->off_out = oo;
            }
            q->phase = ACTIVE;
            q->t_admit = t;
            q->residue0 = st.residue_issued;
            st.owner = q->id;
            st.last_admitted = q->id;
            ++n_issuing_;
            st.queued.pop_front();
            active_.push_back(q);
            out.push_back(q);
            ++stats_.admitted;
            it = queue_.erase(it);
        }
        return out;
    }

    const std::vector<Request*>& active() const { return active_; }
    int issuing() const { return n_issuing_; }  // active requests with samples not yet issued

    // The next step: every active request whose input is on the device and
    // that has samples not yet given to a step takes up to `quota` frames;
    // its stream's residue advances as the step's state update will.
    std::vector<StepItem> build_step(double t) {
        std::vector<StepItem> items;
        int64_t n_ready = 0;
        for (Request* q : active_)
            if (q->in_ready && q->samples_issued < q->n_samples) ++n_ready;
        if (n_ready == 0) return items;
        const int64_t quota = fps_ * std::max<int64_t>(1, max_active_ / n_ready);
        for (Request* q : active_) {
            if (!q->in_ready || q->samples_issued >= q->n_samples) continue;
            Stream& st = streams_[q->stream];
            const int64_t r = st.residue_issued;
            const int64_t s = std::min(q->n_samples - q->samples_issued, quota * st.P - r);
            const int64_t frames = (r + s) / st.P;
            items.push_back(StepItem{q, q->id, q->samples_issued, s, q->frames_issued, frames});
            q->samples_issued += s;
            q->frames_issued += frames;
            st.residue_issued = (r + s) % st.P;
            if (q->steps++ == 0) q->t_first_step = t;
            if (q->samples_issued == q->n_samples) release_issue(q);
        }
        ++stats_.steps;
        return items;
    }

    // A step completed (ok) or failed (!ok: its requests end with `status`;
    // items of requests already ended are ignored).  Returns the requests
    // whose samples have all been processed by completed steps (the driver
    // copies their output back, then calls finish).
    std::vector<Request*> step_done(const std::vector<StepItem>& items, bool ok, int status, double t,
                                    std::vector<Request*>* ended = nullptr) {
        std::vector<Request*> complete;
        if (!ok) {
            // The step's requests end, and with them every later request of
            // their streams already admitted (its chunks would follow output
            // this step did not produce).
            std::vector<int> failed;
            for (const StepItem& it : items) {
                Request* q = find(it.id);  // a request that ended early may be gone
                if (!q || q->phase != ACTIVE) continue;
                failed.push_back(q->stream);
                end_active(q, status, t);
                if (ended) ended->push_back(q);
            }
            std::vector<Request*> later;
            for (Request* q : active_)
                if (std::find(failed.begin(), failed.end(), q->stream) != failed.end()) later.push_back(q);
            for (Request* q : later) {
                end_active(q, status, t);
                if (ended) ended->push_back(q);
            }
            return complete;
        }
        for (const StepItem& it : items) {
            Request* q = find(it.id);  // a request that ended early may be gone
            if (!q || q->phase != ACTIVE) continue;
            q->samples_done += it.n_samples;
            q->frames_done += it.frames;
            stats_.samples += it.n_samples;
            stats_.frames += it.frames;
            if (q->samples_done == q->n_samples) complete.push_back(q);
        }
        for (Request* q : complete) to_draining(q);
        return complete;
    }

    // Admitted requests with nothing to process (zero samples) whose input
    // event has passed: complete at once, after any earlier request of their
    // stream.
    std::vector<Request*> take_empty() {
        std::vector<Request*> out;
        auto older_active = [&](const Request* q) {  // a stream's requests complete in order
            for (const Request* o : active_)
                if (o->stream == q->stream && o->id < q->id) return true;
            return false;
        };
        for (Request* q : active_)
            if (q->in_ready && q->n_samples == 0 && !older_active(q)) out.push_back(q);
        for (Request* q : out) to_draining(q);
        return out;
    }

    // The request's output is back (or needs no copy): DONE with status.
    void finish(Request* q, int status, double t) {
        if (q->phase == ACTIVE) remove_active(q);
        release_buffers(q);
        q->status = status;
        q->t_done = t;
        q->phase = DONE;
        if (status == 0) ++stats_.completed;
    }

    // Cancel every queued request (the server is stopping).
    void cancel_all_queued(double t) {
        for (uint64_t id : queue_) {
            Request* q = find(id);
            q->status = -1;
            q->t_done = t;
            q->phase = DONE;
        }
        for (Stream& st : streams_) st.queued.clear();
        queue_.clear();
    }

    // Ids of every request still held (finished ones until erased).
    std::vector<uint64_t> ids() const {
        std::vector<uint64_t> v;
        for (const auto& kv : reqs_) v.push_back(kv.first);
        return v;
    }

    const Stats& stats() const { return stats_; }
    const Arena& arena() const { return arena_; }
    size_t queued() const { return queue_.size(); }
    const std::deque<uint64_t>& queue() const { return queue_; }

  private:
    void release_issue(Request* q) {
        Stream& st = streams_[q->stream];
        if (st.owner == q->id) {
            st.owner = 0;
            --n_issuing_;
        }
    }
    void remove_active(Request* q) {
        auto it = std::find(active_.begin(), active_.end(), q);
        if (it != active_.end()) active_.erase(it);
        release_issue(q);
    }
    void release_buffers(Request* q) {
        if (q->off_in >= 0) arena_.release(q->off_in);
        if (q->off_out >= 0) arena_.release(q->off_out);
        q->off_in = q->off_out = -1;
    }
    void to_draining(Request* q) {
        remove_active(q);
        q->phase = DRAINING;
    }
    void end_active(Request* q, int status, double t) {
        // The stream continues as if the whole request had been processed,
        // so that later requests complete the frames counted at their submit
        // (the driver resets the stream's state to this residue).  A request
        // admitted after it already continues from there.
        Stream& st = streams_[q->stream];
        if (st.last_admitted == q->id) st.residue_issued = (q->residue0 + q->n_samples) % st.P;
        remove_active(q);
        release_buffers(q);
        q->status = status;
        q->t_done = t;
        q->phase = DONE;
    }

    int max_active_, max_queued_;
    int n_issuing_ = 0;
    int64_t fps_;
    uint64_t next_id_ = 1;
    Arena arena_;
    std::vector<Stream> streams_;
    std::deque<uint64_t> queue_;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::vector<Request*> active_;
    Stats stats_;
};

}  // namespace sched
}  // namespace tina
