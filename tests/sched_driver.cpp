// Host build of the serving scheduler (paper_2408_16551_amd/csrc/scheduler.h)
// under sanitizers: randomised scenarios with a submitter thread and a loop
// thread sharing the scheduler under one mutex, as the server does, checking
// its invariants after every operation and that every request ends with all
// of its frames.  Built and run by tests/test_sched_host.py.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "scheduler.h"

using namespace tina::sched;

#define REQUIRE(c)                                                             \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);    \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

struct Scenario {
    int max_active, max_queued;
    int64_t fps, arena;
    int n_streams, n_requests;
    unsigned seed;
};

// Slots: at most max_active requests with samples to issue, at most one per
// stream, and it is the stream's newest admitted request; the stream's older
// active requests are fully issued and wait for their steps.
static void check_invariants(Scheduler& s, int max_active) {
    REQUIRE(s.arena().used() <= s.arena().capacity());
    int issuing = 0;
    std::vector<int> per_stream(s.n_streams(), 0);
    std::vector<uint64_t> newest(s.n_streams(), 0);
    for (Request* q : s.active()) newest[q->stream] = std::max(newest[q->stream], q->id);
    for (Request* q : s.active()) {
        REQUIRE(q->phase == ACTIVE);
        REQUIRE(q->samples_done <= q->samples_issued && q->samples_issued <= q->n_samples);
        REQUIRE(q->frames_done <= q->frames_issued && q->frames_issued <= q->frames_total);
        if (q->samples_issued < q->n_samples) {
            ++issuing;
            REQUIRE(++per_stream[q->stream] == 1);
            REQUIRE(q->id == newest[q->stream]);
            REQUIRE(s.stream(q->stream).owner == q->id);
        }
    }
    REQUIRE(issuing <= s.issuing() && s.issuing() <= max_active);
}

static void run(const Scenario& sc) {
    Scheduler s(sc.max_active, sc.max_queued, sc.fps, sc.arena);
    std::mt19937 rng(sc.seed);
    const int Ps[] = {16, 32, 64, 128};
    for (int i = 0; i < sc.n_streams; ++i) s.add_stream(Ps[rng() % 4]);
    std::mutex mu;
    std::vector<uint64_t> ids;
    bool submit_done = false;

    std::thread submitter([&] {
        std::mt19937 r2(sc.seed * 7 + 1);
        for (int i = 0; i < sc.n_requests; ++i) {
            std::lock_guard<std::mutex> lk(mu);
            const int st = r2() % sc.n_streams;
            const int64_t n = (r2() % 8 == 0) ? 0 : (int64_t)(r2() % 5000);
            Request* q = nullptr;
            const bool dev = r2() % 3 == 0;
            if (s.submit(st, n, dev, 8, 8 * s.stream(st).P, i, &q) == SUBMIT_OK) {
                ids.push_back(q->id);
                if (r2() % 10 == 0 && s.cancel(q->id, i) == 1) REQUIRE(q->phase == DONE);
            }
        }
        std::lock_guard<std::mutex> lk(mu);
        submit_done = true;
    });

    std::deque<std::vector<StepItem>> inflight;
    std::vector<uint64_t> last_done(sc.n_streams, 0);
    std::vector<Request*> draining;
    for (int it = 0;; ++it) {
        std::lock_guard<std::mutex> lk(mu);
        for (Request* q : s.admit(it)) {
            REQUIRE(q->phase == ACTIVE);
            if (q->device) q->in_ready = true;
        }
        for (Request* q : s.active())
            if (!q->in_ready && rng() % 2) q->in_ready = true;
        for (Request* q : s.take_empty()) draining.push_back(q);
        if (inflight.size() < 2) {
            std::vector<StepItem> items = s.build_step(it);
            int64_t n_ready = (int64_t)items.size();
            for (const StepItem& x : items) {
                REQUIRE(x.frames <= sc.fps * std::max<int64_t>(1, sc.max_active / std::max<int64_t>(1, n_ready)));
                REQUIRE(x.n_samples > 0);
            }
            if (!items.empty()) inflight.push_back(items);
        }
        if (!inflight.empty() && rng() % 2) {
            const bool ok = rng() % 50 != 0;
            std::vector<Request*> ended;
            for (Request* q : s.step_done(inflight.front(), ok, 4, it, &ended)) draining.push_back(q);
            for (Request* q : ended) REQUIRE(q->phase == DONE && q->status == 4);
            inflight.pop_front();
        }
        for (Request* q : draining) {
            REQUIRE(q->frames_done == q->frames_total);
            REQUIRE(q->id > last_done[q->stream]);  // a stream's requests complete in order
            last_done[q->stream] = q->id;
            s.finish(q, 0, it);
        }
        draining.clear();
        check_invariants(s, sc.max_active);
        if (submit_done && s.queued() == 0 && s.active().empty() && inflight.empty()) break;
        REQUIRE(it < 10000000);
    }
    submitter.join();
    for (uint64_t id : ids) {
        Request* q = s.find(id);
        REQUIRE(q && q->phase == DONE);
        if (q->status == 0) REQUIRE(q->frames_done == q->frames_total);
        s.erase(id);
    }
    REQUIRE(s.arena().used() == 0);
}

int main() {
    const Scenario scs[] = {
        {4, 64, 8, 1 << 20, 6, 300, 1},
        {1, 8, 3, 1 << 16, 3, 200, 2},
        {32, 512, 64, 1 << 24, 64, 1000, 3},
        {8, 16, 1, 200000, 10, 400, 4},
    };
    for (const Scenario& sc : scs) run(sc);
    printf("scenarios ok\n");
    return 0;
}
