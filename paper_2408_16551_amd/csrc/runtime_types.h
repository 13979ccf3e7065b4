// Private runtime types shared by runtime.hip, batch.hip and server.hip.
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "tina_pfb.h"

// Sets the thread-local error message and returns s.
tina_status tina_fail(tina_status s, const std::string& msg);

#define fail tina_fail

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(TINA_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Makes `dev` current for the scope of a call and restores the caller's device.
// Kernel launch failures are read with hipGetLastError, so a status an earlier
// call of this thread left behind (the caller's, or one of ours that ignores
// it) is cleared first: it must not be taken for this call's.
struct DeviceScope {
    int prev = -1, dev;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int d) : dev(d) {
        (void)hipGetLastError();
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
};

// Orders the calls of one object (a plan, a batch) whose device scratch --
// workspace, argument tables -- every call shares: a call enqueued on another
// stream than the previous call's first waits for that call's work.  Calls
// under stream capture are left to the capturing caller to order.
struct StreamOrder {
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;
    bool valid = false;

    static bool capturing(hipStream_t s) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    }
    hipError_t begin(hipStream_t s) const {
        if (!valid || last == s || capturing(s)) return hipSuccess;
        return hipStreamWaitEvent(s, ev, 0);
    }
    hipError_t end(hipStream_t s) {
        if (capturing(s)) {
            valid = false;
            return hipSuccess;
        }
        if (!ev) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipEventRecord(ev, s);
        valid = e == hipSuccess;
        last = s;
        return e;
    }
    void release() {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
        valid = false;
    }
};

constexpr int64_t kWorkspaceBytes = 512ll << 20;  // FP32 FIR output per piece
constexpr int64_t kStaticScratchBytes = 64ll << 20;  // static scratch of tina_pfb_execute_noalloc, per device

inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

struct tina_pfb_plan_s {
    int device = 0;
    int P = 0, M = 0, cf = 1, W = 0;  // W = floats per frame
    int K = 0, N = 0;                 // GEMM inner and column dims
    int64_t kout = 0;                 // output channels (or P for FIR-only)
    int sample_type = 0, window = 0, precision = 0, output = 0;
    double* h64 = nullptr;
    float* h32 = nullptr;
    void* B[2] = {nullptr, nullptr};
    int dft_algorithm = 0;
    float* fft_mat1 = nullptr;  // factored DFT tables
    float* fft_mat3 = nullptr;
    float* fft_tw = nullptr;
    float* g32 = nullptr;       // synthesis FIR taps (inverse plans)
    float* hist[2] = {nullptr, nullptr};  // history scratch between workspace pieces (inverse plans)
    int cus = 256;
    float* ws = nullptr;
    float* amax = nullptr;
    int32_t* fexp = nullptr;    // per-frame scale exponents of a workspace piece (per-frame scaled forms)
    int64_t ch_frames = 0;
    int64_t amax_parts_cap = 0;
    StreamOrder order;          // execute/synthesize calls share ws, amax, fexp and hist
    // Stage timing (tina_pfb_profile_*): recorded event pairs per stage.
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_fir, ev_dft;

    hipEvent_t next_event() {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    void clear_events() {
        ev_used = 0;
        ev_fir.clear();
        ev_dft.clear();
    }

    void release() {
        order.release();
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        ev_pool.clear();
        clear_events();
        for (void* p : {(void*)h64, (void*)h32, B[0], B[1], (void*)ws, (void*)amax, (void*)fexp, (void*)fft_mat1,
                        (void*)fft_mat3, (void*)fft_tw, (void*)g32, (void*)hist[0], (void*)hist[1]})
            if (p) (void)hipFree(p);
        g32 = hist[0] = hist[1] = nullptr;
        h64 = nullptr; h32 = nullptr; B[0] = B[1] = nullptr; ws = nullptr; amax = nullptr; fexp = nullptr;
        fft_mat1 = fft_mat3 = fft_tw = nullptr;
    }
};

struct tina_pfb_state_s {
    tina_pfb_plan_s* plan = nullptr;
    float* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t residue = 0;     // samples
    int64_t cap_floats = 0;  // floats per buffer
    // The last call that read or wrote buf was an execute or synthesize call
    // of the plan that the plan's stream-order event covers (not a batch, an
    // allocation-free or a captured call).
    bool plan_ordered = false;
};


// Batched execution of one step's items (batch.hip), optionally through the
// batch context's cached step graph.
struct tina_pfb_batch_s;
struct tina_pfb_work;
tina_status batch_run_items(tina_pfb_batch_s* b, tina_pfb_work* w, int32_t n, hipStream_t s, bool use_graph);
// Bound on the GEMM tiles of one step (fixes the grid of captured steps).
void batch_set_graph_bound(tina_pfb_batch_s* b, int64_t max_gemm_tiles);
// Launches every step kernel variant once on an empty table (no graphs).
tina_status batch_warm_kernels(tina_pfb_batch_s* b, hipStream_t s);
// A batch owned by a server: one stream, short frame-stage units.
void batch_set_server_mode(tina_pfb_batch_s* b);
// Captures every step-graph variant in advance (needs the bound above).
tina_status batch_prepare_graphs(tina_pfb_batch_s* b, hipStream_t s);
