// Batched execution of many stream chunks with different channel counts,
// tap counts and lengths in one persistent launch per stage:
//   FIR stage  -> fir_batch_kernel   (all items' FIR units)
//   DFT stage  -> dft_gemm_batch_kernel (all items' GEMM tiles)
//   state      -> gather_batch_kernel (all items' history/residue updates)
// The launches read a device-resident BatchTable (item arguments, first unit
// of each item per stage, and a cost-balanced split of every stage's units
// into one contiguous range per XCD).  The table is uploaded from pinned host
// memory on the caller's stream before the launches, so the launch arguments
// themselves never change; that also makes the three launches capturable in
// a graph and replayable with a new table.
//
// Launch shapes (frames per FIR thread, GEMM blocks per CU) are chosen by a
// small autotuner on the batch's own shape and cached by shape signature,
// in memory and, when TINA_TUNE_CACHE names a file, on disk.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "runtime_types.h"
#include "tina_pfb_batch.h"

using namespace tina;

namespace {

struct Tune {
    int fir_tf_mult = 2;      // frames per FIR thread = mult * MT
    int gemm_tile_n = kGemmBN;  // GEMM tile columns: kGemmBN, or 2 * kGemmBN (FP32 only)
};

std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune_cache;
bool g_tune_loaded = false;

const char* tune_path() { return getenv("TINA_TUNE_CACHE"); }

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* p = tune_path();
    if (!p) return;
    FILE* f = fopen(p, "r");
    if (!f) return;
    char key[512];
    int a, b;
    while (fscanf(f, "%511s %d %d", key, &a, &b) == 3)
        g_tune_cache[key] = Tune{a, (b == kGemmBN || b == 2 * kGemmBN) ? b : kGemmBN};
    fclose(f);
}

void tune_store_locked() {
    const char* p = tune_path();
    if (!p) return;
    FILE* f = fopen(p, "w");
    if (!f) return;
    for (const auto& kv : g_tune_cache) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.fir_tf_mult, kv.second.gemm_tile_n);
    fclose(f);
}

int pow2_at_least(int m) {
    int t = 1;
    while (t < m) t <<= 1;
    return t;
}

}  // namespace

struct tina_pfb_batch_s {
    int device = 0;
    int form = 0;
    int max_items = 0;
    int cus = 256;
    float* ws = nullptr;         // FIR output of all items
    int64_t ws_floats = 0;
    float* amax = nullptr;       // per-frame partial maxima (scaled forms)
    int64_t amax_floats = 0;
    int32_t* fexp = nullptr;     // per-frame scale exponents (scaled forms), amax_floats entries
    BatchTable* d_table = nullptr;
    // Two pinned host tables used in turn: a call fills one while the upload
    // of the other may still be pending, so a caller can build the next step
    // while the previous one runs.  table_free[k]: the last upload from
    // h_tables[k] has completed.
    BatchTable* h_tables[2] = {nullptr, nullptr};
    BatchTable* h_table = nullptr;  // the table being filled / launched
    int next_table = 0;
    size_t table_bytes = 0;
    hipEvent_t table_free[2] = {nullptr, nullptr};
    bool table_pending[2] = {false, false};
    Tune tune;
    bool have_tune = false;
    // Captured step graphs (the launches of one step; the table upload stays
    // outside), keyed by the kernel variant: tap ring, exact taps, launch
    // shape.  gemm_node: the GEMM launch, whose grid is set to each step's own
    // tile count before the replay.
    struct StepGraph {
        hipGraph_t graph = nullptr;  // kept: its nodes name the executable graph's nodes
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t gemm_node = nullptr;
        hipKernelNodeParams gemm_params{};
    };
    std::map<std::string, StepGraph> graphs;
    int64_t graph_gemm_grid = 0;  // GEMM grid the step graphs are captured with (0: no graphs)
    bool frame_stage = true;      // long per-frame scaled items run the single-pass frame stage
    int64_t frame_stage_min = 2048;  // frames an item needs to run the frame stage
    int frame_tf_target = 128;       // frames per frame-stage unit (rounded up to whole ring blocks of M)
    // Items whose plan takes the factored DFT (FP32): one launch per (P,
    // input type) over their frames, with the items' FftItem rows stored in
    // the table buffer after the items (fft_offset).
    struct FftGroup {
        int P;
        bool cplx, q64_ok;
        int first, count;  // rows [first, first + count) of the table's FftItem array
        int64_t F;         // frames of the group's items
        const float *mat1, *mat3, *tw;
    };
    std::vector<FftGroup> fft_groups;
    bool one_stream = false;      // every call comes on one stream: no order event is recorded
    StreamOrder order;            // every call shares ws, amax, fexp and d_table

    void release() {
        order.release();
        for (auto& kv : graphs) {
            (void)hipGraphExecDestroy(kv.second.exec);
            (void)hipGraphDestroy(kv.second.graph);
        }
        graphs.clear();
        for (int k = 0; k < 2; ++k) {
            if (table_free[k]) (void)hipEventDestroy(table_free[k]);
            if (h_tables[k]) (void)hipHostFree(h_tables[k]);
            table_free[k] = nullptr;
            h_tables[k] = nullptr;
        }
        h_table = nullptr;
        for (void* p : {(void*)ws, (void*)amax, (void*)fexp, (void*)d_table})
            if (p) (void)hipFree(p);
        ws = nullptr; amax = nullptr; fexp = nullptr; d_table = nullptr;
    }
};

namespace {

size_t table_size(int n) { return sizeof(BatchTable) + sizeof(BatchItem) * (size_t)(n > 1 ? n - 1 : 0); }
// Byte offset of the factored-DFT rows (FftItem) after n items, and the
// bytes a table of n items with nf such rows uploads.
size_t fft_offset(int n) { return (table_size(n) + 15) / 16 * 16; }
size_t upload_size(int n, int nf) { return nf > 0 ? fft_offset(n) + sizeof(FftItem) * (size_t)nf : table_size(n); }
FftItem* fft_rows(BatchTable* t, int n) { return reinterpret_cast<FftItem*>(reinterpret_cast<uint8_t*>(t) + fft_offset(n)); }

// Cost-balanced split of a stage's units into 8 contiguous ranges: item i has
// units[i] units of cost cost[i] each.
void split_by_cost(const std::vector<int64_t>& units, const std::vector<double>& cost, int64_t (&bounds)[9]) {
    double total = 0.0;
    int64_t total_units = 0;
    for (size_t i = 0; i < units.size(); ++i) {
        total += (double)units[i] * cost[i];
        total_units += units[i];
    }
    int64_t u0 = 0;
    double c0 = 0.0;
    bounds[0] = 0;
    int x = 1;
    for (size_t i = 0; i < units.size() && x < 8; ++i) {
        const double ci = (double)units[i] * cost[i];
        while (x < 8 && c0 + ci >= total * x / 8.0) {
            const double need = total * x / 8.0 - c0;
            int64_t k = cost[i] > 0 ? (int64_t)(need / cost[i] + 0.5) : 0;
            k = std::max<int64_t>(0, std::min<int64_t>(k, units[i]));
            bounds[x] = std::max(bounds[x - 1], u0 + k);
            ++x;
        }
        u0 += units[i];
        c0 += ci;
    }
    for (; x < 8; ++x) bounds[x] = std::max(bounds[x - 1], std::min(u0, total_units));
    bounds[8] = total_units;  // every unit belongs to exactly one range
}

struct GroupPlan {
    int first, count;  // items [first, first + count)
};

// Validates the work items against the batch and returns the frame count of each.
tina_status validate(tina_pfb_batch_s* b, tina_pfb_work* w, int32_t n, std::vector<int64_t>& frames) {
    if (n < 0 || n > b->max_items) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: item count outside [0, max_items]");
    if (n > 0 && !w) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: NULL item array");
    frames.assign(n, 0);
    std::vector<const void*> states;
    for (int i = 0; i < n; ++i) {
        const tina_pfb_work& it = w[i];
        const tina_pfb_plan_s* p = it.plan;
        if (!p) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: item " + std::to_string(i) + " has no plan");
        if (p->device != b->device) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: plan on another device");
        if (p->dft_algorithm != TINA_DFT_DENSE && p->dft_algorithm != TINA_DFT_FACTORED)
            return fail(TINA_ERR_UNSUPPORTED, "batch: plans with the fused or compensated DFT run through tina_pfb_execute only");
        if (p->output != TINA_OUT_PFB || p->precision != b->form)
            return fail(TINA_ERR_INVALID_ARGUMENT, "batch: every plan must be a filter-bank plan of the batch's precision");
        if (it.n_samples < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: negative sample count");
        if (it.n_samples > 0 && !it.d_in) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: NULL input");
        if ((uintptr_t)it.d_in % (p->cf * sizeof(float))) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: input misaligned");
        if ((uintptr_t)it.d_out % 8) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: output misaligned");
        if (it.state && it.state->plan != p) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: state belongs to another plan");
        if (it.state) {
            if (std::find(states.begin(), states.end(), (const void*)it.state) != states.end())
                return fail(TINA_ERR_INVALID_ARGUMENT, "batch: a state appears twice in one batch");
            states.push_back(it.state);
        }
        const int64_t r = it.state ? it.state->residue : 0;
        frames[i] = (r + it.n_samples) / p->P;
        if (frames[i] > 0 && !it.d_out) return fail(TINA_ERR_INVALID_ARGUMENT, "batch: NULL output");
        if (frames[i] > it.out_capacity_frames)
            return fail(TINA_ERR_INVALID_ARGUMENT, "batch: item " + std::to_string(i) + " output capacity below its frame count");
        if (frames[i] * (int64_t)p->W > b->ws_floats)
            return fail(TINA_ERR_TOO_LARGE, "batch: item " + std::to_string(i) + " alone exceeds the batch workspace");
    }
    return TINA_OK;
}

// Fills the host table for items [g.first, g.first + g.count) and returns the
// launch parameters.  `dry` leaves state updates out (tuning runs).
void fill_table(tina_pfb_batch_s* b, tina_pfb_work* w, const std::vector<int64_t>& frames, const GroupPlan& g,
                const Tune& tune, bool dry, int& max_m, bool& all_exact, bool& wide) {
    BatchTable* t = b->h_table;
    t->n_items = g.count;
    // Reduced forms take the single-stream path's wide tiles when every item's
    // K is a whole number of their K tiles (else all take 128 x 128 tiles).
    int wbm = kGemmBM, wbn = tune.gemm_tile_n;
    wide = form_fir_qmode(b->form) != 0;
    for (int i = 0; i < g.count && wide; ++i) wide = gemm_batch_wide_tile(b->form, w[g.first + i].plan->K, wbm, wbn);
    const int tile_m = wide ? wbm : kGemmBM, tile_n = wide ? wbn : tune.gemm_tile_n;
    max_m = 1;
    for (int i = 0; i < g.count; ++i) max_m = std::max(max_m, w[g.first + i].plan->M);
    const int MT = pow2_at_least(max_m);
    all_exact = true;
    for (int i = 0; i < g.count; ++i) all_exact = all_exact && w[g.first + i].plan->M == MT;
    // Frames per FIR thread, a whole number of the unit's ring blocks: the
    // ring is MT frames long, or the item's own M when mixed tap counts up to
    // 16 run per-M units.
    auto frames_per_thread = [&](int ring) {
        return tune.fir_tf_mult * ring < 16 ? ((16 + ring - 1) / ring) * ring : tune.fir_tf_mult * ring;
    };

    std::vector<int64_t> fu(g.count), gu(g.count), su(g.count), ru(g.count);
    std::vector<int> fft_items;  // items taking the factored DFT
    std::vector<double> fc(g.count), gc(g.count), sc(g.count, 1.0), rc(g.count, 1.0);
    int64_t ws_off = 0, amax_off = 0, f0 = 0, g0 = 0, s0 = 0, r0 = 0;
    for (int i = 0; i < g.count; ++i) {
        tina_pfb_work& it = w[g.first + i];
        tina_pfb_plan_s* p = it.plan;
        tina_pfb_state_s* st = it.state;
        BatchItem& bi = t->items[i];
        memset(&bi, 0, sizeof(bi));
        const int64_t F = frames[g.first + i];
        const int64_t r = st ? st->residue : 0;
        if (st) st->plan_ordered = false;  // batch work is not covered by the plan's stream-order event
        FirArgs& fa = bi.fir;
        fa.prefix = st ? st->buf[st->cur] : nullptr;
        fa.plen = (int64_t)(p->M - 1) * p->W + r * p->cf;
        fa.chunk = (const float*)it.d_in;
        fa.nchunk = it.n_samples * p->cf;
        fa.taps = p->h32;
        fa.y = b->ws + ws_off;
        fa.ldy = p->W;
        fa.g0 = 0;
        fa.F = F;
        fa.W = p->W;
        fa.P = p->P;
        fa.M = p->M;
        fa.cf = p->cf;
        fa.amax = form_scaled(b->form) ? b->amax + amax_off : nullptr;
        fa.nparts = p->W >= 32 ? p->W / 32 : 1;  // VEC = 1 in the batched FIR: one part per 32 lanes
        // Operand-form FIR output inside the item's F * W floats: E4M3 codes
        // (then the block scales), or the 16-bit piece(s) one after the other;
        // per-frame scaled forms keep one exponent per frame (amax_off counts
        // at least one part per frame, so it also places them).
        fa.qmode = form_fir_qmode(b->form);
        if (fa.qmode != 0) {
            fa.y = nullptr;
            fa.q = (uint8_t*)(b->ws + ws_off);
            fa.ldq = p->W;
            if (form_mx(b->form)) fa.qs = fa.q + mx_codes_bytes(F, p->W);
            if (b->form == TINA_PREC_BF16X3 || b->form == TINA_PREC_FP16X3) fa.q1 = fa.q + F * p->W * 2;
            if (form_scaled(b->form)) fa.fexp = b->fexp + amax_off;
        }
        ws_off += F * p->W;
        amax_off += F * fa.nparts;
        GemmArgs& ga = bi.gemm;
        ga.A = fa.y;
        ga.lda = p->W;
        ga.B0 = p->B[0];
        ga.B1 = p->B[1];
        ga.out = (float*)it.d_out;
        ga.ldo = p->cf == 2 ? 2 * (int64_t)p->P : (int64_t)p->P + 2;
        ga.F = F;
        ga.K = p->K;
        ga.N = p->N;
        ga.real_pack = p->cf == 1;
        ga.form = b->form;
        ga.Aq = fa.q;
        ga.Aq1 = fa.q1;
        ga.Aqs = fa.qs;
        ga.fexp = fa.fexp;
        // Per-frame scaled items with frame rows of 1024 threads and at least
        // frame_stage_min frames run in one pass (frame stage, units of about
        // frame_tf_target frames); the others in the three FIR launches
        // (units of 256 threads).  A frame-stage unit walks its frames one
        // ring block after another, so short items would take a unit's whole
        // latency for little work.
        bi.fir_single = (b->frame_stage && form_scaled(b->form) && F >= b->frame_stage_min &&
                         fir_frame_batch_vec(fa) != 0) ? 1 : 0;
        bi.frame_unit0 = r0;
        if (bi.fir_single) {
            const int TF = p->M * ((b->frame_tf_target + p->M - 1) / p->M);
            bi.fir_tf = TF;
            fu[i] = 0;
            fc[i] = 1.0;
            ru[i] = F > 0 ? (F + TF - 1) / TF : 0;
            rc[i] = (double)TF * p->W * p->M;
        } else {
            const int ring = (!all_exact && MT <= 16) ? p->M : MT;
            const int TF = frames_per_thread(ring);
            bi.fir_tf = TF;
            const int64_t runs = (F + TF - 1) / TF;
            fu[i] = F > 0 ? (runs * p->W + 255) / 256 : 0;
            fc[i] = (double)TF * ring;
            ru[i] = 0;
        }
        r0 += ru[i];
        const bool factored = p->dft_algorithm == TINA_DFT_FACTORED;
        gu[i] = (F > 0 && !factored) ? ((F + tile_m - 1) / tile_m) * ((p->N + tile_n - 1) / tile_n) : 0;
        if (factored && F > 0) fft_items.push_back(i);
        gc[i] = (double)p->K;
        bi.fir_unit0 = f0;
        bi.gemm_unit0 = g0;
        bi.st_unit0 = s0;
        f0 += fu[i];
        g0 += gu[i];
        if (st && !dry) {
            const int64_t r2 = (r + it.n_samples) % p->P;
            bi.st_dst = st->buf[st->cur ^ 1];
            bi.st_start = F * p->W;
            bi.st_count = (int64_t)(p->M - 1) * p->W + r2 * p->cf;
            su[i] = (bi.st_count + 255) / 256;
        } else {
            su[i] = 0;
        }
        s0 += su[i];
    }
    // Factored-DFT rows, grouped by (P, input type) in item order; a group's
    // rows number its frames one item after the other.
    b->fft_groups.clear();
    std::stable_sort(fft_items.begin(), fft_items.end(), [&](int x, int y) {
        const tina_pfb_plan_s *px = w[g.first + x].plan, *py = w[g.first + y].plan;
        return px->P != py->P ? px->P < py->P : px->cf < py->cf;
    });
    FftItem* rows = fft_rows(t, g.count);
    for (size_t k = 0; k < fft_items.size(); ++k) {
        const int i = fft_items[k];
        const tina_pfb_plan_s* p = w[g.first + i].plan;
        const BatchItem& bi = t->items[i];
        if (b->fft_groups.empty() || b->fft_groups.back().P != p->P || b->fft_groups.back().cplx != (p->cf == 2)) {
            tina_pfb_batch_s::FftGroup fg;
            fg.P = p->P;
            fg.cplx = p->cf == 2;
            fg.q64_ok = true;
            fg.first = (int)k;
            fg.count = 0;
            fg.F = 0;
            fg.mat1 = p->fft_mat1;
            fg.mat3 = p->fft_mat3;
            fg.tw = p->fft_tw;
            b->fft_groups.push_back(fg);
        }
        tina_pfb_batch_s::FftGroup& fg = b->fft_groups.back();
        FftItem& r = rows[k];
        r.y = bi.fir.y;
        r.out = bi.gemm.out;
        r.ldy = bi.fir.ldy;
        r.ldo = bi.gemm.ldo;
        r.f0 = fg.F;
        fg.q64_ok = fg.q64_ok && r.ldy % 4 == 0 && ((uintptr_t)r.y & 15) == 0;
        fg.F += bi.gemm.F;
        fg.count += 1;
    }
    t->gemm_bn = tile_n;
    t->gemm_wide = wide ? 1 : 0;
    t->fir_units = f0;
    t->gemm_units = g0;
    t->st_units = s0;
    t->frame_units = r0;
    split_by_cost(fu, fc, t->fir_bounds);
    split_by_cost(ru, rc, t->frame_bounds);
    split_by_cost(gu, gc, t->gemm_bounds);
    split_by_cost(su, sc, t->st_bounds);
}

// Groups items greedily so that each group's FIR output fits the workspace.
std::vector<GroupPlan> make_groups(tina_pfb_batch_s* b, tina_pfb_work* w, const std::vector<int64_t>& frames, int n) {
    std::vector<GroupPlan> gs;
    int first = 0;
    int64_t used = 0, used_amax = 0;
    for (int i = 0; i < n; ++i) {
        const tina_pfb_plan_s* p = w[i].plan;
        const int64_t need = frames[i] * p->W;
        const int64_t need_amax = frames[i] * (p->W >= 32 ? p->W / 32 : 1);
        if (i > first && (used + need > b->ws_floats || (b->amax && used_amax + need_amax > b->amax_floats))) {
            gs.push_back({first, i - first});
            first = i;
            used = 0;
            used_amax = 0;
        }
        used += need;
        used_amax += need_amax;
    }
    if (n > first) gs.push_back({first, n - first});
    return gs;
}

// Blocks of the batched GEMM launch: 8 x the largest XCD range (one block per
// tile), or the fixed bound of a captured step graph.
int64_t gemm_grid(const BatchTable* t) {
    int64_t mx = 0;
    for (int x = 0; x < 8; ++x) mx = std::max(mx, t->gemm_bounds[x + 1] - t->gemm_bounds[x]);
    return 8 * std::max<int64_t>(mx, 1);
}

tina_status launch_stages(tina_pfb_batch_s* b, hipStream_t s, const Tune& tune, int max_m, bool all_exact,
                          bool wide, bool always, int64_t fixed_gemm_grid = 0) {
    const int grid_fir = b->cus * 4;
    const int64_t grid_gemm = fixed_gemm_grid > 0 ? fixed_gemm_grid : gemm_grid(b->h_table);
    const int qmode = form_fir_qmode(b->form);
    if (always || b->h_table->fir_units > 0 || b->h_table->frame_units > 0)
        HIP_TRY(launch_fir_batch(b->d_table, max_m, all_exact, qmode, grid_fir, s, b->frame_stage));
    if (always || b->h_table->gemm_units > 0)
        HIP_TRY(launch_gemm_batch(b->d_table, b->form, qmode != 0, tune.gemm_tile_n, (int)grid_gemm, s, wide));
    if (!always)  // factored-DFT items: never in a captured step (the groups change from call to call)
        for (const tina_pfb_batch_s::FftGroup& fg : b->fft_groups)
            HIP_TRY(launch_fft_batch(fft_rows(b->d_table, b->h_table->n_items) + fg.first, fg.count, fg.F, fg.P,
                                     fg.cplx, fg.q64_ok, fg.mat1, fg.mat3, fg.tw, b->cus, s));
    if (always || b->h_table->st_units > 0) HIP_TRY(launch_gather_batch(b->d_table, b->cus * 2, s));
    return TINA_OK;
}

// The captured step graph of one kernel variant (tap ring, exact taps,
// launch shape), captured and instantiated on first use.  The GEMM launch is
// found among the graph's kernel nodes by its grid (graph_gemm_grid is kept
// apart from the fixed grids of the other stages).
tina_status step_graph(tina_pfb_batch_s* b, hipStream_t s, const Tune& tune, int max_m, bool all_exact, bool wide,
                       tina_pfb_batch_s::StepGraph*& out) {
    const std::string key = std::to_string(pow2_at_least(max_m)) + (all_exact ? "e" : "p") + (wide ? "w" : "n") +
                            ":" + std::to_string(tune.fir_tf_mult) + ":" + std::to_string(tune.gemm_tile_n);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        tina_status st = launch_stages(b, s, tune, max_m, all_exact, wide, true, b->graph_gemm_grid);
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (st != TINA_OK || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(TINA_ERR_DEVICE, "batch: step graph capture failed");
        }
        tina_pfb_batch_s::StepGraph sg;
        size_t nn = 0;
        hipError_t e = hipGraphGetNodes(graph, nullptr, &nn);
        std::vector<hipGraphNode_t> nodes(nn);
        if (e == hipSuccess && nn > 0) e = hipGraphGetNodes(graph, nodes.data(), &nn);
        for (size_t i = 0; e == hipSuccess && i < nn; ++i) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nodes[i], &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(nodes[i], &kp) == hipSuccess && (int64_t)kp.gridDim.x == b->graph_gemm_grid) {
                sg.gemm_node = nodes[i];
                sg.gemm_params = kp;
            }
        }
        e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(TINA_ERR_DEVICE, std::string("batch: graph instantiate: ") + hipGetErrorString(e));
        }
        sg.graph = graph;
        it = b->graphs.emplace(key, sg).first;
    }
    out = &it->second;
    return TINA_OK;
}

// tables_retired: the caller guarantees that the work of the call before the
// previous one has completed (the server retires a step before building the
// one after the next), so a host table's last upload is known to be done and
// no event is recorded after it.
tina_status run_batch(tina_pfb_batch_s* b, tina_pfb_work* w, int32_t n, hipStream_t s, const Tune& tune, bool dry,
                      const std::vector<int64_t>& frames, bool use_graph = false, bool tables_retired = false) {
    const std::vector<GroupPlan> groups = make_groups(b, w, frames, n);
    use_graph = use_graph && groups.size() == 1;
    // Launch errors are read with hipGetLastError: a status left by an earlier
    // query of a pending event (hipErrorNotReady) must not be read as one.
    (void)hipGetLastError();
    if (!b->one_stream) HIP_TRY(b->order.begin(s));
    for (const GroupPlan& g : groups) {
        const int k = b->next_table;
        b->next_table ^= 1;
        if (b->table_pending[k]) {
            HIP_TRY(hipEventSynchronize(b->table_free[k]));  // this host table's last upload is done
            b->table_pending[k] = false;
        }
        b->h_table = b->h_tables[k];
        int max_m = 1;
        bool all_exact = true, wide = false;
        fill_table(b, w, frames, g, tune, dry, max_m, all_exact, wide);
        int n_fft = 0;
        for (const tina_pfb_batch_s::FftGroup& fg : b->fft_groups) n_fft += fg.count;
        HIP_TRY(hipMemcpyAsync(b->d_table, b->h_table, upload_size(g.count, n_fft), hipMemcpyHostToDevice, s));
        if (!tables_retired || groups.size() > 1) {
            HIP_TRY(hipEventRecord(b->table_free[k], s));
            b->table_pending[k] = true;
        }
        tina_pfb_batch_s::StepGraph* sg = nullptr;
        if (use_graph && b->graph_gemm_grid > 0 && gemm_grid(b->h_table) <= b->graph_gemm_grid && b->fft_groups.empty()) {
            tina_status st = step_graph(b, s, tune, max_m, all_exact, wide, sg);
            if (st != TINA_OK) return st;
            if (sg->gemm_node) {  // this step's GEMM grid: blocks past the tiles' ranges would only return
                hipKernelNodeParams kp = sg->gemm_params;
                kp.gridDim.x = (unsigned)gemm_grid(b->h_table);
                if (hipGraphExecKernelNodeSetParams(sg->exec, sg->gemm_node, &kp) != hipSuccess) {
                    // Replays keep the captured (largest) grid from now on; the
                    // failed call's error is cleared so later launches do not
                    // report it.
                    (void)hipGetLastError();
                    sg->gemm_params.gridDim.x = (unsigned)b->graph_gemm_grid;
                    (void)hipGraphExecKernelNodeSetParams(sg->exec, sg->gemm_node, &sg->gemm_params);
                    (void)hipGetLastError();
                    sg->gemm_node = nullptr;
                }
            }
        }
        if (sg) {
            // Fixed topology: all three launches (a stage with no units returns
            // at once), so one graph per kernel variant serves every step.
            HIP_TRY(hipGraphLaunch(sg->exec, s));
        } else {
            tina_status st = launch_stages(b, s, tune, max_m, all_exact, wide, false);
            if (st != TINA_OK) return st;
        }
        if (!dry) {
            for (int i = 0; i < g.count; ++i) {
                tina_pfb_work& it = w[g.first + i];
                it.frames_written = frames[g.first + i];
                if (it.state) {
                    it.state->cur ^= 1;
                    it.state->residue = (it.state->residue + it.n_samples) % it.plan->P;
                }
            }
        }
    }
    if (!b->one_stream) HIP_TRY(b->order.end(s));
    return TINA_OK;
}

std::string signature(tina_pfb_batch_s* b, tina_pfb_work* w, const std::vector<int64_t>& frames, int n) {
    std::vector<std::string> parts;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        char buf[64];
        snprintf(buf, sizeof buf, "%dx%dx%d", w[i].plan->P, w[i].plan->M, w[i].plan->cf);
        parts.push_back(buf);
        total += frames[i] * w[i].plan->P;
    }
    std::sort(parts.begin(), parts.end());
    parts.erase(std::unique(parts.begin(), parts.end()), parts.end());
    int lg = 0;
    while ((1ll << (lg + 1)) <= total) ++lg;
    std::string key = "form" + std::to_string(b->form) + ":s2^" + std::to_string(lg);
    for (auto& p : parts) key += ":" + p;
    return key;
}

}  // namespace

// Used by the server: the largest GEMM tile count of one of its steps, which
// fixes the grid of the captured step graphs (the cost-balanced split may give
// one XCD up to all of them).
void batch_set_graph_bound(tina_pfb_batch_s* b, int64_t max_gemm_tiles) {
    int64_t g = 8 * std::max<int64_t>(max_gemm_tiles, 1);
    while (g == (int64_t)b->cus * 4 || g == (int64_t)b->cus * 2) g += 8;  // unlike every other stage's grid
    b->graph_gemm_grid = g;
}

// Used by the server, which owns the batch and runs every step on its one
// compute stream.  Per-frame scaled items of at least 256 frames take the
// single-pass frame stage with short units (about 32 frames: a step's items
// are short, and a 128-frame unit's latency, ~70 us, would set the step's
// length; measured on the FP8 serving mix at 0.8 of the batched capacity, p99
// 2.2-2.5 ms against 3.1-3.2 ms with the three launches, and the same at
// 0.5).  No event orders a call after the previous one (a recorded event
// leaves the device idle for ~5 us between two steps).
void batch_set_server_mode(tina_pfb_batch_s* b) {
    b->frame_stage = true;
    b->frame_stage_min = 256;
    b->frame_tf_target = 32;
    b->one_stream = true;
}

// Used by the server: run one step's items, through the cached step graph
// when use_graph is set.  The server builds a step only after retiring the
// step before the previous one (at most two in flight).
tina_status batch_run_items(tina_pfb_batch_s* b, tina_pfb_work* w, int32_t n, hipStream_t s, bool use_graph) {
    std::vector<int64_t> frames;
    tina_status st = validate(b, w, n, frames);
    if (st != TINA_OK) return st;
    DeviceScope ds(b->device);
    // Steps keep the default launch shape: graph steps are captured in
    // advance, and a step's mix of streams changes from one step to the next.
    const Tune tune;
    return run_batch(b, w, n, s, tune, false, frames, use_graph, true);
}

// Used by the server at creation: captures the step graph of every tap-ring
// variant (largest tap count 1..64, exact or mixed) with the default launch
// shape, so that no capture is ever in progress while the server runs: HIP
// refuses a device-wide synchronize from any thread during a capture.
tina_status batch_prepare_graphs(tina_pfb_batch_s* b, hipStream_t s) {
    DeviceScope ds(b->device);
    const Tune tune;
    const int n_wide = form_fir_qmode(b->form) != 0 ? 2 : 1;  // reduced forms: wide and 128 x 128 GEMM tiles
    for (int mt = 1; mt <= 64; mt *= 2)
        for (int exact = 1; exact >= (mt == 1 ? 1 : 0); --exact)
            for (int wide = 0; wide < n_wide; ++wide) {
                tina_pfb_batch_s::StepGraph* sg = nullptr;
                tina_status st = step_graph(b, s, tune, mt, exact != 0, wide != 0, sg);
                if (st != TINA_OK) return st;
            }
    return TINA_OK;
}

// Used by a server that launches its steps without graphs: one launch of
// every kernel variant a step can use, on an empty table (every stage's
// unit ranges are empty, so each block returns at once), so that a first
// step does not pay for loading them.
tina_status batch_warm_kernels(tina_pfb_batch_s* b, hipStream_t s) {
    DeviceScope ds(b->device);
    const Tune tune;
    HIP_TRY(hipMemsetAsync(b->d_table, 0, sizeof(BatchTable), s));
    const int n_wide = form_fir_qmode(b->form) != 0 ? 2 : 1;
    for (int mt = 1; mt <= 64; mt *= 2)
        for (int exact = 1; exact >= (mt == 1 ? 1 : 0); --exact)
            for (int wide = 0; wide < n_wide; ++wide) {
                tina_status st = launch_stages(b, s, tune, mt, exact != 0, wide != 0, true, 8);
                if (st != TINA_OK) return st;
            }
    return TINA_OK;
}

extern "C" {

tina_status tina_pfb_batch_split_units(const int64_t* units, const double* cost, int32_t n, int64_t* bounds9) {
    if (n < 0 || (n > 0 && (!units || !cost)) || !bounds9) return fail(TINA_ERR_INVALID_ARGUMENT, "split_units: NULL argument");
    std::vector<int64_t> u(units, units + n);
    std::vector<double> c(cost, cost + n);
    int64_t b[9];
    split_by_cost(u, c, b);
    for (int i = 0; i < 9; ++i) bounds9[i] = b[i];
    return TINA_OK;
}

tina_status tina_pfb_batch_create(int device, int precision, int max_items, int64_t workspace_bytes,
                                  tina_pfb_batch_t* out) {
    if (!out) return fail(TINA_ERR_INVALID_ARGUMENT, "batch_create: NULL output handle");
    *out = nullptr;
    if (precision < TINA_PREC_FP32 || precision > TINA_PREC_MXFP8)
        return fail(TINA_ERR_INVALID_ARGUMENT, "batch_create: unknown precision");
    if (max_items < 1 || max_items > 65536) return fail(TINA_ERR_INVALID_ARGUMENT, "batch_create: max_items outside [1, 65536]");
    if (workspace_bytes < (1 << 20)) return fail(TINA_ERR_INVALID_ARGUMENT, "batch_create: workspace below 1 MiB");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(TINA_ERR_INVALID_ARGUMENT, "batch_create: bad device");
    DeviceScope ds(device);
    tina_pfb_batch_s* b = new (std::nothrow) tina_pfb_batch_s();
    if (!b) return fail(TINA_ERR_OUT_OF_MEMORY, "batch_create: host allocation");
    b->device = device;
    b->form = precision;
    b->max_items = max_items;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        b->cus = ((prop.multiProcessorCount + 7) / 8) * 8;
    b->ws_floats = workspace_bytes / 4;
    b->table_bytes = upload_size(max_items, max_items);
    auto bail = [&](tina_status st, const char* m) {
        b->release();
        delete b;
        return fail(st, m);
    };
    if (hipMalloc(&b->ws, b->ws_floats * 4) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "batch_create: workspace");
    if (form_scaled(precision)) {
        b->amax_floats = b->ws_floats / 16 + 1024;  // F * max(1, W/32) <= F * W / 16 for W >= 16
        if (hipMalloc(&b->amax, b->amax_floats * 4) != hipSuccess ||
            hipMalloc(&b->fexp, b->amax_floats * sizeof(int32_t)) != hipSuccess)
            return bail(TINA_ERR_OUT_OF_MEMORY, "batch_create: scale workspace");
    }
    if (hipMalloc(&b->d_table, b->table_bytes) != hipSuccess) return bail(TINA_ERR_OUT_OF_MEMORY, "batch_create: table");
    for (int k = 0; k < 2; ++k) {
        if (hipHostMalloc(&b->h_tables[k], b->table_bytes, hipHostMallocDefault) != hipSuccess)
            return bail(TINA_ERR_OUT_OF_MEMORY, "batch_create: pinned table");
        if (hipEventCreateWithFlags(&b->table_free[k], hipEventDisableTiming) != hipSuccess)
            return bail(TINA_ERR_DEVICE, "batch_create: event");
    }
    b->h_table = b->h_tables[0];
    *out = b;
    return TINA_OK;
}

tina_status tina_pfb_batch_destroy(tina_pfb_batch_t b) {
    if (!b) return TINA_OK;
    DeviceScope ds(b->device);
    (void)hipDeviceSynchronize();
    b->release();
    delete b;
    return TINA_OK;
}

tina_status tina_pfb_batch_execute(tina_pfb_batch_t b, tina_pfb_work* w, int32_t n, void* stream) {
    if (!b) return fail(TINA_ERR_INVALID_ARGUMENT, "batch_execute: NULL batch");
    std::vector<int64_t> frames;
    tina_status st = validate(b, w, n, frames);
    if (st != TINA_OK) return st;
    DeviceScope ds(b->device);
    Tune tune;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune_cache.find(signature(b, w, frames, n));
        if (it != g_tune_cache.end()) tune = it->second;
    }
    return run_batch(b, w, n, (hipStream_t)stream, tune, false, frames);
}

tina_status tina_pfb_batch_tune(tina_pfb_batch_t b, tina_pfb_work* w, int32_t n, void* stream,
                                int32_t* fir_tf_mult, int32_t* gemm_tile_n) {
    if (!b) return fail(TINA_ERR_INVALID_ARGUMENT, "batch_tune: NULL batch");
    std::vector<int64_t> frames;
    tina_status st = validate(b, w, n, frames);
    if (st != TINA_OK) return st;
    DeviceScope ds(b->device);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int mults[] = {1, 2, 4};
    // 128 x 256 GEMM tiles halve the A re-reads and suit FP32's long K tiles;
    // the other forms keep 128 x 128.
    const int tile_ns[] = {kGemmBN, 2 * kGemmBN};
    const int n_tiles = b->form == FORM_FP32 ? 2 : 1;
    Tune best;
    float best_ms = 1e30f;
    for (int m : mults)
        for (int ti = 0; ti < n_tiles; ++ti) {
            Tune t{m, tile_ns[ti]};
            st = run_batch(b, w, n, s, t, true, frames);  // warm-up, no state updates
            if (st != TINA_OK) break;
            HIP_TRY(hipEventRecord(e0, s));
            for (int rep = 0; rep < 3 && st == TINA_OK; ++rep) st = run_batch(b, w, n, s, t, true, frames);
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (st == TINA_OK && ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TINA_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        g_tune_cache[signature(b, w, frames, n)] = best;
        tune_store_locked();
    }
    if (fir_tf_mult) *fir_tf_mult = best.fir_tf_mult;
    if (gemm_tile_n) *gemm_tile_n = best.gemm_tile_n;
    return TINA_OK;
}

}  // extern "C"
