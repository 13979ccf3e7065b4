// Internal declarations shared by the library's translation units.
// Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tina {

// Arithmetic forms of the DFT stage (same values as tina_precision).
enum Form : int {
    FORM_FP32 = 0, FORM_BF16 = 1, FORM_BF16X3 = 2, FORM_FP16 = 3, FORM_FP16X3 = 4, FORM_FP8 = 5, FORM_MXFP8 = 6
};

// Forms with a per-frame scale (the FIR also writes per-frame partial maxima).
inline bool form_scaled(int f) { return f == FORM_FP16 || f == FORM_FP16X3 || f == FORM_FP8; }
// Block-scaled FP8: the FIR writes E4M3 codes plus one E8M0 scale per 32
// floats of a frame, and the GEMM reads them as they are.
inline bool form_mx(int f) { return f == FORM_MXFP8; }
inline int form_pieces(int f) { return (f == FORM_BF16X3 || f == FORM_FP16X3) ? 2 : 1; }
inline int form_elem_bytes(int f) { return f == FORM_FP32 ? 4 : ((f == FORM_FP8 || f == FORM_MXFP8) ? 1 : 2); }
// Bytes of one block-scaled FP8 matrix of `rows` x `k` entries: codes, then
// one scale byte per 32 entries of each row.
inline int64_t mx_codes_bytes(int64_t rows, int64_t k) { return rows * k; }
inline int64_t mx_bytes(int64_t rows, int64_t k) { return rows * k + rows * (k / 32); }

// Map a hardware block index to a logical tile index so that the blocks the
// dispatcher places on one XCD (it deals blocks round-robin over the 8 XCDs)
// receive consecutive logical tiles, which then share that XCD's L2.
__device__ inline int64_t xcd_logical_block(int64_t b, int64_t nb) {
    const int64_t x = b & 7, i = b >> 3;
    const int64_t q = nb >> 3, rmd = nb & 7;
    return x * q + (x < rmd ? x : rmd) + i;
}

// ---------------------------------------------------------------- generation
// Prototype window h[n], n < P*M, in FP64 (sinc x window), plus its FP32 copy.
hipError_t launch_window(double* h64, float* h32, int P, int M, int window, hipStream_t s);
// FP32 copy of FP64 taps (custom window).
hipError_t launch_taps_to_f32(const double* h64, float* h32, int64_t L, hipStream_t s);
// DFT operand Bt[N][K] (row n = output column, K contiguous) in the pieces of
// `form`: piece0 (and piece1 for split forms), element size form_elem_bytes.
// FORM_MXFP8: piece0 = E4M3 codes [N][K], piece1 = E8M0 scales [N][K/32].
hipError_t launch_dft_operand(void* piece0, void* piece1, int P, int complex_input, int form,
                              hipStream_t s, int inverse = 0);
// Block-reversed FP32 taps of the synthesis FIR.
hipError_t launch_synthesis_taps(const double* h64, float* g32, int P, int M, hipStream_t s);

// ----------------------------------------------------------------------- FIR
struct FirArgs {
    const float* prefix;  // history + residue (floats); nullptr = zeros
    int64_t plen;         // floats in the prefix
    const float* chunk;   // new samples (floats)
    int64_t nchunk;       // floats in the chunk
    const float* taps;    // FP32 prototype h[0..P*M)
    float* y;             // output rows
    int64_t ldy;          // floats per output row
    int64_t g0;           // first output frame (frame numbering of prefix-residue ++ chunk)
    int64_t F;            // frames to produce
    int32_t W;            // floats per frame (P * cf)
    int32_t P, M, cf;     // channels, taps, floats per sample
    float* amax;          // optional per-frame partial |y| maxima [F][nparts]
    int32_t nparts;       // filled in by launch_fir
    // Operand-form output instead of y (qmode != 0): piece 0 at q and piece 1
    // at q1, [F][ldq elements] each; qmode 1 block-scaled FP8 (E4M3 codes plus
    // E8M0 scales [F][W/32] at qs), 2 bf16, 3 bf16 hi + lo.
    uint8_t* q;
    uint8_t* q1;
    int64_t ldq;
    uint8_t* qs;
    int32_t qmode;
    // Per-frame scaled operand output (qmode 4 FP8 E4M3, 5 fp16, 6 fp16 hi +
    // lo): launch_fir first finds every frame's maximum (into amax), then its
    // exponent e_f (fexp[f], the frame's values are scaled by 2^-e_f), then
    // writes the scaled codes.
    int32_t* fexp;
};
// Chooses the vector width and unroll; returns the number of partial maxima
// per frame through a.nparts when a.amax is set.
hipError_t launch_fir(FirArgs& a, hipStream_t s);
// Number of partial maxima per frame launch_fir would produce.
int fir_amax_parts(const FirArgs& a);

// dst[i] = ext[start + i], i < count, where ext = prefix ++ chunk (floats).
hipError_t launch_gather_ext(const float* prefix, int64_t plen, const float* chunk, int64_t nchunk,
                             float* dst, int64_t start, int64_t count, hipStream_t s);

// ---------------------------------------------------------------------- GEMM
struct GemmArgs {
    const float* A;        // FIR output [F][K] FP32, row stride lda
    int64_t lda;
    const void* B0;        // Bt piece 0 [N][K]
    const void* B1;        // Bt piece 1 (split forms)
    float* out;            // output rows (floats), row stride ldo
    int64_t ldo;
    int64_t F;
    int32_t K, N;
    int32_t real_pack;     // real input: column 0 -> X_0, column 1 -> X_{P/2}, rest in place
    int32_t form;
    // A in operand form (every form but FP32, whose A is the FP32 rows
    // above): piece 0 / piece 1 [F][lda elements], and for FORM_MXFP8 the
    // E8M0 scales [F][K/32] (then B0/B1 = Bt codes / scales).
    const uint8_t* Aq;
    const uint8_t* Aq1;
    const uint8_t* Aqs;
    const int32_t* fexp;   // per-frame scaled forms with A in operand form: A row f carries 2^-fexp[f]
    int32_t compensated;   // FP32 only: compensated K accumulation (TwoSum per K tile)
    const float* tw;       // FP32 only, non-null: Bt assembled from this P x (cos, sin) twiddle table (B0 unused)
};
hipError_t launch_dft_gemm(const GemmArgs& a, hipStream_t s);
// The FIR fused into the FP32 GEMM (g.A unused; x describes the input stream
// and taps as for launch_fir, x.y unused).  fused_supported: FP32, M <= 16,
// W a multiple of 32, 16-byte aligned input with the prefix a whole number of
// float4s.
bool fused_supported(const FirArgs& x, int form);
hipError_t launch_dft_fused(const GemmArgs& g, const FirArgs& x, hipStream_t s);
// Forms whose A the FIR can write in operand form.
bool gemm_raw_form(int form);

// ------------------------------------------------------------- factored DFT
struct FftArgs {
    const float* y;        // FIR output [F][ldy] (P real or P complex values per frame)
    int64_t ldy;
    int64_t F;
    const float* mat1;     // realified DFT_{P1} (2 P1 x 2 P1)
    const float* mat3;     // realified DFT_{P2} (2 P2 x 2 P2); unused when P1 == P2
    const float* tw;       // cos, sin of 2 pi r / P
    float* out;            // output rows (complex64), row stride ldo floats
    int64_t ldo;
    int32_t P, cplx, cus;
};
bool fft_supported(int P);
void fft_factors(int P, int& P1, int& P2);
hipError_t launch_fft_tables(float* mat1, float* mat3, float* tw, int P, hipStream_t s);
// tw (P x 2): cos, sin of 2 pi r / P in FP64, rounded to FP32.
hipError_t launch_twiddle_table(float* tw, int P, hipStream_t s);
hipError_t launch_fft_dft(const FftArgs& a, hipStream_t s);
// One batch item's frames in a batched factored-DFT launch (device array,
// sorted by f0): FIR output rows y, output rows out, and the item's first
// frame among the launch's frames.
struct FftItem {
    const float* y;
    float* out;
    int64_t ldy, ldo, f0;
};
// Every frame of n items with the same P and input type (F frames in all);
// q64_ok: every y row is 16-byte aligned with ldy a multiple of 4 floats.
hipError_t launch_fft_batch(const FftItem* items, int n, int64_t F, int P, bool cplx, bool q64_ok, const float* mat1,
                            const float* mat3, const float* tw, int cus, hipStream_t s);

// --------------------------------------------------------------- batched path
// One item of a batched launch: the FIR and GEMM arguments of one stream
// chunk, its first work unit in each stage, and its state update.
struct BatchItem {
    FirArgs fir;            // fir.y points into the batch workspace
    GemmArgs gemm;          // gemm.A == fir.y
    int64_t fir_unit0;      // first FIR unit (256-thread block) of this item
    int64_t gemm_unit0;     // first GEMM tile of this item
    int64_t st_unit0;       // first state-update unit
    int32_t fir_tf;         // frames per FIR thread (fir_single: frames per frame-stage unit)
    int32_t fir_single;     // per-frame scaled form: one pass, whole frame rows per unit (frame stage)
    int64_t frame_unit0;    // first unit of the frame stage
    float* st_dst;          // state buffer to fill (nullptr: no state)
    int64_t st_start, st_count;
};

// Device-resident table read by the persistent kernels.  Each stage's units
// are split into 8 contiguous ranges of about equal cost, one per XCD.
struct BatchTable {
    int32_t n_items;
    int32_t pad_;
    int64_t fir_units, gemm_units, st_units, frame_units;
    int64_t fir_bounds[9], gemm_bounds[9], st_bounds[9], frame_bounds[9];
    int32_t gemm_bn;        // GEMM tile columns of this launch (kGemmBN or 2 * kGemmBN, or the wide tile's)
    int32_t gemm_wide;      // the launch uses the wide raw-operand tiles
    BatchItem items[1];     // n_items entries follow
};

// Index of the item that owns unit u of a stage (0 FIR, 1 GEMM, 2 state,
// 3 single-pass per-frame FIR):
// the last item whose first unit is <= u.
__device__ inline int batch_find(const BatchItem* items, int n, int64_t u, int stage) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t s = stage == 0 ? items[mid].fir_unit0
                          : stage == 1 ? items[mid].gemm_unit0
                          : stage == 2 ? items[mid].st_unit0
                                       : items[mid].frame_unit0;
        if (s <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// GEMM tile geometry shared with the batch planner.
constexpr int kGemmBM = 128, kGemmBN = 128;

// Per-frame scaled qmodes run three launches: partial maxima, per-frame
// exponents, scaled codes.
// frame_stage: per-frame scaled forms also launch the single-pass frame stage
// (the items flagged fir_single).
hipError_t launch_fir_batch(const BatchTable* t, int max_m, bool all_exact, int qmode, int grid, hipStream_t s,
                            bool frame_stage);
// Per-frame scaled items a batch runs in one pass (whole frame rows of 1024
// threads): the floats per thread, or 0 (three launches).  A unit walks the
// item's fir_tf frames (a whole number of ring blocks of M).
int fir_frame_batch_vec(const FirArgs& a);
// FirArgs::qmode the FIR writes for a DFT form (0: FP32 y): every form but
// FP32 takes its operand straight from the FIR.
inline int form_fir_qmode(int form) {
    switch (form) {
        case FORM_MXFP8: return 1;
        case FORM_BF16: return 2;
        case FORM_BF16X3: return 3;
        case FORM_FP8: return 4;
        case FORM_FP16: return 5;
        case FORM_FP16X3: return 6;
        default: return 0;
    }
}
// qmode values whose codes carry a per-frame scale.
inline bool qmode_frame_scaled(int qm) { return qm >= 4 && qm <= 6; }

// Per-frame scale 2^e with the frame's largest |y| * 2^-e <= limit (448 for
// FP8 E4M3, 32768 for fp16); 0 for a zero or non-finite maximum.
__device__ inline int frame_exponent(float amax, float limit) {
    if (!(amax > 0.0f) || !isfinite(amax)) return 0;
    int e;
    frexpf(amax / limit, &e);  // amax/limit in [2^(e-1), 2^e)
    while (e > -120 && ldexpf(limit, e - 1) >= amax) --e;
    while (e < 120 && ldexpf(limit, e) < amax) ++e;
    return e;
}
// tile_n: the table's GEMM tile columns (kGemmBN for every form; 2 * kGemmBN
// also for FP32 with A in FP32).
// wide: A in operand form on the single-stream path's wide tiles (every
// item's K a whole number of their K tiles; gemm_batch_wide_tile).
hipError_t launch_gemm_batch(const BatchTable* t, int form, bool raw, int tile_n, int grid, hipStream_t s,
                             bool wide = false);
// The wide raw-operand tile (bm x bn) of `form`, if it serves an operand of K
// columns (K a whole number of its K tiles); false for FP32 and other K.
bool gemm_batch_wide_tile(int form, int K, int& bm, int& bn);
hipError_t launch_gather_batch(const BatchTable* t, int grid, hipStream_t s);

}  // namespace tina
