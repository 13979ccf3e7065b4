/*
 * FP64 CPU oracle for the polyphase filter bank (PFB) channelizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * GPU library and is deliberately plain: direct sums in double precision, in
 * the order the paper states them, parallelised only across frames.
 *
 * What it computes (paper: TINA, arXiv 2408.16551):
 *   - the prototype window h (the paper only says the taps are divided
 *     between the P branches, Sec. 5.2; the sinc x window family is the
 *     workload's choice, see oracle_window);
 *   - the polyphase FIR of Eq. (20): y_p(n') = sum_{m=0}^{M-1} h_p(m) x_p(n'-m),
 *     a causal FIR per branch (Sec. 4.3, Eq. (15));
 *   - the DFT across branches of each frame, Z = X F with F the Fourier
 *     matrix (Sec. 4.1, Eq. (12)), forward sign, unnormalised;
 *   - the unfolding (sliding-window) operation Y(i, j) = X(i*stride + j)
 *     (Sec. 4.4, Eq. (17), stride 1 in the paper);
 *   - the inverse DFT of Sec. 4.2, Eq. (14);
 *   - a block-scaled FP8 form of the DFT (see oracle_mx_dft).
 *
 * Readings taken where the paper is silent:
 *   branch p of frame f holds x[f*P + p];
 *   tap m of branch p is h[(M-1-m)*P + p]  (m counts back from the newest frame);
 *   history before the first frame is zero unless supplied;
 *   a real input yields the P/2+1 non-redundant channels, a complex input P.
 *
 * Precision: every sample is promoted exactly to double; every sum is a
 * double-precision sum in ascending index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/*
 * ORACLE_MUTATION plants one known mistake (tests only: they compile such
 * variants into a temporary directory to show that the pins catch each one).
 * The default build defines none.
 */
#ifndef ORACLE_MUTATION
#define ORACLE_MUTATION 0
#endif

enum { OR_WIN_RECT = 0, OR_WIN_HANN = 1, OR_WIN_HAMMING = 2, OR_WIN_BLACKMAN = 3 };

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops that follow (n >= 1); for timing only. */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * cos(2*pi*r/P) and sin(2*pi*r/P) for an integer r, with r reduced modulo P
 * in integer arithmetic first.  The angle is split into a whole number of
 * quarter turns q and a remainder phi in [0, pi/2), so that multiples of a
 * quarter turn come out as exact 0 and +-1.
 */
void oracle_twiddle(int64_t r, int64_t P, double* c, double* s) {
    r %= P;
    if (r < 0) r += P;
    int64_t n = 4 * r;              /* angle = (pi/2) * n / P */
    int64_t q = n / P;              /* whole quarter turns, 0..3 */
    int64_t rem = n - q * P;        /* remainder, 0 <= rem < P */
    double phi = (M_PI / 2.0) * ((double)rem / (double)P);
    double cp = (rem == 0) ? 1.0 : cos(phi);
    double sp = (rem == 0) ? 0.0 : sin(phi);
    switch (q) {
        case 0: *c = cp;  *s = sp;  break;
        case 1: *c = -sp; *s = cp;  break;
#if ORACLE_MUTATION == 4
        case 2: *c = -sp; *s = -cp; break; /* planted: wrong quadrant rotation */
#else
        case 2: *c = -cp; *s = -sp; break;
#endif
        default: *c = sp; *s = -cp; break;
    }
}

/* sin(pi t) / (pi t), equal to 1 at t = 0. */
static double sinc(double t) {
    if (t == 0.0) return 1.0;
    return sin(M_PI * t) / (M_PI * t);
}

/*
 * Prototype low-pass filter of length L = P*M:
 *   h[n] = sinc((n - (L-1)/2) / P) * w[n],  n = 0..L-1,
 * a sinc with cutoff 1/(2P) cycles/sample centred on the filter, times a
 * symmetric window over L points (denominator L-1).  No normalisation.
 */
int oracle_window(int64_t P, int64_t M, int kind, double* h) {
    if (P < 1 || M < 1 || !h) return -1;
    int64_t L = P * M;
#if ORACLE_MUTATION == 5
    double centre = (double)L / 2.0; /* planted: window off-centre */
#else
    double centre = (double)(L - 1) / 2.0;
#endif
    for (int64_t n = 0; n < L; ++n) {
        double w;
        double a = (L > 1) ? 2.0 * M_PI * (double)n / (double)(L - 1) : 0.0;
        switch (kind) {
            case OR_WIN_RECT: w = 1.0; break;
            case OR_WIN_HANN: w = (L > 1) ? 0.5 - 0.5 * cos(a) : 1.0; break;
            case OR_WIN_HAMMING: w = (L > 1) ? 0.54 - 0.46 * cos(a) : 1.0; break;
            case OR_WIN_BLACKMAN:
                w = (L > 1) ? 0.42 - 0.5 * cos(a) + 0.08 * cos(2.0 * a) : 1.0;
                break;
            default: return -1;
        }
        h[n] = sinc(((double)n - centre) / (double)P) * w;
    }
    return 0;
}

/*
 * Unfolding (sliding window): Y[i][j] = x[i*stride + j] for
 * i = 0 .. (I-J)/stride, j = 0 .. J-1.  With stride 1 this is the paper's
 * Eq. (17); the frame window of the filter bank is the same operation with
 * stride P and width P*M.
 */
int64_t oracle_unfold(const double* x, int64_t I, int64_t J, int64_t stride, double* Y) {
    if (I < J || J < 1 || stride < 1) return 0;
    int64_t rows = (I - J) / stride + 1;
    if (Y) {
        for (int64_t i = 0; i < rows; ++i)
            for (int64_t j = 0; j < J; ++j) Y[i * J + j] = x[i * stride + j];
    }
    return rows;
}

/*
 * Polyphase FIR, Eq. (20), for the frames listed in `frames` (or all frames
 * 0..nframes-1 when `frames` is NULL).
 *
 * x_ext holds (M-1)*P history samples followed by the framed signal; a
 * sample is one double (real) or two doubles re, im (complex).  Frame f of
 * the framed signal starts at x_ext sample (f + M - 1) * P.
 *   y[f][p] = sum_{m=0}^{M-1} h[(M-1-m)*P + p] * x_ext[(f - m + M - 1)*P + p]
 * Output y: one row of P samples per requested frame.
 */
static void fir_frame(int64_t P, int64_t M, int cplx, const double* h, const double* x_ext,
                      int64_t f, double* y) {
    int cf = cplx ? 2 : 1;
    for (int64_t p = 0; p < P; ++p) {
        for (int c = 0; c < cf; ++c) {
            double acc = 0.0;
#if ORACLE_MUTATION == 1
            for (int64_t m = 0; m < M - 1; ++m) { /* planted: oldest tap dropped */
#else
            for (int64_t m = 0; m < M; ++m) {
#endif
#if ORACLE_MUTATION == 2
                double tap = h[m * P + p]; /* planted: taps not reversed */
#else
                double tap = h[(M - 1 - m) * P + p];
#endif
                double xv = x_ext[((f - m + M - 1) * P + p) * cf + c];
                acc += tap * xv;
            }
            y[p * cf + c] = acc;
        }
    }
}

/*
 * DFT across branches of one frame (Sec. 4.1, Eq. (12): Z = X F with
 * F[p][k] = exp(-2 pi i p k / P)):
 *   X[k] = sum_{p=0}^{P-1} y[p] (cos t - i sin t),  t = 2 pi ((p k) mod P) / P.
 * Channels k = 0..P/2 for a real frame, k = 0..P-1 for a complex frame.
 * `tw` holds cos/sin of 2 pi r / P for r = 0..P-1 (oracle_twiddle values);
 * (p k) mod P is carried exactly in integers as p increases.
 */
static void dft_frame(int64_t P, int cplx, const double* tw, const double* y, double* X) {
    int64_t K = cplx ? P : P / 2 + 1;
    for (int64_t k = 0; k < K; ++k) {
        double re = 0.0, im = 0.0;
        int64_t r = 0; /* (p * k) mod P */
        for (int64_t p = 0; p < P; ++p) {
            double c = tw[2 * r], s = tw[2 * r + 1];
            if (cplx) {
                double a = y[2 * p], b = y[2 * p + 1];
#if ORACLE_MUTATION == 7
                re += a * c - b * s; /* planted: sign of the cross term */
#else
                re += a * c + b * s;
#endif
                im += b * c - a * s;
            } else {
                double a = y[p];
                re += a * c;
#if ORACLE_MUTATION == 3
                im += a * s; /* planted: conjugated twiddle */
#else
                im -= a * s;
#endif
            }
#if ORACLE_MUTATION == 6
            r += k + (p == P / 2); /* planted: phase index slips once */
            while (r >= P) r -= P;
#else
            r += k;
            if (r >= P) r -= P;
#endif
        }
        X[2 * k] = re;
        X[2 * k + 1] = im;
    }
}

static double* twiddle_table(int64_t P) {
    double* tw = (double*)malloc(sizeof(double) * 2 * (size_t)P);
    if (!tw) return NULL;
    for (int64_t r = 0; r < P; ++r) oracle_twiddle(r, P, &tw[2 * r], &tw[2 * r + 1]);
    return tw;
}

int oracle_fir(int64_t P, int64_t M, int cplx, const double* h, const double* x_ext,
               int64_t n_ext, int64_t nframes, const int64_t* frames, double* y) {
    if (P < 1 || M < 1 || !h || !x_ext || !y) return -1;
    int64_t avail = (n_ext - (M - 1) * P) / P;
    int cf = cplx ? 2 : 1;
    for (int64_t i = 0; i < nframes; ++i) {
        int64_t f = frames ? frames[i] : i;
        if (f < 0 || f >= avail) return -2;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nframes; ++i) {
        int64_t f = frames ? frames[i] : i;
        fir_frame(P, M, cplx, h, x_ext, f, y + i * P * cf);
    }
    return 0;
}

int oracle_dft(int64_t P, int cplx, const double* y, int64_t nframes, double* X) {
    if (P < 2 || !y || !X) return -1;
    double* tw = twiddle_table(P);
    if (!tw) return -3;
    int cf = cplx ? 2 : 1;
    int64_t K = cplx ? P : P / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nframes; ++i) dft_frame(P, cplx, tw, y + i * P * cf, X + i * K * 2);
    free(tw);
    return 0;
}

/*
 * Inverse DFT of each frame (Sec. 4.2, Eq. (14): X = Z IF, the inverse
 * Fourier matrix): v[p] = (1/P) sum_{k=0}^{P-1} X[k] (cos t + i sin t),
 * t = 2 pi ((p k) mod P) / P.  Complex in, complex out (re, im doubles).
 */
int oracle_idft(int64_t P, const double* X, int64_t nframes, double* v) {
    if (P < 1 || !X || !v) return -1;
    double* tw = twiddle_table(P);
    if (!tw) return -3;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nframes; ++f) {
        const double* Xf = X + f * P * 2;
        double* vf = v + f * P * 2;
        for (int64_t p = 0; p < P; ++p) {
            double re = 0.0, im = 0.0;
            int64_t r = 0; /* (k * p) mod P */
            for (int64_t k = 0; k < P; ++k) {
                double c = tw[2 * r], s = tw[2 * r + 1];
                double a = Xf[2 * k], b = Xf[2 * k + 1];
                re += a * c - b * s;
                im += a * s + b * c;
                r += p;
                if (r >= P) r -= P;
            }
            vf[2 * p] = re / (double)P;
            vf[2 * p + 1] = im / (double)P;
        }
    }
    free(tw);
    return 0;
}

/*
 * The filter bank: for each requested frame, the polyphase FIR of Eq. (20)
 * followed by the DFT across its P branches.  Output X: K complex values
 * (re, im doubles) per requested frame.  If y_out is not NULL the FIR output
 * of each requested frame is stored there too.
 */
int oracle_pfb(int64_t P, int64_t M, int cplx, const double* h, const double* x_ext,
               int64_t n_ext, int64_t nframes, const int64_t* frames, double* X, double* y_out) {
    if (P < 2 || M < 1 || !h || !x_ext || !X) return -1;
    int64_t avail = (n_ext - (M - 1) * P) / P;
    for (int64_t i = 0; i < nframes; ++i) {
        int64_t f = frames ? frames[i] : i;
        if (f < 0 || f >= avail) return -2;
    }
    double* tw = twiddle_table(P);
    if (!tw) return -3;
    int cf = cplx ? 2 : 1;
    int64_t K = cplx ? P : P / 2 + 1;
    int failed = 0;
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * (size_t)(P * cf));
        if (!y) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < nframes; ++i) {
                int64_t f = frames ? frames[i] : i;
                fir_frame(P, M, cplx, h, x_ext, f, y);
                dft_frame(P, cplx, tw, y, X + i * K * 2);
                if (y_out) memcpy(y_out + i * P * cf, y, sizeof(double) * (size_t)(P * cf));
            }
            free(y);
        }
    }
    free(tw);
    return failed ? -3 : 0;
}

/*
 * Block-scaled FP8 DFT (a quantised form of the DFT of Sec. 4.1, Eq. (12);
 * the paper names quantisation as one of the NN-side optimisations the
 * mapping opens up, Sec. 1).  No precision is fixed by the paper; this is the
 * definition the GPU's block-scaled form is held to:
 *
 *   - FP8 E4M3 (OCP): 1 sign, 4 exponent (bias 7), 3 mantissa bits; normals
 *     2^-6 .. 448, subnormals in steps of 2^-9; rounding to nearest, ties to
 *     even; magnitudes above 448 saturate to 448.
 *   - Blocks: 32 consecutive entries of a real vector (the last block may be
 *     shorter).  Each block gets one power-of-two scale 2^e, e the smallest
 *     integer in [-127, 127] with max|v| <= 448 * 2^e (e = 0 for an all-zero
 *     block), and each entry becomes 2^e * E4M3(v * 2^-e).
 *   - The DFT of one frame is written as real dot products over the frame's
 *     real vector (K = P reals, or K = 2P interleaved re, im for a complex
 *     frame): Re X_k and Im X_k each have their own coefficient vector
 *     (cos t / -sin t for a real frame; (cos t, sin t) and (-sin t, cos t)
 *     per branch for a complex one, t = 2 pi pk/P).  The frame vector and
 *     every coefficient vector are block-quantised as above, and each output
 *     is the exact sum of the products of the quantised entries.
 */
double oracle_e4m3(double v) {
    if (v != v || v == 0.0) return v;
    double a = fabs(v);
    if (a >= 448.0) return copysign(448.0, v);
    int E;
    frexp(a, &E);                   /* a = m * 2^E, m in [0.5, 1): binade 2^(E-1) */
    int eb = E - 1;
    if (eb < -6) eb = -6;           /* subnormals share the spacing of the lowest binade */
    double q = ldexp(1.0, eb - 3);  /* grid spacing: 3 mantissa bits */
    double r = nearbyint(a / q) * q;
    if (r > 448.0) r = 448.0;
    return copysign(r, v);
}

int oracle_mx_exponent(double amax) {
    if (!(amax > 0.0) || isinf(amax)) return 0;
    int e = -127;
    while (e < 127 && ldexp(448.0, e) < amax) ++e;
#if ORACLE_MUTATION == 9
    if (e > -127) --e; /* planted: scale one binade too small (saturates) */
#endif
    return e;
}

/* Block-quantised copy of v[0..n): out[j] = 2^e * E4M3(v[j] * 2^-e). */
int oracle_mx_quantize(const double* v, int64_t n, double* out) {
    if (n < 0 || (n > 0 && (!v || !out))) return -1;
    for (int64_t b = 0; b < n; b += 32) {
        int64_t end = b + 32 < n ? b + 32 : n;
        double amax = 0.0;
        for (int64_t j = b; j < end; ++j)
            if (fabs(v[j]) > amax) amax = fabs(v[j]);
        int e = oracle_mx_exponent(amax);
        for (int64_t j = b; j < end; ++j) out[j] = ldexp(oracle_e4m3(ldexp(v[j], -e)), e);
    }
    return 0;
}

int oracle_mx_dft(int64_t P, int cplx, const double* y, int64_t nframes, double* X) {
    if (P < 2 || nframes < 0 || (nframes > 0 && (!y || !X))) return -1;
    int cf = cplx ? 2 : 1;
    int64_t Kin = P * cf, Kout = cplx ? P : P / 2 + 1;
    double* tw = twiddle_table(P);
    double* yq = (double*)malloc(sizeof(double) * (size_t)(Kin * (nframes > 0 ? nframes : 1)));
    if (!tw || !yq) {
        free(tw);
        free(yq);
        return -3;
    }
    for (int64_t f = 0; f < nframes; ++f) oracle_mx_quantize(y + f * Kin, Kin, yq + f * Kin);
    int failed = 0;
#pragma omp parallel
    {
        double* w = (double*)malloc(sizeof(double) * 4 * (size_t)Kin);
        if (!w) {
#pragma omp atomic write
            failed = 1;
        } else {
            double *wr = w, *wi = w + Kin, *qr = w + 2 * Kin, *qi = w + 3 * Kin;
#pragma omp for schedule(dynamic, 4)
            for (int64_t k = 0; k < Kout; ++k) {
                int64_t r = 0; /* (p * k) mod P */
                for (int64_t p = 0; p < P; ++p) {
                    double c = tw[2 * r], s = tw[2 * r + 1];
                    if (cplx) {
                        wr[2 * p] = c;
                        wr[2 * p + 1] = s;
                        wi[2 * p] = -s;
                        wi[2 * p + 1] = c;
                    } else {
                        wr[p] = c;
                        wi[p] = -s;
                    }
                    r += k;
                    if (r >= P) r -= P;
                }
#if ORACLE_MUTATION == 8
                memcpy(qr, wr, sizeof(double) * (size_t)Kin); /* planted: coefficients left unquantised */
                memcpy(qi, wi, sizeof(double) * (size_t)Kin);
#else
                oracle_mx_quantize(wr, Kin, qr);
                oracle_mx_quantize(wi, Kin, qi);
#endif
                for (int64_t f = 0; f < nframes; ++f) {
                    const double* a = yq + f * Kin;
                    double re = 0.0, im = 0.0;
                    for (int64_t j = 0; j < Kin; ++j) {
                        re += a[j] * qr[j];
                        im += a[j] * qi[j];
                    }
                    X[(f * Kout + k) * 2] = re;
                    X[(f * Kout + k) * 2 + 1] = im;
                }
            }
            free(w);
        }
    }
    free(tw);
    free(yq);
    return failed ? -3 : 0;
}
