/*
 * oracle_rda.c -- plain, slow FP64 CPU oracle for the SAR Range Doppler
 * Algorithm (RDA).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library and its binding) never calls it, and the two share no code,
 * header, table or constant generator.
 *
 * Everything is double precision (C99 `double complex`), row-major,
 * interleaved (re, im).  Parallelism: OpenMP over independent lines only;
 * each line is computed exactly as the serial definition says.
 *
 * Paper: "From 8 Seconds to 370 ms: Kernel-Fused SAR Imaging on Apple
 * Silicon via Single-Dispatch FFT Pipelines" (arXiv 2604.03585).
 *   Sec. II.B  -- per-line FFT -> matched-filter multiply -> IFFT;
 *   Sec. II.C  -- IFFT(x) = (1/N) conj(FFT(conj(x)));
 *   Sec. IV.A  -- the RDA steps: range compression, azimuth FFT, RCMC by sinc
 *                interpolation in the range-Doppler domain, azimuth
 *                compression (multiply by H_a(f_a, R0), then IFFT).
 * The paper defines neither filter nor the RCMC kernel; the readings used
 * here (replica matched filters, exact-geometry azimuth phase, 8-tap
 * Kaiser-windowed sinc) are stated at each function below.
 *
 * Parity status of each function is stated in its comment; every one is
 * pinned by a CPU test against a closed form, brute force, or an invariant.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846264338327950288

/* Planted-mistake hooks for the pin-strength tests.  A normal build has
 * ORC_MUTANT == 0 and every MUT(k) is a compile-time false; the tests build
 * copies with -DORC_MUTANT=k to check that some pin catches mistake k. */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif
#define MUT(k) (ORC_MUTANT == (k))

/* ------------------------------------------------------------------ */
/* O1. FFT: iterative radix-2 decimation-in-time with a bit-reversal   */
/* permutation.  Forward is X[k] = sum_n x[n] exp(-2 pi i k n / N),    */
/* unnormalised.  Twiddles exp(-2 pi i j / len) come straight from     */
/* cos/sin of the index, with no recurrence.                           */
/* Pinned: brute-force DFT, Parseval, impulse, CAZAC chirp, long-      */
/* double single bins, round trip.                                     */
/* ------------------------------------------------------------------ */
static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

static void fft_forward(cplx* x, int n)
{
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j && !MUT(2)) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2;
        for (int j = 0; j < half; ++j) {
            double ang = (MUT(1) ? 2.0 : -2.0) * ORC_PI * (double)j / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (int b = 0; b < n; b += len) {
                cplx u = x[b + j];
                cplx v = x[b + j + half] * w;
                x[b + j] = u + v;
                x[b + j + half] = u - v;
            }
        }
    }
}

/* Sec. II.C: IFFT(x) = (1/N) conj(FFT(conj(x))). */
static void fft_inverse(cplx* x, int n)
{
    for (int i = 0; i < n; ++i) x[i] = conj(x[i]);
    fft_forward(x, n);
    double s = MUT(3) ? 1.0 : 1.0 / (double)n;
    for (int i = 0; i < n; ++i) x[i] = conj(x[i]) * s;
}

int orc_fft(double* x, int n, int inverse)
{
    if (!x || !is_pow2(n)) return 1;
    if (inverse) fft_inverse((cplx*)x, n);
    else fft_forward((cplx*)x, n);
    return 0;
}

/* ------------------------------------------------------------------ */
/* O2. Matched filter (Sec. II.B step 3, Sec. IV.A step 1; H_r is not  */
/* defined in the paper).  Replica h[(u mod N)] = exp(sign*j*pi*K*u^2) */
/* for u = -L/2 .. L/2-1 (K = tbp / L^2), zero elsewhere; the filter   */
/* is H = conj(FFT(h)).  sign = +1 for the up-chirp range replica,     */
/* -1 for the down-chirp azimuth replica of the zero-migration model.  */
/* Pinned: full-length CAZAC chirp compresses to N*delta; for L < N    */
/* the compressed replica equals its direct circular autocorrelation.  */
/* ------------------------------------------------------------------ */
int orc_matched_filter(int n, int len, double tbp, int sign, double* H)
{
    if (!H || !is_pow2(n) || len < 1 || len > n) return 1;
    cplx* h = (cplx*)H;
    double K = tbp / ((double)len * (double)len);
    for (int i = 0; i < n; ++i) h[i] = 0.0;
    for (int u = -len / 2 + MUT(5); u < len - len / 2 + MUT(5); ++u) {
        double ph = (double)sign * ORC_PI * K * (double)u * (double)u;
        int idx = ((u % n) + n) % n;
        h[idx] = cos(ph) + I * sin(ph);
    }
    fft_forward(h, n);
    if (!MUT(4))
        for (int i = 0; i < n; ++i) h[i] = conj(h[i]);
    return 0;
}

/* One line: y = IFFT(FFT(x) * H)  (Sec. II.B, steps 2-4). */
static void compress_line(cplx* x, const cplx* H, int n)
{
    fft_forward(x, n);
    for (int i = 0; i < n; ++i) x[i] *= H[i];
    fft_inverse(x, n);
}

/* Range compression of every range line [m][:] (Sec. IV.A step 1).
 * in, out: [rows][n] complex; in == out allowed. */
int orc_compress_rows(const double* in, int rows, int n, const double* H, double* out)
{
    if (!in || !out || !H || !is_pow2(n) || rows < 0) return 1;
    if (out != in) memmove(out, in, sizeof(cplx) * (size_t)rows * (size_t)n);
    cplx* o = (cplx*)out;
    const cplx* h = (const cplx*)H;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) compress_line(o + (size_t)r * n, h, n);
    return 0;
}

/* Forward FFT of every row (azimuth FFT once data is [range][azimuth]). */
int orc_fft_rows(const double* in, int rows, int n, double* out)
{
    if (!in || !out || !is_pow2(n) || rows < 0) return 1;
    if (out != in) memmove(out, in, sizeof(cplx) * (size_t)rows * (size_t)n);
    cplx* o = (cplx*)out;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) fft_forward(o + (size_t)r * n, n);
    return 0;
}

/* O3. Corner turn: out[c][r] = in[r][c].  Pinned: exact permutation. */
int orc_corner_turn(const double* in, int rows, int cols, double* out)
{
    if (!in || !out || in == out || rows < 0 || cols < 0) return 1;
    const cplx* a = (const cplx*)in;
    cplx* b = (cplx*)out;
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c)
            b[MUT(6) ? (size_t)r * cols + c : (size_t)c * rows + r] = a[(size_t)r * cols + c];
    return 0;
}

/* ------------------------------------------------------------------ */
/* O4b. RCMC kernel (Sec. IV.A step 3, "sinc interpolation"; taps,     */
/* window and alignment are our reading): 8 taps t = -3..4 about       */
/* floor(p), x = p - floor(p),                                         */
/*   K(z) = sinc(z) * I0(beta*sqrt(1-(z/4)^2)) / I0(beta), |z| <= 4,   */
/*   w_t(x) = K(t - x) / sum_t' K(t' - x).                             */
/* Pinned: I0 against known values and an independent library; x = 0  */
/* gives the identity; weights sum to 1; fractional shift of a         */
/* band-limited tone; the normalised weights at x = 1/10, 1/4, 1/2,    */
/* 3/4 against a library Kaiser window times a library sinc.           */
/* ------------------------------------------------------------------ */
double orc_bessel_i0(double y)
{
    /* I0(y) = sum_k ((y/2)^k / k!)^2, summed until the terms vanish. */
    double q = 0.25 * y * y, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / (MUT(11) ? (double)k : (double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

static double sinc(double z)
{
    if (z == 0.0) return 1.0;
    return sin(ORC_PI * z) / (ORC_PI * z);
}

static double kaiser_sinc(double z, double beta, double half)
{
    if (fabs(z) > half) return 0.0;
    double r = z / half;
    double b = MUT(13) ? 2.0 * beta : (MUT(15) ? 0.0 : beta);
    double s = MUT(14) ? sqrt(1.0 - fabs(r)) : sqrt(1.0 - r * r);
    return sinc(z) * orc_bessel_i0(b * s) / orc_bessel_i0(b);
}

/* w[0..taps-1] for t = -(taps/2 - 1) .. taps/2. */
int orc_rcmc_weights(double x, double beta, int taps, double* w)
{
    if (!w || taps < 2 || taps > 64 || (taps & 1)) return 1;
    double half = 0.5 * taps, sum = 0.0;
    for (int i = 0; i < taps; ++i) {
        int t = i - (taps / 2 - 1);
        w[i] = kaiser_sinc((double)t - x + (MUT(8) ? 1.0 : 0.0), beta, half);
        sum += w[i];
    }
    if (!MUT(7))
        for (int i = 0; i < taps; ++i) w[i] /= sum;
    return 0;
}

/* ------------------------------------------------------------------ */
/* O4b. Exact-geometry quantities per Doppler bin k (PRF = 1, fftfreq  */
/* ordering, broadside):  f_k = k/Na (k < Na/2) else (k-Na)/Na,        */
/* D_k = sqrt(1 - (lam f_k / (2 V))^2).                                */
/* ------------------------------------------------------------------ */
static double doppler_D(int k, int na, double lam, double v)
{
    double f = (k < na / 2 || MUT(12)) ? (double)k / na : (double)(k - na) / na;
    double xk = lam * f / (2.0 * v);
    return sqrt(1.0 - xk * xk);
}

/* ------------------------------------------------------------------ */
/* O4b. RCMC + azimuth compression, data laid out [range n][Doppler k] */
/* (Sec. IV.A steps 3-4).  For each output range cell n, Doppler k:    */
/*   R0 = r_near + n,  p = n + R0 (1/D_k - 1),  i0 = floor(p),         */
/*   y = sum_t A[i0+t][k] w_t(p - i0)   (rows outside [0, Nr) -> 0),   */
/*   Y = y * exp(+j 4 pi R0 D_k / lam),                                */
/* then the azimuth IFFT over k.  taps == 0 skips the interpolation.   */
/* Pinned: RCMC identity / integer shift, a synthetic range-Doppler    */
/* pulse moved back to R0, and a noise-free hyperbolic point target    */
/* focused at its seeded cell.                                         */
/* ------------------------------------------------------------------ */
int orc_rcmc_azimuth(const double* A_in, int nr, int na, double lam, double v,
                     double r_near, int taps, double beta, double* out)
{
    if (!A_in || !out || A_in == out || !is_pow2(na) || nr < 1) return 1;
    if (taps != 0 && (taps < 2 || taps > 64 || (taps & 1))) return 1;
    if (!(lam > 0.0) || !(v > 0.0)) return 1;
    const cplx* A = (const cplx*)A_in;
    cplx* O = (cplx*)out;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < nr; ++n) {
        double w[64];
        cplx* row = O + (size_t)n * na;
        double R0 = r_near + (double)n;
        for (int k = 0; k < na; ++k) {
            double D = doppler_D(k, na, lam, v);
            cplx y;
            if (taps == 0) {
                y = A[(size_t)n * na + k];
            } else {
                double p = (double)n + (MUT(9) ? -R0 : R0) * (1.0 / D - 1.0);
                double i0 = floor(p);
                orc_rcmc_weights(p - i0, beta, taps, w);
                y = 0.0;
                for (int i = 0; i < taps; ++i) {
                    long r = (long)i0 + (i - (taps / 2 - 1));
                    if (r >= 0 && r < nr) y += A[(size_t)r * na + k] * w[i];
                }
            }
            double ph = (MUT(10) ? -4.0 : 4.0) * ORC_PI * R0 * D / lam;
            row[k] = y * (cos(ph) + I * sin(ph));
        }
        fft_inverse(row, na);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The whole RDA (Sec. IV.A).  raw: complex64 [Na][Nr] (promoted to    */
/* FP64); img: complex128 [Na][Nr].                                    */
/*   az_model 0 (LFM, zero migration): range compression, corner turn, */
/*     per-azimuth-line FFT * H_a * IFFT with the down-chirp replica;  */
/*   az_model 1 (hyperbolic): range compression, corner turn, azimuth  */
/*     FFT, RCMC + exact-geometry phase + IFFT.                        */
/* The result is turned back to [Na][Nr].                              */
/* ------------------------------------------------------------------ */
int orc_rda(const float* raw, int na, int nr, int range_len, double range_tbp,
            int az_model, int az_len, double az_tbp, double lam, double v,
            double r_near, int taps, double beta, double* img)
{
    if (!raw || !img || !is_pow2(na) || !is_pow2(nr)) return 1;
    size_t px = (size_t)na * (size_t)nr;
    double* a = (double*)malloc(sizeof(cplx) * px);
    double* b = (double*)malloc(sizeof(cplx) * px);
    double* Hr = (double*)malloc(sizeof(cplx) * (size_t)nr);
    double* Ha = (double*)malloc(sizeof(cplx) * (size_t)na);
    int rc = 1;
    if (!a || !b || !Hr || !Ha) goto done;
    for (size_t i = 0; i < 2 * px; ++i) a[i] = (double)raw[i];

    if (orc_matched_filter(nr, range_len, range_tbp, +1, Hr)) goto done;
    if (orc_compress_rows(a, na, nr, Hr, a)) goto done;       /* [Na][Nr] */
    if (orc_corner_turn(a, na, nr, b)) goto done;             /* [Nr][Na] */
    if (az_model == 0) {
        if (orc_matched_filter(na, az_len, az_tbp, -1, Ha)) goto done;
        if (orc_compress_rows(b, nr, na, Ha, b)) goto done;
    } else if (az_model == 1) {
        if (orc_fft_rows(b, nr, na, a)) goto done;            /* A[Nr][Na] */
        if (orc_rcmc_azimuth(a, nr, na, lam, v, r_near, taps, beta, b)) goto done;
    } else {
        goto done;
    }
    if (orc_corner_turn(b, nr, na, img)) goto done;           /* [Na][Nr] */
    rc = 0;
done:
    free(a); free(b); free(Hr); free(Ha);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
