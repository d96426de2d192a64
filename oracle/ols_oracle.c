/*
 * ols_oracle.c -- FP64 reference for overlap-save (OLS) variable-bandwidth
 * filtering with HFSO filter DFT coefficients.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Paper: O. Moryakova, H. Johansson, "Efficient Design and Implementation of
 * Fast-Convolution-Based Variable-Bandwidth Filters" (arXiv 2406.14116).
 *
 * Everything is the literal definition, in double precision, with no FFT:
 *   - Sec. II, OLS steps 1-5: the input is cut into N-sample segments that
 *     advance by M samples (M is called `hop` here), each segment goes through
 *     an N-point DFT, a multiply by H(k), an N-point IDFT, the first N-M
 *     samples are dropped and the M-sample pieces are concatenated.
 *   - Sec. III-B, eq. (5): H(k,b) = H_R(k,b) exp(-j 2 pi k (L-1)/2 / N), with
 *     the effective filter length L = N - M + 1, so (L-1)/2 = (N-M)/2 = D.
 *   - Sec. III-B, eq. (6): H_R is 1 on the passband bins, V(k-k1) on the
 *     transition bins and 0 on the stopband bins, with the bin sets
 *     k_p = [0,k1-1] u [N-k1+1,N-1], k_t = [k1,k2] u [N-k2,N-k1],
 *     k_s = [k2+1, N-k2-1] and k2 = k1 + L_V - 1 (eq. (7) with L_V = Delta_N-1).
 *   - Sec. III-A, eq. (4): the inverse transform carries +j in the exponent and
 *     the factor 1/N.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *   - framing: segment m starts at m*M - (N-M), i.e. the stream is preceded by
 *     N-M zeros of history, samples outside [0,len) read as 0, and output
 *     sample m*M + j is z_m(N-M+j).  Output length equals input length.
 *   - mirrored transition bins: H_R(N-k) = H_R(k), i.e. the bins
 *     [N-k2, N-k1] carry V(N-k-k1).  This is the value that makes the impulse
 *     response real, which the paper states for the closed form, eq. (8).
 *   - the delay D = (N-M)/2 must be an integer (N-M even).
 *   - a bandwidth change is given as a schedule of (from_block, k1) pairs;
 *     block m uses the pair with the largest from_block <= m.
 *
 * All functions return 0 on success and a negative value on bad arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_EINVAL (-1)

static const double kTwoPi = 6.283185307179586476925286766559;

/* w[r] = exp(-j 2 pi r / n) = cos(2 pi r/n) - j sin(2 pi r/n), r in [0,n). */
static int make_twiddles(int n, double **wr, double **wi)
{
    *wr = (double *)malloc(sizeof(double) * (size_t)n);
    *wi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!*wr || !*wi) {
        free(*wr);
        free(*wi);
        return ORACLE_EINVAL;
    }
    for (int r = 0; r < n; ++r) {
        double a = kTwoPi * (double)r / (double)n;
        (*wr)[r] = cos(a);
        (*wi)[r] = -sin(a);
    }
    return 0;
}

/* Forward N-point DFT, Sec. II step 1:  X(k) = sum_i s(i) w[(i k) mod n].
 * Arrays hold n interleaved (re, im) pairs. */
static void dft_direct(int n, const double *wr, const double *wi,
                       const double *s, double *X)
{
    for (int k = 0; k < n; ++k) {
        double accr = 0.0, acci = 0.0;
        for (int i = 0; i < n; ++i) {
            int64_t r = ((int64_t)i * (int64_t)k) % n;
            double sr = s[2 * i], si = s[2 * i + 1];
            accr += sr * wr[r] - si * wi[r];
            acci += sr * wi[r] + si * wr[r];
        }
        X[2 * k] = accr;
        X[2 * k + 1] = acci;
    }
}

/* Inverse N-point DFT, Sec. II step 3 with the sign and 1/N of eq. (4):
 *   z(i) = (1/n) sum_k Y(k) conj(w[(i k) mod n]). */
static void idft_direct(int n, const double *wr, const double *wi,
                        const double *Y, double *z)
{
    for (int i = 0; i < n; ++i) {
        double accr = 0.0, acci = 0.0;
        for (int k = 0; k < n; ++k) {
            int64_t r = ((int64_t)i * (int64_t)k) % n;
            double yr = Y[2 * k], yi = Y[2 * k + 1];
            /* multiply by conj(w) = wr - j wi */
            accr += yr * wr[r] + yi * wi[r];
            acci += yi * wr[r] - yr * wi[r];
        }
        z[2 * i] = accr / (double)n;
        z[2 * i + 1] = acci / (double)n;
    }
}

int oracle_dft(int n, const double *s, double *X)
{
    double *wr, *wi;
    if (n < 1 || !s || !X || make_twiddles(n, &wr, &wi))
        return ORACLE_EINVAL;
    dft_direct(n, wr, wi, s, X);
    free(wr);
    free(wi);
    return 0;
}

int oracle_idft(int n, const double *Y, double *z)
{
    double *wr, *wi;
    if (n < 1 || !Y || !z || make_twiddles(n, &wr, &wi))
        return ORACLE_EINVAL;
    idft_direct(n, wr, wi, Y, z);
    free(wr);
    free(wi);
    return 0;
}

/* H_R(k) of eq. (6), bin by bin over the three region sets. */
static double hfso_magnitude_bin(int n, int k1, int lv, const double *v, int k)
{
    int k2 = k1 + lv - 1;
    if ((k >= 0 && k <= k1 - 1) || (k >= n - k1 + 1 && k <= n - 1))
        return 1.0;                         /* passband k_p */
    if (k >= k1 && k <= k2)
        return v[k - k1];                   /* transition k_t, upper edge */
    if (k >= n - k2 && k <= n - k1)
        return v[n - k - k1];               /* transition k_t, mirrored edge */
    return 0.0;                             /* stopband k_s */
}

/* The region sets of eq. (6) are disjoint and cover [0,n) only when the
 * mirrored transition band does not run into the upper one: k2 < n - k2,
 * or the degenerate all-pass case (no transition, k1 = n/2 + 1). */
static int hfso_bins_ok(int n, int k1, int lv, const double *v)
{
    if (n < 2 || lv < 0 || (lv > 0 && !v) || k1 < 1)
        return 0;
    if (lv == 0 && 2 * k1 == n + 2)
        return 1;
    int k2 = k1 + lv - 1;
    return 2 * k2 < n;
}

static int hfso_args_ok(int n, int hop, int k1, int lv, const double *v)
{
    if (hop < 1 || hop > n - 1 || ((n - hop) & 1))
        return 0;
    return hfso_bins_ok(n, k1, lv, v);
}

int oracle_hfso_magnitude(int n, int k1, int lv, const double *v, double *hr)
{
    if (!hr || !hfso_bins_ok(n, k1, lv, v))
        return ORACLE_EINVAL;
    for (int k = 0; k < n; ++k)
        hr[k] = hfso_magnitude_bin(n, k1, lv, v, k);
    return 0;
}

/* Eq. (5): H(k) = H_R(k) exp(-j 2 pi k D / n), D = (L-1)/2 = (n-hop)/2. */
static void hfso_coeffs(int n, int hop, int k1, int lv, const double *v,
                        const double *wr, const double *wi, double *H)
{
    int64_t d = (n - hop) / 2;
    for (int k = 0; k < n; ++k) {
        double hr = hfso_magnitude_bin(n, k1, lv, v, k);
        int64_t r = ((int64_t)k * d) % n;
        H[2 * k] = hr * wr[r];
        H[2 * k + 1] = hr * wi[r];
    }
}

int oracle_hfso_coeffs(int n, int hop, int k1, int lv, const double *v, double *H)
{
    double *wr, *wi;
    if (!H || !hfso_args_ok(n, hop, k1, lv, v) || make_twiddles(n, &wr, &wi))
        return ORACLE_EINVAL;
    hfso_coeffs(n, hop, k1, lv, v, wr, wi, H);
    free(wr);
    free(wi);
    return 0;
}

/* One OLS block (Sec. II, steps 1-4) for an arbitrary coefficient vector H:
 * segment -> DFT -> multiply -> IDFT -> keep z(n-hop .. n-1).  `out` receives
 * hop interleaved samples; samples at or beyond len are computed like any other
 * and left for the caller to drop.  work must hold 6n doubles. */
static void ols_block(const double *x, int64_t len, int n, int hop, int64_t m,
                      const double *H, const double *wr, const double *wi,
                      double *work, double *out)
{
    double *s = work, *X = work + 2 * n, *z = work + 4 * n;
    int64_t start = m * (int64_t)hop - (int64_t)(n - hop);
    for (int i = 0; i < n; ++i) {
        int64_t t = start + i;
        if (t >= 0 && t < len) {
            s[2 * i] = x[2 * t];
            s[2 * i + 1] = x[2 * t + 1];
        } else {
            s[2 * i] = 0.0;
            s[2 * i + 1] = 0.0;
        }
    }
    dft_direct(n, wr, wi, s, X);
    for (int k = 0; k < n; ++k) {           /* step 2: Y(k) = H(k) X(k) */
        double xr = X[2 * k], xi = X[2 * k + 1];
        double hr = H[2 * k], hi = H[2 * k + 1];
        X[2 * k] = hr * xr - hi * xi;
        X[2 * k + 1] = hr * xi + hi * xr;
    }
    idft_direct(n, wr, wi, X, z);
    for (int j = 0; j < hop; ++j) {         /* step 4: drop the first n-hop */
        out[2 * j] = z[2 * (n - hop + j)];
        out[2 * j + 1] = z[2 * (n - hop + j) + 1];
    }
}

static int64_t n_blocks_of(int64_t len, int hop)
{
    return len <= 0 ? 0 : (len + hop - 1) / hop;
}

/* Block-index list: NULL means every block 0 .. nb-1. */
static int64_t block_at(const int64_t *blocks, int64_t b)
{
    return blocks ? blocks[b] : b;
}

/* OLS with one fixed, arbitrary coefficient vector H (time-invariant use of
 * Sec. II).  Writes hop samples per listed block, compactly: out[b*hop + j]. */
int oracle_blocks_generic(const double *x, int64_t len, int n, int hop,
                          const double *H, const int64_t *blocks,
                          int64_t n_sel, double *out)
{
    if ((!x && len > 0) || !H || (!out && n_sel > 0) || n < 2 || hop < 1 || hop > n - 1 ||
        len < 0 || n_sel < 0)
        return ORACLE_EINVAL;
    int64_t nb = n_blocks_of(len, hop);
    for (int64_t b = 0; b < n_sel; ++b)
        if (block_at(blocks, b) < 0 || block_at(blocks, b) >= nb)
            return ORACLE_EINVAL;
    double *wr, *wi;
    if (make_twiddles(n, &wr, &wi))
        return ORACLE_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 6 * (size_t)n);
        if (!work) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < n_sel; ++b)
                ols_block(x, len, n, hop, block_at(blocks, b), H, wr, wi, work,
                          out + 2 * b * (int64_t)hop);
            free(work);
        }
    }
    free(wr);
    free(wi);
    return err ? ORACLE_EINVAL : 0;
}

/* The k1 in force for block m: the schedule pair with the largest
 * from_block <= m.  Pairs may come in any order; a later duplicate
 * from_block wins. */
static int k1_for_block(int n_sched, const int64_t *from, const int32_t *k1s,
                        int64_t m)
{
    int best = -1;
    for (int i = 0; i < n_sched; ++i)
        if (from[i] <= m && (best < 0 || from[i] >= from[best]))
            best = i;
    return best < 0 ? -1 : k1s[best];
}

/* HFSO variable-bandwidth OLS (Sec. II with eqs. (5)-(7)) over the listed
 * blocks.  V holds lv transition values shared by every bandwidth; the
 * schedule gives k1 per block.  Output is compact: out[b*hop + j]. */
int oracle_blocks_hfso(const double *x, int64_t len, int n, int hop, int lv,
                       const double *v, int n_sched, const int64_t *sched_from,
                       const int32_t *sched_k1, const int64_t *blocks,
                       int64_t n_sel, double *out)
{
    if ((!x && len > 0) || (!out && n_sel > 0) || len < 0 || n_sel < 0 || n_sched < 1 ||
        !sched_from || !sched_k1)
        return ORACLE_EINVAL;
    int64_t nb = n_blocks_of(len, hop);
    for (int i = 0; i < n_sched; ++i)
        if (sched_from[i] < 0 || !hfso_args_ok(n, hop, sched_k1[i], lv, v))
            return ORACLE_EINVAL;
    for (int64_t b = 0; b < n_sel; ++b) {
        int64_t m = block_at(blocks, b);
        if (m < 0 || m >= nb || k1_for_block(n_sched, sched_from, sched_k1, m) < 0)
            return ORACLE_EINVAL;
    }
    double *wr, *wi;
    if (make_twiddles(n, &wr, &wi))
        return ORACLE_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 8 * (size_t)n);
        if (!work) {
#pragma omp atomic write
            err = 1;
        } else {
            double *H = work + 6 * n;
            int h_k1 = -1;
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < n_sel; ++b) {
                int64_t m = block_at(blocks, b);
                int k1 = k1_for_block(n_sched, sched_from, sched_k1, m);
                if (k1 != h_k1) {
                    hfso_coeffs(n, hop, k1, lv, v, wr, wi, H);
                    h_k1 = k1;
                }
                ols_block(x, len, n, hop, m, H, wr, wi, work,
                          out + 2 * b * (int64_t)hop);
            }
            free(work);
        }
    }
    free(wr);
    free(wi);
    return err ? ORACLE_EINVAL : 0;
}

/* Whole channel, Sec. II step 5: y(m*hop + j) for every block, truncated to
 * len samples. */
int oracle_channel_hfso(const double *x, int64_t len, int n, int hop, int lv,
                        const double *v, int n_sched, const int64_t *sched_from,
                        const int32_t *sched_k1, double *y)
{
    if ((!y && len > 0) || len < 0 || hop < 1 || n_sched < 1 || !sched_from || !sched_k1)
        return ORACLE_EINVAL;
    for (int i = 0; i < n_sched; ++i)
        if (!hfso_args_ok(n, hop, sched_k1[i], lv, v))
            return ORACLE_EINVAL;
    int64_t nb = n_blocks_of(len, hop);
    if (nb == 0)
        return 0;
    double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)(nb * hop));
    if (!tmp)
        return ORACLE_EINVAL;
    int rc = oracle_blocks_hfso(x, len, n, hop, lv, v, n_sched, sched_from,
                                sched_k1, NULL, nb, tmp);
    if (rc == 0)
        memcpy(y, tmp, sizeof(double) * 2 * (size_t)len);
    free(tmp);
    return rc;
}

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
