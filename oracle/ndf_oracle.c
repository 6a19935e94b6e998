/*
 * Plain FP64 CPU oracle for the direct dependence estimators.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU path is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * table with the GPU library.
 *
 * Arrays are float32 as stored in the ensemble and are promoted to double.
 * A "column" is the local sample e(p) of one grid vertex (Sec. 3): N member
 * values, read with a stride.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Pearson correlation, Sec. 3.1 Eq. (1): r = cov(a,b) / sqrt(var(a) var(b)). */
/* Two passes: means first, then centred sums.  The 1/N (or 1/(N-1)) factors  */
/* of the sample moments cancel.  A vertex with zero variance gives r = 0.    */
/* ------------------------------------------------------------------------ */
double ndf_oracle_pearson(const float *a, int64_t sa, const float *b, int64_t sb, int64_t n)
{
    double ma = 0.0, mb = 0.0;
    for (int64_t m = 0; m < n; ++m) {
        ma += (double)a[m * sa];
        mb += (double)b[m * sb];
    }
    ma /= (double)n;
    mb /= (double)n;
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    for (int64_t m = 0; m < n; ++m) {
        double da = (double)a[m * sa] - ma;
        double db = (double)b[m * sb] - mb;
        sab += da * db;
        saa += da * da;
        sbb += db * db;
    }
    if (saa == 0.0 || sbb == 0.0)
        return 0.0;
    return sab / sqrt(saa * sbb);
}

/* r(ref, q) for every query column of a member-major block q[N][nq]. */
void ndf_oracle_pearson_field(const float *ref, int64_t sref, const float *q, int64_t nq,
                              int64_t n, double *out)
{
    int64_t v;
#pragma omp parallel for schedule(dynamic, 64)
    for (v = 0; v < nq; ++v)
        out[v] = ndf_oracle_pearson(ref, sref, q + v, nq, n);
}

/* Population mean and standard deviation of one column (used by tests of the */
/* standardisation step).                                                     */
void ndf_oracle_moments(const float *a, int64_t sa, int64_t n, double *mean, double *std)
{
    double m0 = 0.0;
    for (int64_t m = 0; m < n; ++m)
        m0 += (double)a[m * sa];
    m0 /= (double)n;
    double s = 0.0;
    for (int64_t m = 0; m < n; ++m) {
        double d = (double)a[m * sa] - m0;
        s += d * d;
    }
    *mean = m0;
    *std = sqrt(s / (double)n);
}

/* ------------------------------------------------------------------------ */
/* Kraskov-Stoegbauer-Grassberger mutual information (Sec. 3.2, Eq. (2); the   */
/* estimator of [KSG04], their first algorithm, max-norm in the joint space).  */
/* ------------------------------------------------------------------------ */

/* Integer codes of one column: min-max normalisation onto [0, 2^23].
 * s = 2^23 / (hi - lo) and code = round-half-even((x - lo) * s), all in IEEE
 * double with single roundings, so any correctly rounded implementation gets
 * the same integers.  Returns 1 if the range is zero (all codes 0), else 0. */
int ndf_oracle_ksg_codes(const float *col, int64_t stride, int64_t n, int32_t *code)
{
    double lo = (double)col[0], hi = (double)col[0];
    for (int64_t m = 1; m < n; ++m) {
        double x = (double)col[m * stride];
        if (x < lo) lo = x;
        if (x > hi) hi = x;
    }
    if (!(hi > lo)) {
        for (int64_t m = 0; m < n; ++m)
            code[m] = 0;
        return 1;
    }
    double s = 8388608.0 / (hi - lo);
    for (int64_t m = 0; m < n; ++m) {
        double t = ((double)col[m * stride] - lo) * s;
        code[m] = (int32_t)nearbyint(t); /* default rounding mode: to nearest even */
    }
    return 0;
}

/* Harmonic numbers H_0 = 0, H_i = H_{i-1} + 1/i.  psi(i) = H_{i-1} - gamma, so
 * the KSG estimate psi(k) + psi(N) - <psi(nx+1) + psi(ny+1)> equals
 * H_{k-1} + H_{N-1} - <H_nx + H_ny> (the Euler constant cancels). */
static double *harmonic_table(int64_t n)
{
    double *h = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    h[0] = 0.0;
    for (int64_t i = 1; i <= n; ++i)
        h[i] = h[i - 1] + 1.0 / (double)i;
    return h;
}

static int64_t iabs64(int64_t a) { return a < 0 ? -a : a; }

/* Brute-force KSG on integer codes x, y (length n), k-th neighbour.
 * eps_i  = k-th smallest of { max(|x_i-x_j|, |y_i-y_j|) : j != i } (ties count)
 * nx_i   = #{ j != i : |x_i - x_j| < eps_i },  ny_i likewise (strict)
 * I      = psi(k) + psi(n) - (1/n) sum_i [psi(nx_i + 1) + psi(ny_i + 1)]
 * Counts are written to nx/ny when those are non-NULL. */
static double ksg_core(const int32_t *x, const int32_t *y, int64_t n, int k, const double *h,
                       int32_t *nx, int32_t *ny, int64_t *best)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int t = 0; t < k; ++t)
            best[t] = INT64_MAX;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            int64_t dx = iabs64((int64_t)x[i] - x[j]);
            int64_t dy = iabs64((int64_t)y[i] - y[j]);
            int64_t d = dx > dy ? dx : dy;
            if (d < best[k - 1]) {
                int t = k - 1;
                while (t > 0 && best[t - 1] > d) {
                    best[t] = best[t - 1];
                    --t;
                }
                best[t] = d;
            }
        }
        int64_t eps = best[k - 1];
        int64_t cx = 0, cy = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            if (iabs64((int64_t)x[i] - x[j]) < eps) ++cx;
            if (iabs64((int64_t)y[i] - y[j]) < eps) ++cy;
        }
        if (nx) nx[i] = (int32_t)cx;
        if (ny) ny[i] = (int32_t)cy;
        acc += h[cx] + h[cy];
    }
    return h[k - 1] + h[n - 1] - acc / (double)n;
}

double ndf_oracle_ksg(const int32_t *x, const int32_t *y, int64_t n, int k, int32_t *nx,
                      int32_t *ny)
{
    if (k < 1 || k >= n)
        return NAN;
    double *h = harmonic_table(n);
    int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    double r = ksg_core(x, y, n, k, h, nx, ny, best);
    free(best);
    free(h);
    return r;
}

/* MI(ref, q) for every query column of a member-major block q[N][nq] (raw
 * float32 values; codes are taken per column as above).  A zero-range column
 * on either side gives MI = 0 and zero counts.  nx/ny, when non-NULL, are
 * [nq][n]. */
void ndf_oracle_ksg_field(const float *ref, int64_t sref, const float *q, int64_t nq, int64_t n,
                          int k, double *out, int32_t *nx, int32_t *ny)
{
    int32_t *cref = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int ref_flat = ndf_oracle_ksg_codes(ref, sref, n, cref);
    double *h = harmonic_table(n);
    int64_t v;
#pragma omp parallel
    {
        int32_t *cq = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
#pragma omp for schedule(dynamic, 4)
        for (v = 0; v < nq; ++v) {
            int flat = ndf_oracle_ksg_codes(q + v, nq, n, cq);
            int32_t *px = nx ? nx + v * n : NULL;
            int32_t *py = ny ? ny + v * n : NULL;
            if (flat || ref_flat) {
                out[v] = 0.0;
                if (px) memset(px, 0, sizeof(int32_t) * (size_t)n);
                if (py) memset(py, 0, sizeof(int32_t) * (size_t)n);
                continue;
            }
            out[v] = ksg_core(cref, cq, n, k, h, px, py, best);
        }
        free(best);
        free(cq);
    }
    free(h);
    free(cref);
}

/* ------------------------------------------------------------------------ */
/* Pairs of columns (training targets, Sec. 4.3, and held-out evaluation):     */
/* column p of the member-major blocks a[N][np] and b[N][np] forms pair p.     */
/* ------------------------------------------------------------------------ */
void ndf_oracle_pearson_pairs(const float *a, const float *b, int64_t np, int64_t n,
                              double *out)
{
    int64_t p;
#pragma omp parallel for schedule(dynamic, 256)
    for (p = 0; p < np; ++p)
        out[p] = ndf_oracle_pearson(a + p, np, b + p, np, n);
}

void ndf_oracle_ksg_pairs(const float *a, const float *b, int64_t np, int64_t n, int k,
                          double *out)
{
    double *h = harmonic_table(n);
    int64_t p;
#pragma omp parallel
    {
        int32_t *ca = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *cb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
#pragma omp for schedule(dynamic, 4)
        for (p = 0; p < np; ++p) {
            int fa = ndf_oracle_ksg_codes(a + p, np, n, ca);
            int fb = ndf_oracle_ksg_codes(b + p, np, n, cb);
            out[p] = (fa || fb) ? 0.0 : ksg_core(ca, cb, n, k, h, NULL, NULL, best);
        }
        free(best);
        free(cb);
        free(ca);
    }
    free(h);
}

/* Threads of the parallel loops above (the CPU baseline times one and all). */
extern void omp_set_num_threads(int);
extern int omp_get_max_threads(void);
void ndf_oracle_set_threads(int n) { omp_set_num_threads(n); }
int ndf_oracle_max_threads(void) { return omp_get_max_threads(); }
