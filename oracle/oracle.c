/*
 * FP64 CPU oracle for the two-stage PLUGIN bandwidth selector for univariate
 * Gaussian kernel density estimation (Gramacki, Sawerwain, Gramacki,
 * "FPGA-Based Bandwidth Selection for Kernel Density Estimation Using High
 * Level Synthesis Approach", arXiv:1505.02100).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, constant table or helper with the HIP library.
 *
 * What it computes (Section 3, Algorithm 1):
 *   Step I    variance and standard deviation of the sample (divisor n-1);
 *   Step II   normal-scale estimate Psi8 = 105 / (32 sqrt(pi) sigma^9);
 *   Step III  g1 = (-2 K6(0) / (mu2 Psi8 n))^(1/9), K6(0) = -15/sqrt(2 pi);
 *   Step IV   Psi6(g1) = (n^2 g1^7)^-1 sum_i sum_j K6((Xi - Xj)/g1);
 *   Step V    g2 = (-2 K4(0) / (mu2 Psi6 n))^(1/7), K4(0) = 3/sqrt(2 pi);
 *   Step VI   Psi4(g2) = (n^2 g2^5)^-1 sum_i sum_j K4((Xi - Xj)/g2);
 *   Step VII  h = (R(K) / (mu2^2 Psi4 n))^(1/5), R(K) = 1/(2 sqrt(pi)), mu2 = 1.
 * The double sums use the symmetric form of equations (6) and (7): twice the
 * strict upper triangle plus n K(0) for the diagonal.
 *
 * Readings where the paper is silent (all recorded with the design notes):
 *  - Step I is evaluated in the two-pass form sum (x - mean)^2 / (n - 1),
 *    which is algebraically the printed one-pass formula without its
 *    cancellation on shifted data.
 *  - The diagonal i = j is part of the estimator (the printed double sums run
 *    over all i and j); it enters as n K(0) exactly as in equations (6)-(7).
 *  - Division by g is a true division (the FPGA design's reciprocal trick is
 *    an implementation choice, not part of the definition).
 *  - Summation order: each row partial sum_{j>i} is accumulated left to right
 *    in plain FP64, and the row partials are added in row order with a
 *    Neumaier compensated sum.  The result therefore does not depend on the
 *    number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENONFINITE (-2)
#define OR_EDEGENERATE (-3)
#define OR_ENOMEM (-4)

static const double OR_PI = 3.14159265358979323846264338327950288;

typedef struct {
    double mean, sigma, psi8, g1, psi6, g2, psi4, h;
} oracle_plugin_result;

/* Kernel derivatives exactly as printed in Algorithm 1, Steps IV and VI:
 *   K6(x) = (x^6 - 15 x^4 + 45 x^2 - 15) exp(-x^2/2) / sqrt(2 pi)
 *   K4(x) = (x^4 - 6 x^2 + 3) exp(-x^2/2) / sqrt(2 pi)                       */
double oracle_K6(double x) {
    double t = x * x;
    double p = ((t - 15.0) * t + 45.0) * t - 15.0;
    return p * exp(-0.5 * t) / sqrt(2.0 * OR_PI);
}

double oracle_K4(double x) {
    double t = x * x;
    double p = (t - 6.0) * t + 3.0;
    return p * exp(-0.5 * t) / sqrt(2.0 * OR_PI);
}

/* r-th derivative of the standard normal density for any even r >= 0, built
 * from the probabilists' Hermite recurrence He_{k+1} = u He_k - k He_{k-1};
 * for even r, phi^(r)(u) = He_r(u) phi(u).  Used by tests only, as a second
 * route to the printed K4/K6 polynomials.                                   */
double oracle_phi_deriv(int r, double u) {
    double hm1 = 1.0, h = u; /* He_0, He_1 */
    if (r == 0) h = 1.0;
    for (int k = 1; k < r; ++k) {
        double hn = u * h - k * hm1;
        hm1 = h;
        h = hn;
    }
    double sgn = (r % 2) ? -1.0 : 1.0;
    return sgn * h * exp(-0.5 * u * u) / sqrt(2.0 * OR_PI);
}

static double kernel_r(int r, double x) {
    return r == 6 ? oracle_K6(x) : oracle_K4(x);
}

static int check_input(const double* x, int64_t n, int64_t nmin) {
    if (!x || n < nmin) return OR_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return OR_ENONFINITE;
    return OR_OK;
}

/* Neumaier's compensated summation of a[0..m) in index order. */
static double neumaier(const double* a, int64_t m) {
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        double v = a[k];
        double t = s + v;
        if (fabs(s) >= fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    return s + c;
}

/* Step I: mean and sigma-hat with divisor n - 1 (two-pass form). */
int oracle_moments(const double* x, int64_t n, double* mean, double* sigma) {
    int st = check_input(x, n, 2);
    if (st) return st;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
    if (!tmp) return OR_ENOMEM;
    double m = neumaier(x, n) / (double)n;
    for (int64_t i = 0; i < n; ++i) {
        double d = x[i] - m;
        tmp[i] = d * d;
    }
    double v = neumaier(tmp, n) / (double)(n - 1);
    free(tmp);
    if (mean) *mean = m;
    if (sigma) *sigma = sqrt(v);
    return OR_OK;
}

/* Strict-upper-triangle sum over a rectangle of the pair matrix:
 *   S = sum_{i in [r0,r1)} sum_{j in [c0,c1), j > i} K^(r)((x_i - x_j)/g).
 * Rows run in parallel; each row partial is a left-to-right FP64 sum and the
 * partials are combined in row order with a Neumaier sum.                  */
int oracle_block_sum(const double* x, int64_t n, int r, double g, int64_t r0,
                     int64_t r1, int64_t c0, int64_t c1, double* out) {
    if (!x || !out || n < 1 || (r != 4 && r != 6)) return OR_EINVAL;
    if (!(g > 0.0) || !isfinite(g)) return OR_EINVAL;
    if (r0 < 0 || c0 < 0 || r1 > n || c1 > n || r0 > r1 || c0 > c1) return OR_EINVAL;
    int64_t m = r1 - r0;
    if (m == 0) { *out = 0.0; return OR_OK; }
    double* rows = (double*)malloc(sizeof(double) * (size_t)m);
    if (!rows) return OR_ENOMEM;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = r0; i < r1; ++i) {
        double acc = 0.0;
        int64_t jb = c0 > i + 1 ? c0 : i + 1;
        for (int64_t j = jb; j < c1; ++j) acc += kernel_r(r, (x[i] - x[j]) / g);
        rows[i - r0] = acc;
    }
    *out = neumaier(rows, m);
    free(rows);
    return OR_OK;
}

int oracle_pair_sum(const double* x, int64_t n, int r, double g, double* out) {
    return oracle_block_sum(x, n, r, g, 0, n, 0, n, out);
}

/* Equations (6)-(7): Psi_r(g) = [2 sum_{i<j} K^(r)((Xi-Xj)/g) + n K^(r)(0)] / (n^2 g^(r+1)). */
int oracle_psi(const double* x, int64_t n, int r, double g, double* psi) {
    if (!psi) return OR_EINVAL;
    int st = check_input(x, n, 1);
    if (st) return st;
    double s;
    st = oracle_pair_sum(x, n, r, g, &s);
    if (st) return st;
    double nd = (double)n;
    *psi = (2.0 * s + nd * kernel_r(r, 0.0)) / (nd * nd * pow(g, (double)(r + 1)));
    return OR_OK;
}

/* Algorithm 1, Steps I-VII on the raw sample. */
int oracle_plugin(const double* x, int64_t n, oracle_plugin_result* out) {
    if (!out) return OR_EINVAL;
    memset(out, 0, sizeof(*out));
    double mean, sigma;
    int st = oracle_moments(x, n, &mean, &sigma);
    if (st) return st;
    out->mean = mean;
    out->sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) return OR_EDEGENERATE;
    double nd = (double)n;
    const double mu2 = 1.0;
    const double K6_0 = -15.0 / sqrt(2.0 * OR_PI);
    const double K4_0 = 3.0 / sqrt(2.0 * OR_PI);
    const double RK = 1.0 / (2.0 * sqrt(OR_PI));
    /* Step II */
    double psi8 = 105.0 / (32.0 * sqrt(OR_PI) * pow(sigma, 9.0));
    out->psi8 = psi8;
    if (!(psi8 > 0.0) || !isfinite(psi8)) return OR_EDEGENERATE;
    /* Step III */
    double g1 = pow(-2.0 * K6_0 / (mu2 * psi8 * nd), 1.0 / 9.0);
    out->g1 = g1;
    if (!(g1 > 0.0) || !isfinite(g1)) return OR_EDEGENERATE;
    /* Step IV */
    double psi6;
    st = oracle_psi(x, n, 6, g1, &psi6);
    if (st) return st;
    out->psi6 = psi6;
    if (!(psi6 < 0.0)) return OR_EDEGENERATE;
    /* Step V */
    double g2 = pow(-2.0 * K4_0 / (mu2 * psi6 * nd), 1.0 / 7.0);
    out->g2 = g2;
    if (!(g2 > 0.0) || !isfinite(g2)) return OR_EDEGENERATE;
    /* Step VI */
    double psi4;
    st = oracle_psi(x, n, 4, g2, &psi4);
    if (st) return st;
    out->psi4 = psi4;
    if (!(psi4 > 0.0)) return OR_EDEGENERATE;
    /* Step VII */
    out->h = pow(RK / (mu2 * mu2 * psi4 * nd), 1.0 / 5.0);
    return OR_OK;
}

/* The z-score route of equations (3)-(4): standardise with the Step I mean
 * and sigma-hat, run Algorithm 1 on Z, and return h_Z * sigma-hat.          */
int oracle_plugin_zscore(const double* x, int64_t n, oracle_plugin_result* out) {
    if (!out) return OR_EINVAL;
    double mean, sigma;
    int st = oracle_moments(x, n, &mean, &sigma);
    if (st) return st;
    if (!(sigma > 0.0) || !isfinite(sigma)) return OR_EDEGENERATE;
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    if (!z) return OR_ENOMEM;
    for (int64_t i = 0; i < n; ++i) z[i] = (x[i] - mean) / sigma;
    st = oracle_plugin(z, n, out);
    free(z);
    if (st) return st;
    out->h *= sigma;
    out->g1 *= sigma;
    out->g2 *= sigma;
    out->mean = mean;
    out->sigma = sigma;
    return OR_OK;
}

/* Equation (1) with the Gaussian kernel of equation (2):
 *   f(x; h) = (n h)^-1 sum_i K((x - X_i)/h),  evaluated at m points.         */
int oracle_kde_eval(const double* x, int64_t n, double h, const double* pts,
                    int64_t m, double* out) {
    if (!x || !pts || !out || n < 1 || m < 0) return OR_EINVAL;
    if (!(h > 0.0) || !isfinite(h)) return OR_EINVAL;
    const double c = 1.0 / sqrt(2.0 * OR_PI);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double u = (pts[k] - x[i]) / h;
            acc += c * exp(-0.5 * u * u);
        }
        out[k] = acc / ((double)n * h);
    }
    return OR_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
