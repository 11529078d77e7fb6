/* Runs the FP64 oracle's entry points under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitize.py with gcc):
 * ordinary and edge-case inputs, including the error paths.  Exit status 0
 * when every call returned what it should; a sanitizer report aborts the
 * process (-fno-sanitize-recover). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double mean, sigma, psi8, g1, psi6, g2, psi4, h;
} result_t;

double oracle_K6(double);
double oracle_K4(double);
double oracle_phi_deriv(int, double);
int oracle_moments(const double*, int64_t, double*, double*);
int oracle_block_sum(const double*, int64_t, int, double, int64_t, int64_t, int64_t, int64_t, double*);
int oracle_pair_sum(const double*, int64_t, int, double, double*);
int oracle_psi(const double*, int64_t, int, double, double*);
int oracle_plugin(const double*, int64_t, result_t*);
int oracle_plugin_zscore(const double*, int64_t, result_t*);
int oracle_kde_eval(const double*, int64_t, double, const double*, int64_t, double*);

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                \
        }                                                           \
    } while (0)

/* a small deterministic sample generator (xorshift), not the method's arithmetic */
static void fill(double* x, int64_t n, uint64_t seed) {
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
    for (int64_t i = 0; i < n; ++i) {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        x[i] = (double)(s >> 11) * 0x1.0p-53 * 4.0 - 2.0;
    }
}

int main(void) {
    const int64_t sizes[] = {1, 2, 3, 8, 63, 64, 65, 257, 1000};
    for (size_t k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
        const int64_t n = sizes[k];
        double* x = (double*)malloc(sizeof(double) * (size_t)n);
        fill(x, n, (uint64_t)n);
        double p4, p6;
        CHECK(oracle_psi(x, n, 4, 0.3, &p4) == 0 && p4 > 0);
        CHECK(oracle_psi(x, n, 6, 0.3, &p6) == 0 && p6 < 0);
        result_t r, z;
        if (n >= 2) {
            CHECK(oracle_plugin(x, n, &r) == 0 && isfinite(r.h) && r.h > 0);
            CHECK(oracle_plugin_zscore(x, n, &z) == 0 && fabs(z.h - r.h) <= 1e-10 * r.h);
            double m, s;
            CHECK(oracle_moments(x, n, &m, &s) == 0 && s > 0);
        }
        double b;
        CHECK(oracle_block_sum(x, n, 4, 0.5, 0, n, 0, n, &b) == 0);
        CHECK(oracle_block_sum(x, n, 6, 0.5, n / 2, n, 0, n / 3, &b) == 0);
        double y[5] = {-3, -1, 0, 1, 3}, f[5];
        CHECK(oracle_kde_eval(x, n, 0.4, y, 5, f) == 0 && f[2] > 0);
        CHECK(oracle_kde_eval(x, n, 0.4, y, 0, f) == 0);
        free(x);
    }
    /* error paths: null pointers, n too small, bad r and g, non-finite data,
       constant data, ranges outside the sample */
    double x[4] = {1.0, 2.0, NAN, 4.0}, c[3] = {2.0, 2.0, 2.0}, v;
    result_t r;
    CHECK(oracle_plugin(NULL, 4, &r) < 0);
    CHECK(oracle_plugin(x, 1, &r) < 0);
    CHECK(oracle_plugin(x, 4, &r) < 0);
    CHECK(oracle_plugin(c, 3, &r) < 0);
    CHECK(oracle_psi(c, 3, 4, 0.5, &v) == 0 && v > 0);
    CHECK(oracle_psi(x, 4, 5, 0.5, &v) < 0);
    CHECK(oracle_psi(c, 3, 4, 0.0, &v) < 0);
    CHECK(oracle_psi(c, 3, 4, INFINITY, &v) < 0);
    CHECK(oracle_block_sum(c, 3, 4, 0.5, 0, 4, 0, 3, &v) < 0);
    CHECK(oracle_block_sum(c, 3, 4, 0.5, 2, 1, 0, 3, &v) < 0);
    CHECK(oracle_moments(x, 4, &v, &v) < 0);
    CHECK(oracle_kde_eval(c, 3, -1.0, c, 3, &v) < 0);
    CHECK(isfinite(oracle_K6(40.0)) && isfinite(oracle_K4(-40.0)) && isfinite(oracle_phi_deriv(8, 3.0)));
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle under sanitizers: ok\n");
    return 0;
}
