/* Host sanitizer run of the C oracle (test infrastructure): small cases of
   every exported function, built with AddressSanitizer and
   UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exits 0 when
   every call returns what its contract says; the sanitizers abort on any
   out-of-bounds access, use after free or undefined operation. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny;
    double phiy_min, phiy_max;
    double E_dc, E_w, omega, B, mu, alpha, dt;
    int32_t n_threads;
} oracle_params;

int oracle_bessel_ratios(double mu, int32_t nmax, double* out);
int oracle_run(const oracle_params* p, int64_t k0, int64_t n_steps, int32_t init_f0,
               int32_t do_startup, double* a_h, double* b_h, double* a_f, double* b_f,
               int64_t win_lo, int64_t win_hi, double* v_trace, double* norm_trace,
               double* obs);
int oracle_equilibrium(const oracle_params* p, double* a0);
int oracle_max_threads(void);
int oracle_characteristic_v(double E_dc, double E_w, double omega, double B, int32_t n_nodes,
                            const double* x0, const double* y0, const double* w,
                            int32_t n_launch, double h, double tau_max, int32_t n_threads,
                            double* v);

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    double r[65];
    CHECK(oracle_bessel_ratios(2.0, 64, r) == 0 && r[0] == 1.0 && r[1] > 0 && r[64] >= 0);
    CHECK(oracle_bessel_ratios(-1.0, 8, r) != 0);

    /* grids with edge sizes: the smallest legal one, odd and ragged ones */
    const int32_t shapes[][2] = {{2, 3}, {3, 5}, {7, 33}, {16, 101}};
    for (int s = 0; s < 4; ++s) {
        oracle_params p = {shapes[s][0], shapes[s][1], -4.0, 4.0, 1.5, 0.3, 2.0, 1.0, 1.0, 0.9,
                           1e-3, 2};
        const size_t n = (size_t)p.nx * p.ny;
        double *ah = calloc(n, sizeof(double)), *bh = calloc(n, sizeof(double));
        double *af = calloc(n, sizeof(double)), *bf = calloc(n, sizeof(double));
        double *a0 = calloc(n, sizeof(double)), *vt = calloc(40, sizeof(double));
        double *nt = calloc(40, sizeof(double)), obs[7];
        CHECK(ah && bh && af && bf && a0 && vt && nt);
        CHECK(oracle_equilibrium(&p, a0) == 0);
        CHECK(oracle_run(&p, 0, 40, 1, 1, ah, bh, af, bf, 10, 40, vt, nt, obs) == 0);
        CHECK(isfinite(obs[0]) && isfinite(obs[1]) && obs[4] == 30.0);
        /* resume from the returned state, without traces */
        CHECK(oracle_run(&p, 40, 7, 0, 0, ah, bh, af, bf, 0, 0, NULL, NULL, obs) == 0);
        p.nx = 1;
        CHECK(oracle_run(&p, 0, 1, 1, 1, ah, bh, af, bf, 0, 0, NULL, NULL, obs) != 0);
        free(ah); free(bh); free(af); free(bf); free(a0); free(vt); free(nt);
    }
    CHECK(oracle_max_threads() >= 1);

    /* characteristic curves: a few quadrature nodes, one period of launches */
    const double x0[3] = {-0.3, 0.0, 0.4}, y0[3] = {0.1, 0.0, -0.2}, w[3] = {0.25, 0.5, 0.25};
    const int32_t n_launch = 16;
    const double omega = 2.0, h = 2.0 * 3.14159265358979323846 / omega / n_launch;
    double v[16];
    CHECK(oracle_characteristic_v(1.0, 0.5, omega, 2.0, 3, x0, y0, w, n_launch, h, 4.0, 2, v) == 0);
    for (int i = 0; i < n_launch; ++i) CHECK(isfinite(v[i]));
    CHECK(oracle_characteristic_v(1.0, 0.5, omega, 2.0, 0, x0, y0, w, n_launch, h, 4.0, 2, v) != 0);
    printf("oracle sanitizer run ok\n");
    return 0;
}
