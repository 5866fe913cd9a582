/*
 * FP64 CPU oracle for the superlattice Boltzmann transport equation solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (D. Priimak, "Finite difference numerical method for the
 * superlattice Boltzmann transport equation ...", arXiv:1401.6047):
 *
 *   - Sec. 2: the Fourier-in-phi_x form of the dimensionless BTE, the
 *     equilibrium coefficients a^(0)_n(phi_y), the initial state
 *     a_n = a^(0)_n, b_n = 0, the field E(t) = E_dc + E_w cos(w t), the
 *     drift velocity v_dr = pi sqrt(alpha) \int b_1 dphi_y and the
 *     normalisation 2 pi sqrt(alpha) \int a_0 dphi_y.
 *   - Sec. 3: the grid n in [0, N_x), m in [0, N_y) with zero boundary cells,
 *     the forward/backward difference pair summed Crank-Nicolson style into
 *     the pointwise operator T (a^{t+1}, b^{t+1} from g, h, nu, xi), the two
 *     staggered grids ("whole" z^0, z^1, ... and "fractional" z^{1/2},
 *     z^{3/2}, ...) advanced leap-frog style, and the start-up
 *     z^{1/2} = T(z^0) taken with the time step dt/2.
 *
 * It is written to be read against the paper, not to be fast: plain loops in
 * the order of the paper's CPU loop (for m, for n), every neighbour read
 * through an accessor that returns zero outside the computational box, no
 * blocking, fusion or reordering.  OpenMP splits the m loop only; every cell
 * of a half-step is independent, so threading does not change a single bit.
 *
 * Readings of points where the paper is silent or garbled (each is also
 * listed in the design notes):
 *   R1  N_x is the number of harmonics kept: a_0..a_{N_x-1}, b_1..b_{N_x-1}.
 *   R3  phi_y(m) = phi_min + m*dphi, dphi = (phi_max-phi_min)/(N_y-1).
 *   R4  the coupling coefficient is B*h/(4*dphi): the continuous equations
 *       of Sec. 2 carry no alpha in the transport terms; alpha enters only
 *       the normalisation of a^(0) and of v_dr.
 *   R5  b^{t+1} = (g mu^{t+1} + h nu)/(nu^2 + (mu^{t+1})^2): Cramer's rule
 *       on nu a + mu b = g, nu b - mu a = h, which is what the summed
 *       forward/backward equations give (the printed sign of the h nu term
 *       would flip b every step at mu = 0).
 *   R6  sigma(0) = 1/2, sigma(n >= 1) = 1 (the printed "n != 1" reads n != 0).
 *   R8  b_0 is a fixed zero cell and is never updated.
 *   R9  start-up: T with every dt replaced by dt/2 (nu, xi, mu, the coupling
 *       coefficient, a^(0) dt), coupling from z^0, field times 0 and dt/2.
 *   R10 the whole-grid step k -> k+1 evaluates mu^t at t = k dt and mu^{t+1}
 *       at (k+1) dt; the fractional step k+1/2 -> k+3/2 at (k+1/2) dt and
 *       (k+3/2) dt.  Times are j*(dt/2) from an integer half-step index j.
 *   R11 within a step the whole grid is advanced first (coupling from the
 *       fractional grid at k+1/2), then the fractional grid (coupling from
 *       the new whole grid at k+1).
 *   R13 observables are taken on the whole grid at integer steps with the
 *       rectangle rule dphi * sum_m.
 *   R14 averages run over steps k in (win_lo, win_hi] with equal weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

typedef struct {
    int32_t nx;          /* harmonics kept (R1) */
    int32_t ny;          /* phi_y points, both ends included (R3) */
    double phiy_min, phiy_max;
    double E_dc, E_w, omega, B, mu, alpha, dt;
    int32_t n_threads;   /* <= 0: OpenMP default */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* Modified Bessel ratios I_n(mu)/I_0(mu), n = 0..nmax.                     */
/* Sec. 2 needs I_n(mu)/I_0(mu) for the equilibrium coefficients a^(0)_n    */
/* and I_0/I_1 for the absorption.  Miller's backward recurrence            */
/* I_{k-1} = (2k/mu) I_k + I_{k+1}, started from (0, tiny) far above nmax;  */
/* the minimal solution dominates on the way down, and since only ratios    */
/* to I_0 are returned no absolute normalisation is needed.  Values are     */
/* rescaled on the way down so that the recurrence stays finite.            */
/* ------------------------------------------------------------------------ */
int oracle_bessel_ratios(double mu, int32_t nmax, double* out)
{
    if (!(mu > 0.0) || nmax < 0 || out == NULL) return -1;
    int32_t start = nmax + 40 + (int32_t)(2.0 * sqrt(40.0 * mu)) + (int32_t)mu;
    if (start < 60) start = 60;
    double* I = (double*)calloc((size_t)start + 2, sizeof(double));
    if (!I) return -2;
    I[start + 1] = 0.0;
    I[start] = 1e-300;
    for (int32_t k = start; k >= 1; --k) {
        I[k - 1] = (2.0 * k / mu) * I[k] + I[k + 1];
        if (I[k - 1] > 1e250) {                 /* rescale to stay finite */
            for (int32_t j = k - 1; j <= start + 1; ++j) I[j] *= 1e-250;
        }
    }
    for (int32_t n = 0; n <= nmax; ++n) out[n] = I[n] / I[0];
    free(I);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Grid state: four arrays [n][m], n in [0,nx), m in [0,ny).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny;
    double* a;   /* a_n(phi_y(m)) */
    double* b;   /* b_n(phi_y(m)); row n = 0 is identically zero (R8) */
} grid_t;

/* Boundary conditions of Sec. 3: a is zero outside n in [0,N], b outside
   n in [1,N], both outside m in [0,M]. */
static double get_a(const grid_t* g, int32_t n, int32_t m)
{
    if (n < 0 || n >= g->nx || m < 0 || m >= g->ny) return 0.0;
    return g->a[(size_t)n * g->ny + m];
}
static double get_b(const grid_t* g, int32_t n, int32_t m)
{
    if (n < 1 || n >= g->nx || m < 0 || m >= g->ny) return 0.0;
    return g->b[(size_t)n * g->ny + m];
}

/* chi(n) of the Fourier system (Sec. 2): 2 for n = 1, else 1. */
static double chi(int32_t n) { return n == 1 ? 2.0 : 1.0; }

static double phi_y(const oracle_params* p, int32_t m)
{
    double dphi = (p->phiy_max - p->phiy_min) / (double)(p->ny - 1);
    return p->phiy_min + (double)m * dphi;
}

/* E(t) = E_dc + E_w cos(omega t) (Sec. 2). */
static double field_E(const oracle_params* p, double t)
{
    return p->E_dc + p->E_w * cos(p->omega * t);
}

/* beta^t_m = E^t + B phi_y(m)  (Sec. 3, definitions under the
   forward/backward equations). */
static double beta(const oracle_params* p, double t, int32_t m)
{
    return field_E(p, t) + p->B * phi_y(p, m);
}

/* a^(0)_{n,m} = sigma(n) I_n/(pi I_0) sqrt(mu/(2 pi alpha)) exp(-mu phi_y^2/2)
   (Sec. 2, Fourier coefficients of the Boltzmann equilibrium; R6). */
static double a0_coef(const oracle_params* p, const double* ratio, int32_t n, int32_t m)
{
    double sigma = (n == 0) ? 0.5 : 1.0;
    double py = phi_y(p, m);
    return sigma * ratio[n] / ORACLE_PI * sqrt(p->mu / (2.0 * ORACLE_PI * p->alpha))
           * exp(-0.5 * p->mu * py * py);
}

/* ------------------------------------------------------------------------ */
/* Operator T (Sec. 3): one Crank-Nicolson step of length h for a single    */
/* cell, given its own old value (a, b), the coupling terms A^t, B^t        */
/* already multiplied by their coefficient, the source a^(0), and          */
/* mu^t = n beta^t h/2, mu^{t+1} = n beta^{t+1} h/2.                        */
/* ------------------------------------------------------------------------ */
static void op_T(double a, double b, double A, double Bc, double a0, double h,
                 double mu_t, double mu_t1, double* a_new, double* b_new)
{
    double nu = 1.0 + h / 2.0;
    double xi = 1.0 - h / 2.0;
    double g = a * xi - b * mu_t + Bc + a0 * h;
    double hh = b * xi + a * mu_t + A;
    double den = nu * nu + mu_t1 * mu_t1;
    *a_new = (g * nu - hh * mu_t1) / den;
    *b_new = (g * mu_t1 + hh * nu) / den;   /* R5 */
}

/* ------------------------------------------------------------------------ */
/* One half-step: grid X advances by h from time t0 to t1, its coupling     */
/* terms A^t, B^t read from grid Y (Sec. 3, leap-frog on staggered grids).  */
/* X(n,m) depends only on its own old value and on Y, so X is updated in    */
/* place.                                                                   */
/* ------------------------------------------------------------------------ */
static void half_step(const oracle_params* p, const double* a0, grid_t* X,
                      const grid_t* Y, double h, double t0, double t1)
{
    double dphi = (p->phiy_max - p->phiy_min) / (double)(p->ny - 1);
    double cc = p->B * h / (4.0 * dphi);                     /* R4 */
    int32_t nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int32_t m = 0; m < ny; ++m) {
        double beta0 = beta(p, t0, m);
        double beta1 = beta(p, t1, m);
        for (int32_t n = 0; n < nx; ++n) {
            double A = cc * (chi(n) * (get_a(Y, n - 1, m + 1) - get_a(Y, n - 1, m - 1))
                             - get_a(Y, n + 1, m + 1) + get_a(Y, n + 1, m - 1));
            double Bc = cc * (get_b(Y, n + 1, m + 1) - get_b(Y, n + 1, m - 1)
                              - get_b(Y, n - 1, m + 1) + get_b(Y, n - 1, m - 1));
            double mu_t = (double)n * beta0 * h / 2.0;
            double mu_t1 = (double)n * beta1 * h / 2.0;
            double a_new, b_new;
            op_T(get_a(X, n, m), get_b(X, n, m), A, Bc, a0[(size_t)n * ny + m], h,
                 mu_t, mu_t1, &a_new, &b_new);
            X->a[(size_t)n * ny + m] = a_new;
            if (n >= 1) X->b[(size_t)n * ny + m] = b_new;    /* R8 */
        }
    }
}

/* Drift velocity v_dr = pi sqrt(alpha) \int b_1 dphi_y and norm
   2 pi sqrt(alpha) \int a_0 dphi_y (Sec. 2), rectangle rule (R13). */
static double drift_velocity(const oracle_params* p, const grid_t* g)
{
    double dphi = (p->phiy_max - p->phiy_min) / (double)(p->ny - 1);
    double s = 0.0;
    for (int32_t m = 0; m < p->ny; ++m) s += get_b(g, 1, m);
    return ORACLE_PI * sqrt(p->alpha) * dphi * s;
}
static double norm_of(const oracle_params* p, const grid_t* g)
{
    double dphi = (p->phiy_max - p->phiy_min) / (double)(p->ny - 1);
    double s = 0.0;
    for (int32_t m = 0; m < p->ny; ++m) s += get_a(g, 0, m);
    return 2.0 * ORACLE_PI * sqrt(p->alpha) * dphi * s;
}

/* Compensated (Kahan) accumulation for the window sums. */
typedef struct { double s, c; } kahan_t;
static void kahan_add(kahan_t* k, double x)
{
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

static int check_params(const oracle_params* p)
{
    if (p->nx < 2 || p->ny < 3) return -1;
    if (!(p->phiy_max > p->phiy_min)) return -1;
    if (!(p->dt > 0.0) || !(p->mu > 0.0) || !(p->alpha > 0.0)) return -1;
    return 0;
}

/*
 * Run the scheme.
 *
 *   k0            integer step of the state passed in (0 for a fresh start).
 *   n_steps       number of whole steps to take: k0 -> k0 + n_steps.
 *   a_h, b_h      in/out [nx][ny] whole-grid state at step k0.  If init_f0
 *                 is nonzero they are overwritten with the equilibrium
 *                 a = a^(0), b = 0 (Sec. 2, initial condition).
 *   a_f, b_f      in/out [nx][ny] fractional-grid state at step k0 + 1/2.
 *                 If do_startup is nonzero it is computed from the whole
 *                 grid by the start-up half-step (R9); k0 must then be 0
 *                 for the field times to be those of the paper.
 *   win_lo,win_hi averaging window: steps k with win_lo < k <= win_hi.
 *   v_trace, norm_trace  optional [n_steps] arrays of v_dr and norm at
 *                 steps k0+1 .. k0+n_steps.
 *   obs           out [7]: v_dr, norm at the last step, S_v, S_vc, K,
 *                 <v> = S_v/K, A = (2 I_0/I_1) S_vc/K (Sec. 2, absorption).
 *                 K = 0 leaves the averages at 0.
 */
int oracle_run(const oracle_params* p, int64_t k0, int64_t n_steps, int32_t init_f0,
               int32_t do_startup, double* a_h, double* b_h, double* a_f, double* b_f,
               int64_t win_lo, int64_t win_hi, double* v_trace, double* norm_trace,
               double* obs)
{
    if (!p || check_params(p) != 0 || n_steps < 0 || !a_h || !b_h || !a_f || !b_f) return -1;
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#endif
    int32_t nx = p->nx, ny = p->ny;
    double* ratio = (double*)malloc(sizeof(double) * (size_t)(nx + 1));
    if (!ratio) return -2;
    if (oracle_bessel_ratios(p->mu, nx, ratio) != 0) { free(ratio); return -1; }

    /* the equilibrium array a0(n,m), kept like the paper's a0 array */
    double* a0 = (double*)malloc(sizeof(double) * (size_t)nx * ny);
    if (!a0) { free(ratio); return -2; }
    for (int32_t n = 0; n < nx; ++n)
        for (int32_t m = 0; m < ny; ++m) a0[(size_t)n * ny + m] = a0_coef(p, ratio, n, m);

    grid_t H = {nx, ny, a_h, b_h};
    grid_t F = {nx, ny, a_f, b_f};

    if (init_f0) {                      /* a_n(0) = a^(0)_n, b_n(0) = 0 */
        memcpy(a_h, a0, sizeof(double) * (size_t)nx * ny);
        memset(b_h, 0, sizeof(double) * (size_t)nx * ny);
    }
    for (int32_t m = 0; m < ny; ++m) { b_h[m] = 0.0; }   /* R8 */

    double dt = p->dt;
    double half = 0.5 * dt;
    if (do_startup) {                   /* z^{1/2} = T_{dt/2}(z^0; coupling from z^0) */
        memcpy(a_f, a_h, sizeof(double) * (size_t)nx * ny);
        memcpy(b_f, b_h, sizeof(double) * (size_t)nx * ny);
        grid_t Z0 = {nx, ny, a_h, b_h};
        half_step(p, a0, &F, &Z0, half, (double)(2 * k0) * half, (double)(2 * k0 + 1) * half);
    }
    for (int32_t m = 0; m < ny; ++m) { b_f[m] = 0.0; }

    kahan_t Sv = {0, 0}, Svc = {0, 0};
    int64_t K = 0;
    double v = drift_velocity(p, &H), nrm = norm_of(p, &H);
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t k = k0 + s;
        /* whole grid: z^{k+1} = T(z^k; A, B from z^{k+1/2}) */
        half_step(p, a0, &H, &F, dt, (double)(2 * k) * half, (double)(2 * k + 2) * half);
        /* fractional grid: z^{k+3/2} = T(z^{k+1/2}; A, B from z^{k+1}) */
        half_step(p, a0, &F, &H, dt, (double)(2 * k + 1) * half, (double)(2 * k + 3) * half);
        v = drift_velocity(p, &H);
        nrm = norm_of(p, &H);
        if (v_trace) v_trace[s] = v;
        if (norm_trace) norm_trace[s] = nrm;
        int64_t kk = k + 1;
        if (kk > win_lo && kk <= win_hi) {
            double t = (double)(2 * kk) * half;
            kahan_add(&Sv, v);
            kahan_add(&Svc, v * cos(p->omega * t));
            K += 1;
        }
    }
    if (obs) {
        obs[0] = v;
        obs[1] = nrm;
        obs[2] = Sv.s;
        obs[3] = Svc.s;
        obs[4] = (double)K;
        obs[5] = K > 0 ? Sv.s / (double)K : 0.0;
        obs[6] = K > 0 ? (2.0 / ratio[1]) * Svc.s / (double)K : 0.0;
    }
    free(a0);
    free(ratio);
    return 0;
}

/* Equilibrium coefficients a^(0)_{n,m} as an [nx][ny] array (Sec. 2). */
int oracle_equilibrium(const oracle_params* p, double* a0)
{
    if (!p || check_params(p) != 0 || !a0) return -1;
    double* ratio = (double*)malloc(sizeof(double) * (size_t)(p->nx + 1));
    if (!ratio) return -2;
    oracle_bessel_ratios(p->mu, p->nx, ratio);
    for (int32_t n = 0; n < p->nx; ++n)
        for (int32_t m = 0; m < p->ny; ++m) a0[(size_t)n * p->ny + m] = a0_coef(p, ratio, n, m);
    free(ratio);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
