/*
 * Drift velocity of the periodic state by characteristic curves (FP64, CPU).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory: nothing on the
 * product path links, loads or calls it, and it shares nothing with the HIP
 * library.
 *
 * What it computes (arXiv:1401.6047, Sec. 4, the zero-temperature check of
 * Fig. 4).  The transport terms of the BTE of Sec. 2 move phase-space points
 * along the pendulum flow (Eqs. pendulum_phi_x, pendulum_phi_y)
 *
 *     d phi_x / dt = E(t) + B phi_y,      d phi_y / dt = -B sin(phi_x),
 *
 * which has zero divergence, and the collision term relaxes f to f0 at unit
 * rate.  Integrating along the flow therefore gives, for any temperature,
 *
 *     v_dr(t) = \int_0^inf e^{-tau} < sin Phi_x(t; t - tau, p0) >_{f0} d tau,
 *
 * where Phi(t; t0, p0) is the flow from the point p0 at time t0 and < >_{f0}
 * averages p0 over the equilibrium distribution normalised as in Sec. 2.  In
 * the zero-temperature limit f0 is a point mass at the origin and this is the
 * exponential-memory drift velocity of Eq. pendulum_drift_velocity; at finite
 * temperature it is the exact continuum solution that the finite-difference
 * scheme approximates.
 *
 * Discretisation (none of it is taken from the paper, which states only the
 * equations):
 *   - the average over p0 is a weighted sum over caller-supplied nodes
 *     (x0[q], y0[q], w[q]), sum w = 1;
 *   - launch times t0 = j h, j = 0 .. n_launch-1, with n_launch h = 2 pi/omega
 *     when E_w != 0 (the state is periodic, so launches one period apart give
 *     time-shifted copies of the same trajectories and one period of launches
 *     is enough); with E_w = 0 the field is constant and n_launch may be 1;
 *   - each trajectory advances by classical fourth-order Runge-Kutta with step
 *     h for tau up to tau_max (truncation e^{-tau_max});
 *   - the tau integral is the trapezoid rule with step h plus the h^2/12
 *     end-point term of the Euler-Maclaurin formula at tau = 0 (the far end
 *     vanishes), which makes it fourth order;
 *   - the value of launch j at tau = k h lands in output slot (j + k) mod
 *     n_launch, i.e. v(t_i) with t_i = i h.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHAR_PI 3.14159265358979323846

/* Right-hand side of the pendulum flow at field value e. */
static void flow(double e, double B, double x, double y, double* dx, double* dy)
{
    *dx = e + B * y;
    *dy = -B * sin(x);
}

int oracle_characteristic_v(double E_dc, double E_w, double omega, double B,
                            int32_t n_nodes, const double* x0, const double* y0,
                            const double* w, int32_t n_launch, double h,
                            double tau_max, int32_t n_threads, double* v)
{
    if (n_nodes < 1 || !x0 || !y0 || !w || !v || n_launch < 1 || !(h > 0.0) ||
        !(tau_max > 0.0) || !isfinite(E_dc) || !isfinite(E_w) || !isfinite(B))
        return -1;
    if (E_w != 0.0) {
        if (!(omega > 0.0)) return -1;
        double period = 2.0 * CHAR_PI / omega;
        if (fabs(n_launch * h - period) > 1e-12 * period) return -2;
    }
    const int64_t n_tau = (int64_t)ceil(tau_max / h);
    /* E at every half step of the launch grid, one period long: index s is
       time s h / 2 (mod the period when the field oscillates). */
    const int64_t n_half = 2 * (int64_t)n_launch;
    double* field = (double*)malloc(sizeof(double) * (size_t)n_half);
    if (!field) return -3;
    for (int64_t s = 0; s < n_half; ++s)
        field[s] = E_dc + E_w * cos(omega * ((double)s * 0.5 * h));
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    int nt = 1;
    (void)n_threads;
#endif
    /* row j holds the contributions of the points launched at t_j to every
       sample time; the rows are summed in order afterwards, so the result
       does not depend on the thread count or on which thread ran which j */
    double* part = (double*)calloc((size_t)n_launch * (size_t)n_launch, sizeof(double));
    if (!part) { free(field); return -3; }
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1) reduction(|: bad)
#endif
    for (int32_t j = 0; j < n_launch; ++j) {
        double* acc = part + (size_t)j * n_launch;
        for (int32_t q = 0; q < n_nodes; ++q) {
            double x = x0[q], y = y0[q];
            /* tau = 0: trapezoid end weight 1/2, and the Euler-Maclaurin
               term h^2/12 * d/dtau[e^{-tau} sin Phi_x] at tau = 0, divided
               by h because the slot is scaled by h at the end. */
            double e0 = field[(2 * (int64_t)j) % n_half];
            double dfdtau = -sin(x) + cos(x) * (e0 + B * y);
            acc[j] += w[q] * (0.5 * sin(x) + (h / 12.0) * dfdtau);
            for (int64_t k = 1; k <= n_tau; ++k) {
                /* one RK4 step from time (j + k - 1) h to (j + k) h */
                int64_t s = 2 * ((int64_t)j + k - 1);
                double ea = field[s % n_half];
                double em = field[(s + 1) % n_half];
                double eb = field[(s + 2) % n_half];
                double k1x, k1y, k2x, k2y, k3x, k3y, k4x, k4y;
                flow(ea, B, x, y, &k1x, &k1y);
                flow(em, B, x + 0.5 * h * k1x, y + 0.5 * h * k1y, &k2x, &k2y);
                flow(em, B, x + 0.5 * h * k2x, y + 0.5 * h * k2y, &k3x, &k3y);
                flow(eb, B, x + h * k3x, y + h * k3y, &k4x, &k4y);
                x += (h / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
                y += (h / 6.0) * (k1y + 2.0 * k2y + 2.0 * k3y + k4y);
                acc[(j + k) % n_launch] += w[q] * exp(-(double)k * h) * sin(x);
            }
            if (!isfinite(x) || !isfinite(y)) bad = 1;
        }
    }
    for (int32_t i = 0; i < n_launch; ++i) {
        double s = 0.0;
        for (int32_t j = 0; j < n_launch; ++j) s += part[(size_t)j * n_launch + i];
        v[i] = h * s;
    }
    free(part);
    free(field);
    return bad ? -4 : 0;
}
