// Internal declarations shared by the kernels and the host runtime of the
// superlattice BTE solver.  Not part of the public C ABI (include/bte.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace bte {

// Memory layout of one state plane (a_h, b_h, a_f or b_f):
//   rows n = -kPadRows .. n_x - 1 + kPadRows, row stride `ld` elements,
//   column m of the paper's phi_y lattice stored at physical column m + kPadCols.
// Everything outside 0 <= n < n_x, 0 <= m < n_y is zero and never written, so
// the stencil's boundary conditions (zero cells around the box) cost no branch.
constexpr int kPadRows = 4;
constexpr int kPadCols = 4;
constexpr int kWave = 64;
// Output columns of one wavefront.  A half-step needs the other grid one
// column beyond its outputs, so a tile chaining h half-steps in registers
// keeps h halo lanes on each side: the single half-step h = 1, the fused
// step h = 2, the two-step kernel h = 4, the three-step kernel h = 6.
constexpr int kHalfCols = kWave - 2;
constexpr int kFusedCols = kWave - 4;
constexpr int kFused2Cols = kWave - 8;
constexpr int kFused3Cols = kWave - 12;

// Largest physical column (m + kPadCols) any tile of a kernel with `cols`
// output columns and `halo` halo lanes touches for an N_y-column grid, + 1.
inline int col_extent(int ny, int cols, int halo)
{
    const int tiles = (ny + cols - 1) / cols;
    return (tiles - 1) * cols - halo + kWave - 1 + kPadCols + 1;
}

// Device-resident control block, read by every step kernel.  Keeping the step
// counter on the device lets one captured graph be replayed for any k.
struct Ctl {
    int64_t k;        // whole step of the current state
    int64_t win_lo;   // averaging window: win_lo < k+1 <= win_hi
    int64_t win_hi;
    double norm_ref;  // sum_m a_0(m) of the initial state (stability check)
    double norm_eq;   // sum_m a0_{0,m} = s_0 sum_m g_m: the value sum_m a_0 relaxes to
};

// Per-solver scalars, fixed at creation.
struct Consts {
    int32_t nx, ny, ld;
    int32_t pad;
    double dt;        // time step
    double half_dt;   // a half-step index j is the time j * half_dt
    double phimin, dphi;
    double B, E_dc, E_w, omega;
    double c_full;    // B dt / (4 dphi): coupling coefficient of a full step
    double nu, xi;    // 1 + dt/2, 1 - dt/2
};

template <typename T>
struct Planes {
    T* a_h;
    T* b_h;
    T* a_f;
    T* b_f;
};

// Launch shapes (see bte_tuning in the public header).
struct Shape {
    int rows_per_wave;
    int waves_per_block;
};

// ---- host helpers (bte_solver.hip) -----------------------------------------
// Checked arguments of the state-observables entry points.
struct StateObsArgs {
    Consts cs;        // nx, ny, ld set; the rest zero
    double f;         // pi sqrt(alpha) dphi
    int edge_w;       // phi_y points per edge strip
    int top_from;     // first harmonic of the top of the spectrum
};
// Validate (a, b, n_x, n_y, ld, box, alpha, out) as bte_state_observables
// documents; sets bte_last_error and returns BTE_EINVAL on failure.
int state_obs_validate(const double* a, const double* b, int32_t n_x, int32_t n_y, int64_t ld,
                       double phiy_min, double phiy_max, double alpha, const double* out,
                       StateObsArgs& v);
// Byte offset of the reduction outputs after the partial sums of nx rows.
size_t state_obs_red_offset(int nx);
// Message returned by bte_last_error() on this thread.
void set_last_error(const char* msg);
// I_n(mu)/I_0(mu) for n = 0..nmax.
std::vector<double> bessel_ratio_table(double mu, int nmax);

// ---- launchers (bte_kernels.hip) ------------------------------------------
// All pointers to planes point at logical (n = 0, m = 0).

// One fused leap-frog step: whole grid k -> k+1 from `src`, fractional grid
// k+1/2 -> k+3/2, both written to `dst`.  The step index is ctl->k + j_off.
template <typename T>
hipError_t launch_fused_step(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                             const double* s_n, const double* g_m, double* acc_v,
                             double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st);

// Three fused leap-frog steps k -> k+3 in one pass (six half-steps chained in
// registers), from `src` to `dst`.  The step index is ctl->k + j_off.
template <typename T>
hipError_t launch_fused_step3(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                              const double* s_n, const double* g_m, double* acc_v,
                              double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st);

// Two fused leap-frog steps k -> k+2 in one pass (four half-steps chained in
// registers), from `src` to `dst`.  The step index is ctl->k + j_off.
template <typename T>
hipError_t launch_fused_step2(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                              const double* s_n, const double* g_m, double* acc_v,
                              double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st);

// One half-step in place: X <- T(X; coupling from Y) with step h between
// half-step times 2*(ctl->k + j_off) + off0 and 2*(ctl->k + j_off) + off1.
// When `accumulate` is set the new b_1 row enters the window sums at step
// ctl->k + j_off + 1.
template <typename T>
hipError_t launch_half_step(const Consts& cs, const Shape& sh, T* xa, T* xb, const T* ya,
                            const T* yb, const double* s_n, const double* g_m, double h,
                            int off0, int off1, int accumulate, double* acc_v, double* acc_vc,
                            const Ctl* ctl, int j_off, hipStream_t st);

// Fill the whole grid with the equilibrium a = s_n g_m, b = 0 (padding zero).
template <typename T>
hipError_t launch_init_equilibrium(const Consts& cs, T* a, T* b, const double* s_n,
                                   const double* g_m, hipStream_t st);

// ctl->k += n (one thread, vector store).
hipError_t launch_advance_counter(Ctl* ctl, int64_t n, hipStream_t st);

// Observables of a whole-grid state, reduced in a fixed order (deterministic):
// one workgroup per harmonic row (plus one for the window sums) writes its
// partial sums to `part` (3 * (nx + 1) doubles), then one workgroup combines
// them into out[0..6]:
//   out[0] = sum_m a_0(m)            out[1] = sum_m b_1(m)
//   out[2] = sum_m acc_v(m)          out[3] = sum_m acc_vc(m)   (0 if acc_v is NULL)
//   out[4] = sum over the edge strips (edge_w points each side) of |a_0(m)|
//   out[5] = sum_m [2 a_0^2 + sum_{n>=1} (a_n^2 + b_n^2)]
//   out[6] = the same sum over harmonics n >= top_from only.
// a_h, b_h point at logical (0, 0) of planes with row stride cs.ld.
constexpr int kObsOut = 7;
template <typename T>
hipError_t launch_reduce_obs(const Consts& cs, const T* a_h, const T* b_h, const double* acc_v,
                             const double* acc_vc, int edge_w, int top_from, double* part,
                             double* out, hipStream_t st);

// launch_reduce_obs on caller arrays (no window sums), then out[0..3] =
// (norm, v_dr, edge_mass, top_harm_mass) with f = pi sqrt(alpha) dphi.
// `part` holds 3 * (nx + 1) doubles, `red` kObsOut.
hipError_t launch_state_observables(const Consts& cs, const double* a, const double* b,
                                   int edge_w, int top_from, double f, double* part,
                                   double* red, double* out, hipStream_t st);

// Stability check of the state after a run of steps: if sum_m a_0(m) or
// sum_m b_1(m) is not finite, or sum_m a_0 lies further from its equilibrium
// value ctl->norm_eq than the initial state did (ctl->norm_ref) by more than
// 1e-2 of norm_eq, store 1 into *flag (host-visible memory, system scope).
// Relaxation moves sum_m a_0 monotonically from norm_ref toward norm_eq
// (factor xi/nu per step); the transport only adds the flux through the box
// edges, which is negligible for a resolved state.
template <typename T>
hipError_t launch_check_stable(const Consts& cs, const T* a_h, const T* b_h, const Ctl* ctl,
                               int* flag, hipStream_t st);

}  // namespace bte
