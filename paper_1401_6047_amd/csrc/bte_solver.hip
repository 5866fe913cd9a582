// Host runtime and C ABI of the superlattice BTE solver (see include/bte.h).
//
// A solver owns a device workspace laid out as
//   [ctl | reduction | s_n | g_m | acc_v | acc_vc | 8 state planes]
// (two ping-pong sets of a_h, b_h, a_f, b_f).  The host computes the few
// O(N_x + N_y) constants (Bessel ratios, the phi_y envelope of the
// equilibrium) once; every per-cell operation runs in the kernels.
// Steps are queued as replays of a captured HIP graph of `graph_steps`
// launches plus direct launches for the remainder; the step counter lives on
// the device, so one graph serves every k.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"
#include "bte_reconstruct.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace bte {

void set_last_error(const char* msg) { g_last_error = msg; }

// I_n(mu)/I_0(mu) for n = 0..nmax.  The ratios r_n = I_n/I_{n-1} satisfy
// r_n = 1/(2n/mu + r_{n+1}) (the three-term recurrence divided through);
// iterating that continued fraction downward from far above nmax converges
// to the minimal solution, and I_n/I_0 is the running product of r_1..r_n.
std::vector<double> bessel_ratio_table(double mu, int nmax)
{
    int top = nmax + 64 + static_cast<int>(4.0 * std::sqrt(mu + 1.0) + mu);
    std::vector<double> r(top + 2, 0.0);
    double next = 0.0;
    for (int n = top; n >= 1; --n) {
        next = 1.0 / (2.0 * n / mu + next);
        r[n] = next;
    }
    std::vector<double> out(nmax + 1);
    out[0] = 1.0;
    double p = 1.0;
    for (int n = 1; n <= nmax; ++n) {
        p *= r[n];
        out[n] = p;
    }
    return out;
}

size_t state_obs_red_offset(int nx)
{
    return (3 * sizeof(double) * (nx + 1) + 255) / 256 * 256;
}

}  // namespace bte

namespace {
using bte::bessel_ratio_table;

bte_status fail(bte_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(BTE_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
// A wave keeps the source coefficients of its rows (plus one halo row on each
// side) one per lane.
constexpr int kMaxRowsPerWave = bte::kWave - 2;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int ld = 0;             // row stride of a plane, elements
    int rows = 0;           // padded rows per plane
    size_t elem = 8;        // bytes per state element
    size_t plane_bytes = 0;
    size_t off_ctl = 0, off_red = 0, off_part = 0, off_s = 0, off_g = 0, off_accv = 0,
           off_accvc = 0;
    size_t off_planes = 0;
    size_t total = 0;
};

Layout make_layout(const bte_grid& g, int precision)
{
    Layout L;
    using namespace bte;
    int need = std::max({col_extent(g.n_y, kHalfCols, 1), col_extent(g.n_y, kFusedCols, 2),
                         col_extent(g.n_y, kFused2Cols, 4), col_extent(g.n_y, kFused3Cols, 6),
                         g.n_y + 2 * kPadCols});
    L.ld = (need + 63) / 64 * 64;
    L.rows = g.n_x + 2 * kPadRows;
    L.elem = precision == BTE_FP32_BULK ? 4 : 8;
    L.plane_bytes = align_up(static_cast<size_t>(L.rows) * L.ld * L.elem);
    size_t o = 0;
    L.off_ctl = o; o += align_up(sizeof(Ctl));
    L.off_red = o; o += align_up(8 * sizeof(double));
    L.off_part = o; o += align_up(3 * sizeof(double) * (g.n_x + 1));
    L.off_s = o; o += align_up(sizeof(double) * g.n_x);
    L.off_g = o; o += align_up(sizeof(double) * g.n_y);
    L.off_accv = o; o += align_up(sizeof(double) * g.n_y);
    L.off_accvc = o; o += align_up(sizeof(double) * g.n_y);
    L.off_planes = o; o += 8 * L.plane_bytes;
    L.total = o;
    return L;
}

bool finite(double x) { return std::isfinite(x); }

bte_status validate(const bte_grid* g, const bte_params* p)
{
    if (!g || !p) return fail(BTE_EINVAL, "grid and params must not be NULL");
    if (g->n_x < 2) return fail(BTE_EINVAL, "n_x must be >= 2 (got %d)", g->n_x);
    if (g->n_y < 3) return fail(BTE_EINVAL, "n_y must be >= 3 (got %d)", g->n_y);
    if (g->n_x > 16384 || g->n_y > (1 << 24))
        return fail(BTE_EINVAL, "grid too large (%d x %d)", g->n_x, g->n_y);
    if (!finite(g->phiy_min) || !finite(g->phiy_max) || !(g->phiy_max > g->phiy_min))
        return fail(BTE_EINVAL, "need finite phiy_min < phiy_max");
    const double vals[] = {p->E_dc, p->E_w, p->omega, p->B, p->mu, p->alpha, p->tau, p->dt};
    for (double v : vals)
        if (!finite(v)) return fail(BTE_EINVAL, "parameters must be finite");
    if (!(p->dt > 0)) return fail(BTE_EINVAL, "dt must be > 0");
    if (!(p->mu > 0)) return fail(BTE_EINVAL, "mu must be > 0");
    if (!(p->alpha > 0)) return fail(BTE_EINVAL, "alpha must be > 0");
    if (p->tau != 1.0) return fail(BTE_EINVAL, "tau must be 1 (time is in units of tau)");
    if (p->E_w != 0.0 && !(p->omega > 0))
        return fail(BTE_EINVAL, "omega must be > 0 when E_w != 0");
    if (p->omega < 0) return fail(BTE_EINVAL, "omega must be >= 0");
    if (p->precision != BTE_FP64 && p->precision != BTE_FP32_BULK)
        return fail(BTE_EINVAL, "unknown precision %d", p->precision);
    if (g->n_x > 16384 || g->n_y > (1 << 24)) return fail(BTE_EINVAL, "grid too large");
    if (p->flags != 0) return fail(BTE_EINVAL, "flags must be 0");
    {
        // kernels address a set of four state planes with 32-bit byte offsets
        const Layout L = make_layout(*g, p->precision);
        if (4.0 * static_cast<double>(L.plane_bytes) >= 2147483648.0)
            return fail(BTE_EINVAL, "grid too large: a set of four state planes must stay below 2 GiB");
    }
    const double dphi = (g->phiy_max - g->phiy_min) / (g->n_y - 1);
    const double cfl = p->dt * std::fabs(p->B) / (2.0 * dphi);
    if (!(cfl < 1.0))
        return fail(BTE_EINVAL, "leap-frog bound violated: dt |B| / (2 dphi) = %g >= 1", cfl);
    return BTE_OK;
}

}  // namespace

struct bte_solver {
    bte_grid grid{};
    bte_params params{};
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    bool owns_ws = false;
    Layout L;
    bte::Consts cs{};
    bte_tuning tune{};
    int cur = 0;                    // ping-pong set holding the current state
    int64_t step = 0;               // host mirror of ctl->k
    int64_t win_lo = 0, win_hi = 0;
    int64_t acc_from = 0;           // accumulators count steps > acc_from
    double ratio1 = 0;              // I_1(mu)/I_0(mu)
    double norm0 = 0;               // normalisation of the initial state
    double norm_ref = 0;            // sum_m a_0(m) of the initial state (device check)
    double norm_eq = 0;             // sum_m a0_{0,m}: the value sum_m a_0 relaxes to
    bool unstable = false;
    int* flag_host = nullptr;       // sticky instability flag, written by the device
    int* flag_dev = nullptr;        // its device address
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // by starting set
    bool graph_flip[2] = {false, false};            // graph ends in the other set
    int graph_steps_built = -1;
    double* pinned = nullptr;       // host landing buffer for reductions

    bte::Ctl* ctl() { return reinterpret_cast<bte::Ctl*>(ws + L.off_ctl); }
    double* red() { return reinterpret_cast<double*>(ws + L.off_red); }
    double* part() { return reinterpret_cast<double*>(ws + L.off_part); }
    double* s_n() { return reinterpret_cast<double*>(ws + L.off_s); }
    double* g_m() { return reinterpret_cast<double*>(ws + L.off_g); }
    double* acc_v() { return reinterpret_cast<double*>(ws + L.off_accv); }
    double* acc_vc() { return reinterpret_cast<double*>(ws + L.off_accvc); }
    char* plane_base(int set, int which) { return ws + L.off_planes + (set * 4 + which) * L.plane_bytes; }
    // pointer to logical (n = 0, m = 0)
    template <typename T>
    T* plane(int set, int which)
    {
        return reinterpret_cast<T*>(plane_base(set, which)) + bte::kPadRows * L.ld + bte::kPadCols;
    }
    template <typename T>
    bte::Planes<T> planes(int set)
    {
        return bte::Planes<T>{plane<T>(set, 0), plane<T>(set, 1), plane<T>(set, 2), plane<T>(set, 3)};
    }
    bool fp32() const { return params.precision == BTE_FP32_BULK; }
};

namespace {

void drop_graphs(bte_solver* s)
{
    for (auto& g : s->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    s->graph_steps_built = -1;
}

bte_tuning default_tuning(const bte_grid& g)
{
    bte_tuning t{};
    t.kernel = BTE_KERNEL_FUSED;
    // Enough wavefronts to cover the 256 CUs several times over, without
    // chunks so short that the two halo harmonics dominate.
    const long cols = (g.n_y + bte::kFusedCols - 1) / bte::kFusedCols;
    int R = 24;
    while (R > 4 && cols * ((g.n_x + R - 1) / R) < 2048) R = R > 8 ? R / 2 + R / 4 : R - 2;
    t.rows_per_wave = std::min(R, g.n_x);
    t.waves_per_block = 1;
    const double cells = static_cast<double>(g.n_x) * g.n_y;
    // a multiple of 6, so that a graph holds only two-step or only
    // three-step launches (no one-step remainder inside a replay)
    t.graph_steps = cells < 4e6 ? 96 : 48;
    return t;
}

bte_status check_tuning(const bte_tuning& t)
{
    if (t.kernel != BTE_KERNEL_FUSED && t.kernel != BTE_KERNEL_TWO_PASS &&
        t.kernel != BTE_KERNEL_FUSED2 && t.kernel != BTE_KERNEL_FUSED3)
        return fail(BTE_EINVAL, "unknown kernel form %d", t.kernel);
    if (t.rows_per_wave < 1 || t.rows_per_wave > kMaxRowsPerWave)
        return fail(BTE_EINVAL, "rows_per_wave must be in 1..%d", kMaxRowsPerWave);
    if (t.waves_per_block != 1 && t.waves_per_block != 2 && t.waves_per_block != 4 &&
        t.waves_per_block != 8)
        return fail(BTE_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
    if (t.graph_steps < 0 || (t.graph_steps & 1) || t.graph_steps > 4096)
        return fail(BTE_EINVAL, "graph_steps must be even and in 0..4096");
    return BTE_OK;
}

// Queue `count` (1, 2 or 3) steps starting at step offset j_off.
template <typename T>
hipError_t queue_steps_of(bte_solver* s, int j_off, int count, hipStream_t st)
{
    bte::Shape sh{s->tune.rows_per_wave, s->tune.waves_per_block};
    if (s->tune.kernel == BTE_KERNEL_TWO_PASS) {
        // two passes in place on the current set: whole, then fractional
        auto P = s->planes<T>(s->cur);
        hipError_t e = bte::launch_half_step<T>(s->cs, sh, P.a_h, P.b_h, P.a_f, P.b_f, s->s_n(),
                                                s->g_m(), s->cs.dt, 0, 2, 1, s->acc_v(),
                                                s->acc_vc(), s->ctl(), j_off, st);
        if (e != hipSuccess) return e;
        return bte::launch_half_step<T>(s->cs, sh, P.a_f, P.b_f, P.a_h, P.b_h, s->s_n(),
                                        s->g_m(), s->cs.dt, 1, 3, 0, s->acc_v(), s->acc_vc(),
                                        s->ctl(), j_off, st);
    }
    const int src = s->cur, dst = 1 - s->cur;
    hipError_t e;
    if (count == 3)
        e = bte::launch_fused_step3<T>(s->cs, sh, s->planes<T>(src), s->planes<T>(dst), s->s_n(),
                                       s->g_m(), s->acc_v(), s->acc_vc(), s->ctl(), j_off, st);
    else if (count == 2)
        e = bte::launch_fused_step2<T>(s->cs, sh, s->planes<T>(src), s->planes<T>(dst), s->s_n(),
                                       s->g_m(), s->acc_v(), s->acc_vc(), s->ctl(), j_off, st);
    else
        e = bte::launch_fused_step<T>(s->cs, sh, s->planes<T>(src), s->planes<T>(dst), s->s_n(),
                                      s->g_m(), s->acc_v(), s->acc_vc(), s->ctl(), j_off, st);
    s->cur = dst;
    return e;
}

hipError_t queue_steps_direct(bte_solver* s, int n, hipStream_t st)
{
    int j = 0;
    while (j < n) {
        const int kf = s->tune.kernel;
        const int count = (kf == BTE_KERNEL_FUSED3 && n - j >= 3) ? 3
                          : ((kf == BTE_KERNEL_FUSED2 || kf == BTE_KERNEL_FUSED3) && n - j >= 2) ? 2
                                                                                               : 1;
        hipError_t e = s->fp32() ? queue_steps_of<float>(s, j, count, st)
                                 : queue_steps_of<double>(s, j, count, st);
        if (e != hipSuccess) return e;
        j += count;
    }
    if (n > 0) {
        hipError_t e = bte::launch_advance_counter(s->ctl(), n, st);
        if (e != hipSuccess) return e;
        return s->fp32() ? bte::launch_check_stable<float>(s->cs, s->plane<float>(s->cur, 0),
                                                           s->plane<float>(s->cur, 1), s->ctl(),
                                                           s->flag_dev, st)
                         : bte::launch_check_stable<double>(s->cs, s->plane<double>(s->cur, 0),
                                                            s->plane<double>(s->cur, 1), s->ctl(),
                                                            s->flag_dev, st);
    }
    return hipSuccess;
}

// Capture `graph_steps` steps starting from the current ping-pong set.  The
// graph ends in the same set or in the other one (graph_flip), depending on
// how many ping-pong launches it holds.
bte_status build_graph(bte_solver* s)
{
    const int n = s->tune.graph_steps;
    const int start = s->cur;
    if (!s->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = queue_steps_direct(s, n, s->capture_stream);
    hipError_t e2 = hipStreamEndCapture(s->capture_stream, &g);
    s->graph_flip[start] = (s->cur != start);
    s->cur = start;   // capturing executed nothing
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(BTE_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(BTE_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    s->graph[start] = ex;
    return BTE_OK;
}

template <typename T>
bte_status queue_startup(bte_solver* s)
{
    // z^{1/2} = T_{dt/2}(z^0; coupling from z^0): copy z^0 into the fractional
    // planes, then one half-step of length dt/2 at half-step times 0 -> 1
    // (t = 0 and t = dt/2) with the coupling read from the whole grid.
    const int set = s->cur;
    const size_t bytes = s->L.plane_bytes;
    HIP_TRY(hipMemcpyAsync(s->plane_base(set, 2), s->plane_base(set, 0), bytes,
                           hipMemcpyDeviceToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->plane_base(set, 3), s->plane_base(set, 1), bytes,
                           hipMemcpyDeviceToDevice, s->stream));
    auto P = s->planes<T>(set);
    bte::Shape sh{std::min(16, s->grid.n_x), 4};
    // The start-up runs at k = 0 with half-step offsets 0 -> 1 and a step of dt/2.
    HIP_TRY(bte::launch_half_step<T>(s->cs, sh, P.a_f, P.b_f, P.a_h, P.b_h, s->s_n(), s->g_m(),
                                     0.5 * s->cs.dt, 0, 1, 0, s->acc_v(), s->acc_vc(), s->ctl(),
                                     0, s->stream));
    return BTE_OK;
}

bte_status write_ctl(bte_solver* s)
{
    bte::Ctl c{};
    c.k = s->step;
    c.win_lo = s->win_lo;
    c.win_hi = s->win_hi;
    c.norm_ref = s->norm_ref;
    c.norm_eq = s->norm_eq;
    HIP_TRY(hipMemcpyAsync(s->ctl(), &c, sizeof(c), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return BTE_OK;
}

bte_status clear_acc(bte_solver* s)
{
    HIP_TRY(hipMemsetAsync(s->acc_v(), 0, sizeof(double) * s->grid.n_y, s->stream));
    HIP_TRY(hipMemsetAsync(s->acc_vc(), 0, sizeof(double) * s->grid.n_y, s->stream));
    s->acc_from = s->step;
    return BTE_OK;
}

// phi_y points of each edge strip and first harmonic of the top of the
// spectrum for the resolution diagnostics of bte_obs.
int edge_width(int ny) { return std::max(1, (ny + 63) / 64); }
int top_from(int nx) { return nx - std::max(1, nx / 8); }

}  // namespace

int bte::state_obs_validate(const double* a, const double* b, int32_t n_x, int32_t n_y,
                            int64_t ld, double phiy_min, double phiy_max, double alpha,
                            const double* out, StateObsArgs& v)
{
    if (!a || !b || !out) return fail(BTE_EINVAL, "a, b and out must not be NULL");
    const auto misaligned = [](const void* p) {
        return reinterpret_cast<uintptr_t>(p) % alignof(double) != 0;
    };
    if (misaligned(a) || misaligned(b) || misaligned(out))
        return fail(BTE_EINVAL, "a, b and out must be 8-byte aligned");
    if (n_x < 2 || n_x > 16384) return fail(BTE_EINVAL, "n_x must be in 2..16384");
    if (n_y < 3 || n_y > (1 << 24) || ld < n_y || ld > (int64_t(1) << 31) - 1)
        return fail(BTE_EINVAL, "need 3 <= n_y <= 2^24 and n_y <= ld < 2^31");
    if (!std::isfinite(phiy_min) || !std::isfinite(phiy_max) || !(phiy_max > phiy_min))
        return fail(BTE_EINVAL, "need finite phiy_min < phiy_max");
    if (!std::isfinite(alpha) || !(alpha > 0))
        return fail(BTE_EINVAL, "alpha must be finite and > 0");
    v.cs = bte::Consts{};
    v.cs.nx = n_x;
    v.cs.ny = n_y;
    v.cs.ld = static_cast<int32_t>(ld);
    v.f = kPi * std::sqrt(alpha) * ((phiy_max - phiy_min) / (n_y - 1));
    v.edge_w = edge_width(n_y);
    v.top_from = top_from(n_x);
    return BTE_OK;
}

namespace {

// Reduce the current set: out[0..6] as launch_reduce_obs documents.
bte_status reduce(bte_solver* s, double out[bte::kObsOut])
{
    const int set = s->cur;
    const int ew = edge_width(s->grid.n_y), tf = top_from(s->grid.n_x);
    hipError_t e;
    if (s->fp32())
        e = bte::launch_reduce_obs<float>(s->cs, s->plane<float>(set, 0), s->plane<float>(set, 1),
                                          s->acc_v(), s->acc_vc(), ew, tf, s->part(), s->red(),
                                          s->stream);
    else
        e = bte::launch_reduce_obs<double>(s->cs, s->plane<double>(set, 0),
                                           s->plane<double>(set, 1), s->acc_v(), s->acc_vc(), ew,
                                           tf, s->part(), s->red(), s->stream);
    if (e != hipSuccess) return fail(BTE_EDEVICE, "reduction launch: %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpyAsync(s->pinned, s->red(), bte::kObsOut * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::memcpy(out, s->pinned, bte::kObsOut * sizeof(double));
    return BTE_OK;
}

int64_t window_count(const bte_solver* s)
{
    const int64_t lo = std::max(s->win_lo, s->acc_from);
    const int64_t hi = std::min(s->win_hi, s->step);
    return hi > lo ? hi - lo : 0;
}

template <typename T>
bte_status copy_plane_out(bte_solver* s, int set, int which, double* host)
{
    const int nx = s->grid.n_x, ny = s->grid.n_y;
    const T* src = s->plane<T>(set, which);
    std::vector<T> tmp(static_cast<size_t>(nx) * ny);
    HIP_TRY(hipMemcpy2DAsync(tmp.data(), sizeof(T) * ny, src, sizeof(T) * s->L.ld, sizeof(T) * ny,
                             nx, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < tmp.size(); ++i) host[i] = static_cast<double>(tmp[i]);
    return BTE_OK;
}

template <typename T>
bte_status copy_plane_in(bte_solver* s, int set, int which, const double* host, bool zero_row0)
{
    const int nx = s->grid.n_x, ny = s->grid.n_y;
    std::vector<T> tmp(static_cast<size_t>(nx) * ny);
    for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = static_cast<T>(host[i]);
    if (zero_row0) std::fill(tmp.begin(), tmp.begin() + ny, T(0));
    T* dst = s->plane<T>(set, which);
    HIP_TRY(hipMemcpy2DAsync(dst, sizeof(T) * s->L.ld, tmp.data(), sizeof(T) * ny, sizeof(T) * ny,
                             nx, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return BTE_OK;
}

// Record the normalisation of the current state as the reference of the
// stability checks (host: bte_observables; device: after every run of steps)
// and clear the sticky flag.
bte_status measure_norm0(bte_solver* s)
{
    double r[bte::kObsOut];
    bte_status st = reduce(s, r);
    if (st != BTE_OK) return st;
    s->norm0 = 2.0 * kPi * std::sqrt(s->params.alpha) * s->cs.dphi * r[0];
    s->norm_ref = r[0];
    __atomic_store_n(s->flag_host, 0, __ATOMIC_SEQ_CST);
    return write_ctl(s);
}

}  // namespace

extern "C" {

bte_status bte_workspace_bytes(const bte_grid* grid, const bte_params* params, size_t* bytes)
{
    bte_status st = validate(grid, params);
    if (st != BTE_OK) return st;
    if (!bytes) return fail(BTE_EINVAL, "bytes must not be NULL");
    *bytes = make_layout(*grid, params->precision).total;
    return BTE_OK;
}

bte_status bte_create(const bte_grid* grid, const bte_params* params, void* workspace,
                      size_t workspace_bytes, void* hip_stream, bte_solver** out)
{
    if (!out) return fail(BTE_EINVAL, "out must not be NULL");
    *out = nullptr;
    bte_status st = validate(grid, params);
    if (st != BTE_OK) return st;
    Layout L = make_layout(*grid, params->precision);
    if (workspace && workspace_bytes < L.total)
        return fail(BTE_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return fail(BTE_EINVAL, "workspace must be 256-byte aligned");

    bte_solver* s = new bte_solver();
    s->grid = *grid;
    s->params = *params;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->L = L;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(BTE_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (workspace) {
        s->ws = static_cast<char*>(workspace);
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&s->ws), L.total);
        if (e != hipSuccess) {
            delete s;
            return fail(BTE_ENOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
        }
        s->owns_ws = true;
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&s->pinned), 8 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->flag_host), sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        *s->flag_host = 0;
        e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->flag_dev), s->flag_host, 0);
    }
    if (e != hipSuccess) {
        bte_destroy(s);
        return fail(BTE_ENOMEM, "pinned host buffers: %s", hipGetErrorString(e));
    }

    const double dphi = (grid->phiy_max - grid->phiy_min) / (grid->n_y - 1);
    bte::Consts& cs = s->cs;
    cs.nx = grid->n_x;
    cs.ny = grid->n_y;
    cs.ld = L.ld;
    cs.dt = params->dt;
    cs.half_dt = 0.5 * params->dt;
    cs.phimin = grid->phiy_min;
    cs.dphi = dphi;
    cs.B = params->B;
    cs.E_dc = params->E_dc;
    cs.E_w = params->E_w;
    cs.omega = params->omega;
    cs.c_full = params->B * params->dt / (4.0 * dphi);
    cs.nu = 1.0 + 0.5 * params->dt;
    cs.xi = 1.0 - 0.5 * params->dt;
    s->tune = default_tuning(*grid);

    // Equilibrium a^(0)_{n,m} = s_n g_m (Sec. 2): s_n carries sigma(n), the
    // Bessel ratio and the normalisation, g_m the phi_y envelope.
    std::vector<double> ratio = bessel_ratio_table(params->mu, grid->n_x);
    s->ratio1 = ratio[1];
    std::vector<double> sn(grid->n_x), gm(grid->n_y);
    const double norm = std::sqrt(params->mu / (2.0 * kPi * params->alpha)) / kPi;
    for (int n = 0; n < grid->n_x; ++n) sn[n] = (n == 0 ? 0.5 : 1.0) * ratio[n] * norm;
    double gsum = 0.0;
    for (int m = 0; m < grid->n_y; ++m) {
        const double phi = grid->phiy_min + m * dphi;
        gm[m] = std::exp(-0.5 * params->mu * phi * phi);
        gsum += gm[m];
    }
    s->norm_eq = sn[0] * gsum;

    auto bail = [&](bte_status code) {
        std::string msg = g_last_error;
        bte_destroy(s);
        g_last_error = msg;
        return code;
    };
    e = hipMemsetAsync(s->ws, 0, L.total, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->s_n(), sn.data(), sizeof(double) * sn.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->g_m(), gm.data(), sizeof(double) * gm.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(fail(BTE_EDEVICE, "workspace init: %s", hipGetErrorString(e)));

    st = write_ctl(s);
    if (st != BTE_OK) return bail(st);
    e = s->fp32() ? bte::launch_init_equilibrium<float>(cs, s->plane<float>(0, 0), s->plane<float>(0, 1), s->s_n(), s->g_m(), s->stream)
                  : bte::launch_init_equilibrium<double>(cs, s->plane<double>(0, 0), s->plane<double>(0, 1), s->s_n(), s->g_m(), s->stream);
    if (e != hipSuccess) return bail(fail(BTE_EDEVICE, "init launch: %s", hipGetErrorString(e)));
    st = s->fp32() ? queue_startup<float>(s) : queue_startup<double>(s);
    if (st != BTE_OK) return bail(st);
    st = measure_norm0(s);
    if (st != BTE_OK) return bail(st);
    *out = s;
    return BTE_OK;
}

bte_status bte_step(bte_solver* s, int64_t n_steps)
{
    if (!s) return fail(BTE_EINVAL, "solver is NULL");
    if (n_steps < 0) return fail(BTE_EINVAL, "n_steps must be >= 0");
    // the device sets the flag when a run of steps ends with a non-finite or
    // drifted norm or drift velocity; reading it costs no synchronisation
    if (__atomic_load_n(s->flag_host, __ATOMIC_ACQUIRE) != 0) s->unstable = true;
    if (s->unstable) return fail(BTE_EUNSTABLE, "solver is flagged unstable; reset the state");
    int64_t left = n_steps;
    const int G = s->tune.graph_steps;
    if (G > 0 && left >= G) {
        if (s->graph_steps_built != G) {
            drop_graphs(s);
            s->graph_steps_built = G;
        }
        while (left >= G) {
            if (!s->graph[s->cur]) {
                bte_status st = build_graph(s);
                if (st != BTE_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream));
            if (s->graph_flip[s->cur]) s->cur = 1 - s->cur;
            left -= G;
            s->step += G;
        }
    }
    while (left > 0) {
        const int n = static_cast<int>(std::min<int64_t>(left, 64));
        HIP_TRY(queue_steps_direct(s, n, s->stream));
        left -= n;
        s->step += n;
    }
    return BTE_OK;
}

bte_status bte_set_window(bte_solver* s, int64_t lo, int64_t hi)
{
    if (!s) return fail(BTE_EINVAL, "solver is NULL");
    if (hi < lo) return fail(BTE_EINVAL, "window needs lo <= hi");
    s->win_lo = lo;
    s->win_hi = hi;
    bte_status st = clear_acc(s);
    if (st != BTE_OK) return st;
    return write_ctl(s);
}

bte_status bte_observables(bte_solver* s, bte_obs* out)
{
    if (!s || !out) return fail(BTE_EINVAL, "solver and out must not be NULL");
    double r[bte::kObsOut];
    bte_status st = reduce(s, r);
    if (st != BTE_OK) return st;
    const double f = kPi * std::sqrt(s->params.alpha) * s->cs.dphi;
    std::memset(out, 0, sizeof(*out));
    out->step = s->step;
    out->t = static_cast<double>(s->step) * s->params.dt;
    out->norm = 2.0 * f * r[0];
    out->v_dr = f * r[1];
    out->n_avg = window_count(s);
    out->S_v = f * r[2];
    out->S_vc = f * r[3];
    out->edge_mass = 2.0 * f * r[4];
    out->top_harm_mass = r[5] > 0 ? r[6] / r[5] : 0.0;
    if (out->n_avg > 0) {
        const double K = static_cast<double>(out->n_avg);
        out->v_avg = out->S_v / K;
        out->absorption = (2.0 / s->ratio1) * out->S_vc / K;
        // cosine at the accumulated steps, at the kernels' times (2 (k) half_dt)
        const int64_t lo = std::max(s->win_lo, s->acc_from);
        double sc = 0.0;
        for (int64_t k = lo + 1; k <= lo + out->n_avg; ++k)
            sc += std::cos(s->params.omega * (static_cast<double>(2 * k) * s->cs.half_dt));
        out->S_c = sc;
        out->absorption_cov = (2.0 / s->ratio1) * (out->S_vc - out->v_avg * sc) / K;
    }
    // the normalisation relaxes from its initial value toward the equilibrium
    // one; it must not move further away than it started (plus 1e-2 of it)
    const double eq = 2.0 * f * s->norm_eq;
    const bool bad = !std::isfinite(out->norm) || !std::isfinite(out->v_dr) ||
                     !std::isfinite(out->S_v) || !std::isfinite(out->S_vc) ||
                     !std::isfinite(r[5]) ||
                     !(std::fabs(out->norm - eq) <= std::fabs(s->norm0 - eq) + 1e-2 * std::fabs(eq));
    if (bad || __atomic_load_n(s->flag_host, __ATOMIC_ACQUIRE) != 0) s->unstable = true;
    out->status = s->unstable ? BTE_EUNSTABLE : BTE_OK;
    return BTE_OK;
}

bte_status bte_run_periods(bte_solver* s, double tol, int32_t min_periods, int32_t max_periods,
                           int32_t confirm, bte_result* out)
{
    if (!s || !out) return fail(BTE_EINVAL, "solver and out must not be NULL");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(BTE_EINVAL, "tol must be finite and > 0");
    if (min_periods < 2 || max_periods < min_periods)
        return fail(BTE_EINVAL, "need 2 <= min_periods <= max_periods");
    if (confirm < 1) return fail(BTE_EINVAL, "confirm must be >= 1");
    if (!(s->params.omega > 0)) return fail(BTE_EINVAL, "omega must be > 0 to define a period");
    const double steps_per_period = 2.0 * kPi / (s->params.omega * s->params.dt);
    if (!(steps_per_period < 4e18)) return fail(BTE_EINVAL, "period too long in steps");
    const int64_t L = std::max<int64_t>(1, std::llround(steps_per_period));
    std::memset(out, 0, sizeof(*out));
    const int64_t k0 = s->step;
    double A_prev = 0.0;
    int run_ok = 0;
    for (int p = 1;; ++p) {
        const int64_t lo = k0 + static_cast<int64_t>(p - 1) * L, hi = lo + L;
        bte_status st = bte_set_window(s, lo, hi);
        if (st == BTE_OK) st = bte_step(s, L);
        bte_obs o;
        if (st == BTE_OK) st = bte_observables(s, &o);
        if (st == BTE_EUNSTABLE) {
            out->status = BTE_EUNSTABLE;
            return BTE_OK;
        }
        if (st != BTE_OK) return st;
        const double dA = p > 1 ? std::fabs(o.absorption_cov - A_prev) : 0.0;
        out->absorption = o.absorption_cov;
        out->v_avg = o.v_avg;
        out->dA = dA;
        out->steps = s->step - k0;
        out->periods = p;
        out->status = o.status;
        if (o.status != BTE_OK || !std::isfinite(o.absorption_cov)) {
            out->status = BTE_EUNSTABLE;
            return BTE_OK;
        }
        run_ok = (p > 1 && dA < tol) ? run_ok + 1 : 0;
        if (p >= min_periods && run_ok >= confirm) {
            out->converged = 1;
            return BTE_OK;
        }
        if (p >= max_periods) return BTE_OK;
        A_prev = o.absorption_cov;
    }
}

bte_status bte_get_state(bte_solver* s, double* a_h, double* b_h, double* a_f, double* b_f)
{
    if (!s) return fail(BTE_EINVAL, "solver is NULL");
    double* outs[4] = {a_h, b_h, a_f, b_f};
    for (int w = 0; w < 4; ++w) {
        if (!outs[w]) continue;
        bte_status st = s->fp32() ? copy_plane_out<float>(s, s->cur, w, outs[w])
                                  : copy_plane_out<double>(s, s->cur, w, outs[w]);
        if (st != BTE_OK) return st;
    }
    return BTE_OK;
}

bte_status bte_set_state(bte_solver* s, const double* a_h, const double* b_h, const double* a_f,
                         const double* b_f, int64_t step)
{
    if (!s || !a_h || !b_h) return fail(BTE_EINVAL, "solver, a_h and b_h must not be NULL");
    if ((a_f == nullptr) != (b_f == nullptr)) return fail(BTE_EINVAL, "give both a_f and b_f or neither");
    if (!a_f && step != 0) return fail(BTE_EINVAL, "a start-up from (a_h, b_h) is at step 0");
    if (step < 0) return fail(BTE_EINVAL, "step must be >= 0");
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double* ins[4] = {a_h, b_h, a_f, b_f};
    for (int w = 0; w < 4; ++w) {
        if (!ins[w]) continue;
        const bool zero0 = (w == 1 || w == 3);
        bte_status st = s->fp32() ? copy_plane_in<float>(s, s->cur, w, ins[w], zero0)
                                  : copy_plane_in<double>(s, s->cur, w, ins[w], zero0);
        if (st != BTE_OK) return st;
    }
    s->step = step;
    s->unstable = false;
    bte_status st = clear_acc(s);
    if (st != BTE_OK) return st;
    st = write_ctl(s);
    if (st != BTE_OK) return st;
    if (!a_f) {
        st = s->fp32() ? queue_startup<float>(s) : queue_startup<double>(s);
        if (st != BTE_OK) return st;
    }
    return measure_norm0(s);
}

bte_status bte_set_tuning(bte_solver* s, const bte_tuning* t)
{
    if (!s || !t) return fail(BTE_EINVAL, "solver and tuning must not be NULL");
    bte_tuning v = *t;
    bte_tuning d = default_tuning(s->grid);
    if (v.rows_per_wave == 0) v.rows_per_wave = d.rows_per_wave;
    if (v.waves_per_block == 0) v.waves_per_block = d.waves_per_block;
    bte_status st = check_tuning(v);
    if (st != BTE_OK) return st;
    if (v.kernel != s->tune.kernel || v.rows_per_wave != s->tune.rows_per_wave ||
        v.waves_per_block != s->tune.waves_per_block || v.graph_steps != s->tune.graph_steps)
        drop_graphs(s);
    s->tune = v;
    return BTE_OK;
}

bte_status bte_get_tuning(const bte_solver* s, bte_tuning* t)
{
    if (!s || !t) return fail(BTE_EINVAL, "solver and tuning must not be NULL");
    *t = s->tune;
    return BTE_OK;
}

bte_status bte_reconstruct(bte_solver* s, int32_t n_phix, double* out)
{
    if (!s || !out) return fail(BTE_EINVAL, "solver and out must not be NULL");
    if (reinterpret_cast<uintptr_t>(out) % alignof(double) != 0)
        return fail(BTE_EINVAL, "out must be 8-byte aligned");
    if (n_phix < 1 || n_phix > (1 << 20)) return fail(BTE_EINVAL, "n_phix must be in 1..2^20");
    const hipError_t e =
        s->fp32() ? bte::launch_reconstruct<float>(s->stream, s->plane<float>(s->cur, 0),
                                                   s->plane<float>(s->cur, 1), s->L.ld,
                                                   s->grid.n_x, s->grid.n_y, n_phix, out)
                  : bte::launch_reconstruct<double>(s->stream, s->plane<double>(s->cur, 0),
                                                    s->plane<double>(s->cur, 1), s->L.ld,
                                                    s->grid.n_x, s->grid.n_y, n_phix, out);
    if (e != hipSuccess) return fail(BTE_EDEVICE, "reconstruct launch: %s", hipGetErrorString(e));
    return BTE_OK;
}

bte_status bte_reconstruct_coeffs(const double* a, const double* b, int32_t n_x, int32_t n_y,
                                  int64_t ld, int32_t n_phix, double* out, void* hip_stream)
{
    if (!a || !b || !out) return fail(BTE_EINVAL, "a, b and out must not be NULL");
    const auto misaligned = [](const void* p) {
        return reinterpret_cast<uintptr_t>(p) % alignof(double) != 0;
    };
    if (misaligned(a) || misaligned(b) || misaligned(out))
        return fail(BTE_EINVAL, "a, b and out must be 8-byte aligned");
    if (n_x < 1 || n_y < 1 || ld < n_y) return fail(BTE_EINVAL, "need n_x >= 1, n_y >= 1, ld >= n_y");
    if (n_x > 16384 || n_y > (1 << 24)) return fail(BTE_EINVAL, "sizes too large");
    if (n_phix < 1 || n_phix > (1 << 20)) return fail(BTE_EINVAL, "n_phix must be in 1..2^20");
    const hipError_t e = bte::launch_reconstruct<double>(static_cast<hipStream_t>(hip_stream), a, b,
                                                         ld, n_x, n_y, n_phix, out);
    if (e != hipSuccess) return fail(BTE_EDEVICE, "reconstruct launch: %s", hipGetErrorString(e));
    return BTE_OK;
}

bte_status bte_state_observables_bytes(int32_t n_x, size_t* bytes)
{
    if (!bytes) return fail(BTE_EINVAL, "bytes must not be NULL");
    if (n_x < 2 || n_x > 16384) return fail(BTE_EINVAL, "n_x must be in 2..16384");
    *bytes = bte::state_obs_red_offset(n_x) + align_up(bte::kObsOut * sizeof(double));
    return BTE_OK;
}

bte_status bte_state_observables(const double* a, const double* b, int32_t n_x, int32_t n_y,
                                 int64_t ld, double phiy_min, double phiy_max, double alpha,
                                 void* workspace, size_t workspace_bytes, void* hip_stream,
                                 double* out)
{
    bte::StateObsArgs v;
    bte_status st = static_cast<bte_status>(
        bte::state_obs_validate(a, b, n_x, n_y, ld, phiy_min, phiy_max, alpha, out, v));
    if (st != BTE_OK) return st;
    size_t need = 0;
    st = bte_state_observables_bytes(n_x, &need);
    if (st != BTE_OK) return st;
    if (workspace && workspace_bytes < need)
        return fail(BTE_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    if (workspace && reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(BTE_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
    if (!ws) {
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipMalloc(reinterpret_cast<void**>(&ws), need));
    }
    double* part = reinterpret_cast<double*>(ws);
    double* red = reinterpret_cast<double*>(ws + bte::state_obs_red_offset(n_x));
    hipError_t e = bte::launch_state_observables(v.cs, a, b, v.edge_w, v.top_from, v.f, part, red,
                                                 out, stream);
    if (!workspace) {
        const hipError_t e2 = hipStreamSynchronize(stream);
        (void)hipFree(ws);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(BTE_EDEVICE, "state observables: %s", hipGetErrorString(e));
    return BTE_OK;
}

}  // extern "C"

// ---- bte_state_observables without allocation ---------------------------------
// The partial sums and reduction outputs live in one file-scope device array.
// In host code `scratch` names a host-side stand-in, not device memory: every
// use on the host goes through the address hipGetSymbolAddress returns for the
// current device, looked up once per device and kept in g_scratch_dev.
namespace {
constexpr int kNoAllocMaxNx = BTE_STATE_OBS_NOALLOC_MAX_NX;
constexpr size_t kNoAllocScratchBytes =
    (3 * sizeof(double) * (kNoAllocMaxNx + 1) + kAlign - 1) / kAlign * kAlign + kAlign;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
bte_status noalloc_scratch(void** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(BTE_EDEVICE, "device %d is beyond the %d this library serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BTE_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return BTE_OK;
}
}  // namespace

extern "C" {

bte_status bte_state_observables_noalloc(const double* a, const double* b, int32_t n_x,
                                         int32_t n_y, int64_t ld, double phiy_min,
                                         double phiy_max, double alpha, void* hip_stream,
                                         double* out)
{
    bte::StateObsArgs v;
    bte_status st = static_cast<bte_status>(
        bte::state_obs_validate(a, b, n_x, n_y, ld, phiy_min, phiy_max, alpha, out, v));
    if (st != BTE_OK) return st;
    if (n_x > kNoAllocMaxNx)
        return fail(BTE_EINVAL, "n_x = %d exceeds the no-allocation limit %d", n_x, kNoAllocMaxNx);
    size_t need = 0;
    st = bte_state_observables_bytes(n_x, &need);
    if (st != BTE_OK) return st;
    if (need > kNoAllocScratchBytes)
        return fail(BTE_EINVAL, "n_x = %d needs %zu scratch bytes, the static array holds %zu",
                    n_x, need, kNoAllocScratchBytes);
    void* ws = nullptr;
    st = noalloc_scratch(&ws);
    if (st != BTE_OK) return st;
    char* base = static_cast<char*>(ws);
    double* part = reinterpret_cast<double*>(base);
    double* red = reinterpret_cast<double*>(base + bte::state_obs_red_offset(n_x));
    const hipError_t e = bte::launch_state_observables(v.cs, a, b, v.edge_w, v.top_from, v.f,
                                                       part, red, out,
                                                       static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(BTE_EDEVICE, "state observables: %s", hipGetErrorString(e));
    return BTE_OK;
}

}  // extern "C"

namespace {
// Plain streaming copy: each workgroup copies one run of kCopyUnits 16-byte
// units, every thread four of them a workgroup-width apart (all four loads in
// flight before the stores), with non-temporal loads and stores since no byte
// is touched twice.  One pass over the buffer, no grid-stride loop: measured
// on 2 GiB this reaches 5.7 TB/s read+write, a grid-stride loop over 2048
// workgroups 4.4 TB/s.
typedef unsigned int copy_v4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;
constexpr int kCopyUnits = 4 * kCopyThreads;

__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const copy_v4* __restrict__ src,
                                                              copy_v4* __restrict__ dst, size_t n16)
{
    const size_t base = static_cast<size_t>(blockIdx.x) * kCopyUnits + threadIdx.x;
    if (base + 3 * kCopyThreads < n16) {
        const copy_v4 a = __builtin_nontemporal_load(src + base);
        const copy_v4 b = __builtin_nontemporal_load(src + base + kCopyThreads);
        const copy_v4 c = __builtin_nontemporal_load(src + base + 2 * kCopyThreads);
        const copy_v4 d = __builtin_nontemporal_load(src + base + 3 * kCopyThreads);
        __builtin_nontemporal_store(a, dst + base);
        __builtin_nontemporal_store(b, dst + base + kCopyThreads);
        __builtin_nontemporal_store(c, dst + base + 2 * kCopyThreads);
        __builtin_nontemporal_store(d, dst + base + 3 * kCopyThreads);
    } else {
        for (int k = 0; k < 4; ++k) {
            const size_t i = base + static_cast<size_t>(k) * kCopyThreads;
            if (i < n16) dst[i] = src[i];
        }
    }
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + kCopyUnits - 1) / kCopyUnits;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3(static_cast<unsigned>(blocks)), dim3(kCopyThreads), 0, st,
                       static_cast<const copy_v4*>(src), static_cast<copy_v4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace

extern "C" {

bte_status bte_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    if (!src || !dst) return fail(BTE_EINVAL, "src and dst must not be NULL");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(BTE_EINVAL, "bytes and both buffers must be multiples of 16");
    const char* a = static_cast<const char*>(src);
    const char* b = static_cast<const char*>(dst);
    if (a < b + bytes && b < a + bytes) return fail(BTE_EINVAL, "src and dst overlap");
    if (bytes == 0) return BTE_OK;
    HIP_TRY(launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)));
    return BTE_OK;
}

void bte_destroy(bte_solver* s)
{
    if (!s) return;
    if (s->stream || s->ws) (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->flag_host) (void)hipHostFree(s->flag_host);
    if (s->owns_ws && s->ws) (void)hipFree(s->ws);
    delete s;
}

const char* bte_last_error(void) { return g_last_error.c_str(); }

const char* bte_version(void) { return "bte-mi355x 0.1 (gfx950)"; }

}  // extern "C"
