// Single-instance step kernels: one tile per wavefront, the step index and
// averaging window read from the device control block.

#include <map>
#include <mutex>
#include <tuple>

#include "bte_device.h"

namespace bte {
namespace {

using namespace detail;

__device__ __forceinline__ bool in_window(const Ctl& c, int64_t step)
{
    return step > c.win_lo && step <= c.win_hi;
}

template <typename T>
struct StepArgs {
    TileEnv<T> env;           // k and the window flags are filled per launch
    const Ctl* ctl;
    int j_off;                // this launch advances step ctl->k + j_off
    int ntiles;
};

template <typename T>
__global__ __launch_bounds__(512) void k_fused_step(StepArgs<T> A)
{
    const int tile = wave_tile();
    if (tile >= A.ntiles) return;                    // wave-uniform
    const Ctl ctl = *A.ctl;
    TileEnv<T> E = A.env;
    E.k = ctl.k + A.j_off;
    E.acc1 = in_window(ctl, E.k + 1);
    E.acc2 = false;
    fused_tile<T>(E, tile);
}

// Three wavefronts per SIMD: the loop's registers fit in 168 VGPRs (the
// allocation granule rounds 169 up to 176, which would leave room for two).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_fused_step2(StepArgs<T> A)
{
    __shared__ double s_tab[4][kWave];
    const int tile = wave_tile();
    if (tile >= A.ntiles) return;                    // wave-uniform
    const Ctl ctl = *A.ctl;
    TileEnv<T> E = A.env;
    E.k = ctl.k + A.j_off;
    E.acc1 = in_window(ctl, E.k + 1);
    E.acc2 = in_window(ctl, E.k + 2);
    fused2_tile<T>(E, tile, &s_tab[threadIdx.x / kWave][0]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fused_step3(StepArgs<T> A)
{
    __shared__ double s_tab[4][kWave];
    const int tile = wave_tile();
    if (tile >= A.ntiles) return;                    // wave-uniform
    const Ctl ctl = *A.ctl;
    TileEnv<T> E = A.env;
    E.k = ctl.k + A.j_off;
    E.acc1 = in_window(ctl, E.k + 1);
    E.acc2 = in_window(ctl, E.k + 2);
    E.acc3 = in_window(ctl, E.k + 3);
    fused3_tile<T>(E, tile, &s_tab[threadIdx.x / kWave][0]);
}

template <typename T>
struct HalfArgs {
    HalfEnv<T> env;
    int accumulate;
    const Ctl* ctl;
    int j_off;
    int ntiles;
};

// One half-step of the paper's two-kernel structure, in place on X (a cell of
// X reads only its own old value; all neighbour reads hit Y).
template <typename T>
__global__ __launch_bounds__(512) void k_half_step(HalfArgs<T> A)
{
    const int tile = wave_tile();
    if (tile >= A.ntiles) return;
    const Ctl ctl = *A.ctl;
    HalfEnv<T> E = A.env;
    E.k = ctl.k + A.j_off;
    E.acc1 = A.accumulate && in_window(ctl, E.k + 1);
    half_tile<T>(E, tile);
}

template <typename T>
__global__ void k_init_equilibrium(Consts cs, T* a, T* b, const double* s_n, const double* g_m)
{
    // a, b point at logical (0,0); cover the whole padded plane.
    const int rows = cs.nx + 2 * kPadRows;
    const int64_t total = static_cast<int64_t>(rows) * cs.ld;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int row = static_cast<int>(i / cs.ld);
    const int col = static_cast<int>(i - static_cast<int64_t>(row) * cs.ld);
    const int n = row - kPadRows;
    const int m = col - kPadCols;
    T* a_base = a - (kPadRows * cs.ld + kPadCols);
    T* b_base = b - (kPadRows * cs.ld + kPadCols);
    double v = 0.0;
    if (n >= 0 && n < cs.nx && m >= 0 && m < cs.ny) v = s_n[n] * g_m[m];
    a_base[i] = static_cast<T>(v);
    b_base[i] = static_cast<T>(0.0);
}

__global__ void k_advance_counter(Ctl* ctl, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->k += n;
}

// ---- reductions ----------------------------------------------------------------
constexpr int kRedThreads = 256;

// Sum of v over the workgroup in a fixed order: a butterfly of wavefront
// shuffles (every lane ends with the same bits: each level adds the same two
// partial sums, only in swapped order), then the wavefront sums in order
// through LDS.  Every thread returns the total.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < static_cast<int>(blockDim.x / kWave); ++i) s += lds[i];
    __syncthreads();
    return s;
}

// Partial sums of one harmonic row (block n < nx) or of the window
// accumulators (block nx): part[3 n .. 3 n + 2] = (energy, x, y) with
//   row 0: (sum 2 a_0^2, sum a_0, sum over the edge strips of |a_0|)
//   row 1: (sum a_1^2 + b_1^2, sum b_1, 0), other rows (sum a_n^2 + b_n^2, 0, 0)
//   block nx: (0, sum acc_v, sum acc_vc).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_obs_rows(Consts cs, const T* a_h, const T* b_h,
                                                          const double* acc_v,
                                                          const double* acc_vc, int edge_w,
                                                          double* part)
{
    __shared__ double lds[kRedThreads / kWave];
    const int n = blockIdx.x;
    double e = 0.0, x = 0.0, y = 0.0;
    if (n < cs.nx) {
        const T* ar = a_h + static_cast<ptrdiff_t>(n) * cs.ld;
        const T* br = b_h + static_cast<ptrdiff_t>(n) * cs.ld;
        for (int m = threadIdx.x; m < cs.ny; m += kRedThreads) {
            const double a = static_cast<double>(ar[m]);
            if (n == 0) {
                e += 2.0 * (a * a);
                x += a;
                if (m < edge_w || m >= cs.ny - edge_w) y += fabs(a);
            } else {
                const double b = static_cast<double>(br[m]);
                e += a * a + b * b;
                if (n == 1) x += b;
            }
        }
    } else if (acc_v) {
        for (int m = threadIdx.x; m < cs.ny; m += kRedThreads) {
            x += acc_v[m];
            y += acc_vc[m];
        }
    }
    e = block_sum(e, lds);
    x = block_sum(x, lds);
    y = block_sum(y, lds);
    if (threadIdx.x == 0) {
        part[3 * n] = e;
        part[3 * n + 1] = x;
        part[3 * n + 2] = y;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_obs_final(int nx, int top_from,
                                                           const double* part, double* out)
{
    __shared__ double lds[kRedThreads / kWave];
    double tot = 0.0, top = 0.0;
    for (int n = threadIdx.x; n < nx; n += kRedThreads) {
        const double e = part[3 * n];
        tot += e;
        if (n >= top_from) top += e;
    }
    tot = block_sum(tot, lds);
    top = block_sum(top, lds);
    if (threadIdx.x == 0) {
        out[0] = part[1];
        out[1] = part[3 + 1];
        out[2] = part[3 * nx + 1];
        out[3] = part[3 * nx + 2];
        out[4] = part[2];
        out[5] = tot;
        out[6] = top;
    }
}

// Observables of a state from the reduction: out[0] = norm, out[1] = v_dr,
// out[2] = edge_mass, out[3] = top_harm_mass; f = pi sqrt(alpha) dphi.
__global__ void k_obs_finish(double f, const double* red, double* out)
{
    if (threadIdx.x == 0) {
        out[0] = 2.0 * f * red[0];
        out[1] = f * red[1];
        out[2] = 2.0 * f * red[4];
        out[3] = red[5] > 0.0 ? red[6] / red[5] : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_check_stable(Consts cs, const T* a_h,
                                                              const T* b_h, const Ctl* ctl,
                                                              int* flag)
{
    __shared__ double lds[kRedThreads / kWave];
    double sa = 0.0, sb = 0.0;
    for (int m = threadIdx.x; m < cs.ny; m += kRedThreads) {
        sa += static_cast<double>(a_h[m]);
        sb += static_cast<double>(b_h[cs.ld + m]);
    }
    sa = block_sum(sa, lds);
    sb = block_sum(sb, lds);
    if (threadIdx.x == 0) {
        const double eq = ctl->norm_eq;
        const double allowed = fabs(ctl->norm_ref - eq) + 1e-2 * fabs(eq);
        const bool bad = !isfinite(sa) || !isfinite(sb) || !(fabs(sa - eq) <= allowed);
        if (bad) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

inline int round_up8(int x) { return (x + 7) & ~7; }

// The step tiles address a state set through one buffer descriptor: its four
// planes must lie at one positive stride in the order a_h, b_h, a_f, b_f, and
// the set must stay below 2 GiB (32-bit byte offsets).
template <typename T>
bool uniform_set(const Planes<T>& P)
{
    const char* a = reinterpret_cast<const char*>(P.a_h);
    const std::ptrdiff_t st = reinterpret_cast<const char*>(P.b_h) - a;
    return st > 0 && reinterpret_cast<const char*>(P.a_f) - a == 2 * st &&
           reinterpret_cast<const char*>(P.b_f) - a == 3 * st && 4 * st < (std::ptrdiff_t{1} << 31);
}

// Whether the issue priority by progress (march_priority) pays for a launch of
// `blocks` workgroups of `threads` threads of kernel `fn`: every workgroup is
// resident at once (one round of wavefronts) and they fill at least a quarter
// of the device's slots (the device's CU count times the kernel's occupancy in
// workgroups per CU, looked up once per device, kernel and block size).
// Measured: launches filling 47 % to 96 % of the slots gained 3 % to 18 %, one
// filling 15 % (a 128 x 1001 grid) lost 3 %.
bool even_progress_pays(const void* fn, int threads, int blocks)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int>, long long> cap;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    const auto key = std::make_tuple(dev, fn, threads);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cap.find(key);
    if (it == cap.end()) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess)
            return false;
        it = cap.emplace(key, static_cast<long long>(per_cu) * cus).first;
    }
    return blocks <= it->second && 4LL * blocks >= it->second;
}

// logical (0,0) pointer -> physical plane base (row -kPadRows, column -kPadCols)
template <typename T>
T* phys(T* p, const Consts& cs)
{
    return p - (static_cast<ptrdiff_t>(kPadRows) * cs.ld + kPadCols);
}

template <typename T>
Planes<T> phys(Planes<T> p, const Consts& cs)
{
    return Planes<T>{phys(p.a_h, cs), phys(p.b_h, cs), phys(p.a_f, cs), phys(p.b_f, cs)};
}

}  // namespace

template <typename T>
static TileEnv<T> make_env(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                           const double* s_n, const double* g_m, double* acc_v, double* acc_vc,
                           int max_rows)
{
    TileEnv<T> E{};
    E.src = phys(src, cs);
    E.dst = phys(dst, cs);
    E.s_n = s_n;
    E.g_m = g_m;
    E.acc_v = acc_v;
    E.acc_vc = acc_vc;
    E.cs = cs;
    E.salt = 0;
    E.R = std::min(sh.rows_per_wave, max_rows);
    E.nchunks = (cs.nx + E.R - 1) / E.R;
    return E;
}

template <typename T>
hipError_t launch_fused_step(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                             const double* s_n, const double* g_m, double* acc_v,
                             double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st)
{
    if (!uniform_set(src) || !uniform_set(dst)) return hipErrorInvalidValue;
    StepArgs<T> A;
    A.env = make_env(cs, sh, src, dst, s_n, g_m, acc_v, acc_vc, kWave - 2);
    A.ctl = ctl;
    A.j_off = j_off;
    A.ntiles = A.env.nchunks * ((cs.ny + kFusedCols - 1) / kFusedCols);
    const int wpb = sh.waves_per_block;
    const int blocks = round_up8((A.ntiles + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_fused_step<T>, dim3(blocks), dim3(wpb * kWave), 0, st, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_step3(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                              const double* s_n, const double* g_m, double* acc_v,
                              double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st)
{
    if (!uniform_set(src) || !uniform_set(dst)) return hipErrorInvalidValue;
    StepArgs<T> A;
    // the wave's source coefficients cover its R harmonics plus 5 + 5 halo
    // harmonics, one per lane
    A.env = make_env(cs, sh, src, dst, s_n, g_m, acc_v, acc_vc, kWave - 10);
    A.ctl = ctl;
    A.j_off = j_off;
    const int wpb = std::min(sh.waves_per_block, 4);
    A.env.cgroup = wpb;
    A.ntiles = fused3_tile_count(cs.ny, A.env.nchunks, wpb);
    const int blocks = round_up8((A.ntiles + wpb - 1) / wpb);
    A.env.even_progress = even_progress_pays(reinterpret_cast<const void*>(&k_fused_step3<T>), wpb * kWave, blocks);
    hipLaunchKernelGGL(k_fused_step3<T>, dim3(blocks), dim3(wpb * kWave), 0, st, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_step2(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                              const double* s_n, const double* g_m, double* acc_v,
                              double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st)
{
    if (!uniform_set(src) || !uniform_set(dst)) return hipErrorInvalidValue;
    StepArgs<T> A;
    // the wave's source coefficients cover its R harmonics plus 3 + 3 halo
    // harmonics, one per lane
    A.env = make_env(cs, sh, src, dst, s_n, g_m, acc_v, acc_vc, kWave - 6);
    A.ctl = ctl;
    A.j_off = j_off;
    const int wpb = std::min(sh.waves_per_block, 4);
    A.env.cgroup = wpb;
    A.ntiles = fused2_tile_count(cs.ny, A.env.nchunks, wpb);
    const int blocks = round_up8((A.ntiles + wpb - 1) / wpb);
    A.env.even_progress = even_progress_pays(reinterpret_cast<const void*>(&k_fused_step2<T>), wpb * kWave, blocks);
    hipLaunchKernelGGL(k_fused_step2<T>, dim3(blocks), dim3(wpb * kWave), 0, st, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_half_step(const Consts& cs, const Shape& sh, T* xa, T* xb, const T* ya,
                            const T* yb, const double* s_n, const double* g_m, double h,
                            int off0, int off1, int accumulate, double* acc_v, double* acc_vc,
                            const Ctl* ctl, int j_off, hipStream_t st)
{
    HalfArgs<T> A;
    HalfEnv<T>& E = A.env;
    E = HalfEnv<T>{};
    E.xa = phys(xa, cs);
    E.xb = phys(xb, cs);
    E.ya = phys(ya, cs);
    E.yb = phys(yb, cs);
    E.s_n = s_n;
    E.g_m = g_m;
    E.acc_v = acc_v;
    E.acc_vc = acc_vc;
    E.cs = cs;
    E.h = h;
    E.off0 = off0;
    E.off1 = off1;
    E.salt = 0;
    E.R = std::min(sh.rows_per_wave, kWave);
    E.nchunks = (cs.nx + E.R - 1) / E.R;
    A.accumulate = accumulate;
    A.ctl = ctl;
    A.j_off = j_off;
    A.ntiles = E.nchunks * ((cs.ny + kHalfCols - 1) / kHalfCols);
    const int wpb = sh.waves_per_block;
    const int blocks = round_up8((A.ntiles + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_half_step<T>, dim3(blocks), dim3(wpb * kWave), 0, st, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_equilibrium(const Consts& cs, T* a, T* b, const double* s_n,
                                   const double* g_m, hipStream_t st)
{
    const int64_t total = static_cast<int64_t>(cs.nx + 2 * kPadRows) * cs.ld;
    const int threads = 256;
    const int blocks = static_cast<int>((total + threads - 1) / threads);
    hipLaunchKernelGGL(k_init_equilibrium<T>, dim3(blocks), dim3(threads), 0, st, cs, a, b, s_n,
                       g_m);
    return hipGetLastError();
}

hipError_t launch_advance_counter(Ctl* ctl, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(64), 0, st, ctl, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_obs(const Consts& cs, const T* a_h, const T* b_h, const double* acc_v,
                             const double* acc_vc, int edge_w, int top_from, double* part,
                             double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_obs_rows<T>, dim3(cs.nx + 1), dim3(kRedThreads), 0, st, cs, a_h, b_h,
                       acc_v, acc_vc, edge_w, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kRedThreads), 0, st, cs.nx, top_from, part, out);
    return hipGetLastError();
}

hipError_t launch_state_observables(const Consts& cs, const double* a, const double* b,
                                   int edge_w, int top_from, double f, double* part,
                                   double* red, double* out, hipStream_t st)
{
    hipError_t e = launch_reduce_obs<double>(cs, a, b, nullptr, nullptr, edge_w, top_from, part,
                                             red, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_finish, dim3(1), dim3(kWave), 0, st, f, red, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_stable(const Consts& cs, const T* a_h, const T* b_h, const Ctl* ctl,
                               int* flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_stable<T>, dim3(1), dim3(kRedThreads), 0, st, cs, a_h, b_h, ctl,
                       flag);
    return hipGetLastError();
}

#define BTE_INSTANTIATE(T)                                                                     \
    template hipError_t launch_fused_step<T>(const Consts&, const Shape&, Planes<T>, Planes<T>, \
                                             const double*, const double*, double*, double*,   \
                                             const Ctl*, int, hipStream_t);                    \
    template hipError_t launch_fused_step2<T>(const Consts&, const Shape&, Planes<T>, Planes<T>, \
                                              const double*, const double*, double*, double*,  \
                                              const Ctl*, int, hipStream_t);                   \
    template hipError_t launch_fused_step3<T>(const Consts&, const Shape&, Planes<T>, Planes<T>, \
                                              const double*, const double*, double*, double*,  \
                                              const Ctl*, int, hipStream_t);                   \
    template hipError_t launch_half_step<T>(const Consts&, const Shape&, T*, T*, const T*,      \
                                            const T*, const double*, const double*, double,    \
                                            int, int, int, double*, double*, const Ctl*, int,  \
                                            hipStream_t);                                      \
    template hipError_t launch_init_equilibrium<T>(const Consts&, T*, T*, const double*,        \
                                                   const double*, hipStream_t);                \
    template hipError_t launch_reduce_obs<T>(const Consts&, const T*, const T*, const double*,  \
                                             const double*, int, int, double*, double*,        \
                                             hipStream_t);                                     \
    template hipError_t launch_check_stable<T>(const Consts&, const T*, const T*, const Ctl*,   \
                                               int*, hipStream_t);

BTE_INSTANTIATE(double)
BTE_INSTANTIATE(float)

}  // namespace bte
