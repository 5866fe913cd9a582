// gfx950 kernels of the superlattice BTE solver.
//
// The scheme (arXiv:1401.6047, Sec. 3): two staggered grids, "whole"
// z^k = (a_n, b_n)(phi_y) at integer steps and "fractional" z^{k+1/2}.  Each
// half-step applies the pointwise Crank-Nicolson operator T to a cell, with
// the transport coupling A^t, B^t (a 4-point cross in (n, m): n +- 1, m +- 1)
// read from the other grid.  Per cell and half-step that is ~25 flops and one
// FP64 reciprocal against 48 bytes of state traffic in FP64, so the kernels
// are bandwidth kernels: no MFMA, coalesced rows, registers for reuse.
//
// Work decomposition.  One wavefront owns a tile of 64 consecutive phi_y
// columns (lane = column, coalesced) and a chunk of `R` consecutive harmonics
// that it marches through in registers: harmonic n needs the other grid at
// n - 1 and n + 1, so each row is loaded once and kept for the next two
// iterations (register reuse along n).  Neighbours at m +- 1 come from the
// adjacent lanes through cross-lane shuffles, not from memory.
//
// The fused step computes the whole-grid update for one extra column and
// harmonic on each side of the tile (redundantly), which is what the
// fractional update of the tile's own cells needs from the new whole grid;
// so 60 of the 64 lanes produce output and the tile never waits for another.
// Reads and writes go to different (ping-pong) buffers.

#include "bte_internal.h"

namespace bte {
namespace {

__device__ __forceinline__ double shfl_from_left(double v) { return __shfl_up(v, 1); }
__device__ __forceinline__ double shfl_from_right(double v) { return __shfl_down(v, 1); }

template <typename T>
__device__ __forceinline__ double ld_state(const T* p) { return static_cast<double>(*p); }

template <typename T>
__device__ __forceinline__ void st_state(T* p, double v) { *p = static_cast<T>(v); }

// Operator T of Sec. 3 for one cell: Crank-Nicolson over a step h.
//   g = a xi - b mu0 + B^t + a0 h,   h' = b xi + a mu0 + A^t,
//   nu a' + mu1 b' = g,  nu b' - mu1 a' = h'  =>  Cramer's rule.
__device__ __forceinline__ void op_T(double a, double b, double At, double Bt, double a0h,
                                     double mu0, double mu1, double nu, double xi, double& an,
                                     double& bn)
{
    const double g = fma(a, xi, fma(-b, mu0, Bt + a0h));
    const double hh = fma(b, xi, fma(a, mu0, At));
    const double inv = 1.0 / fma(mu1, mu1, nu * nu);
    an = fma(g, nu, -hh * mu1) * inv;
    bn = fma(g, mu1, hh * nu) * inv;
}

// cos(omega t) for the four half-step times 2k .. 2k+3, one per lane 0..3,
// broadcast to the wave.
__device__ __forceinline__ void field_cosines(const Consts& cs, int64_t k, double c[4])
{
    const int lane = threadIdx.x & (kWave - 1);
    double t = static_cast<double>(2 * k + (lane & 3)) * cs.half_dt;
    double v = cos(cs.omega * t);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = __shfl(v, i);
}

// Blocks are dispatched round-robin over the 8 XCDs.  Map them so that each
// XCD works on a contiguous range of tiles: vertically adjacent tiles share
// halo rows and then hit the same L2.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x;
    const int per = nb >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

template <typename T>
struct FusedArgs {
    Planes<T> src;
    Planes<T> dst;
    const double* s_n;
    const double* g_m;
    double* acc_v;
    double* acc_vc;
    const Ctl* ctl;
    Consts cs;
    int j_off;
    int R;        // harmonics per wave
    int nchunks;  // ceil(nx / R)
    int ntiles;   // nchunks * ceil(ny / kFusedCols)
};

template <typename T>
__global__ __launch_bounds__(512) void k_fused_step(FusedArgs<T> A)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    const int tile = xcd_block() * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (tile >= A.ntiles) return;                    // wave-uniform
    const int ct = tile / A.nchunks;
    const int r0 = (tile - ct * A.nchunks) * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kFusedCols - 2 + lane;        // this lane's phi_y column
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 2) && (lane < kWave - 2) && col_ok;

    const Ctl ctl = *A.ctl;
    const int64_t k = ctl.k + A.j_off;
    double cw[4];
    field_cosines(cs, k, cw);
    const bool acc_step = (k + 1 > ctl.win_lo) && (k + 1 <= ctl.win_hi);

    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gm = col_ok ? A.g_m[m] : 0.0;
    const double hdt = 0.5 * cs.dt;
    // mu^t = n beta^t dt/2 with beta^t = E(t) + B phi: per-lane factor q, mu = n q.
    const double q0h = (fma(cs.E_w, cw[0], cs.E_dc) + cs.B * phi) * hdt;  // t = k dt
    const double q1h = (fma(cs.E_w, cw[2], cs.E_dc) + cs.B * phi) * hdt;  // t = (k+1) dt
    const double q0f = (fma(cs.E_w, cw[1], cs.E_dc) + cs.B * phi) * hdt;  // (k+1/2) dt
    const double q1f = (fma(cs.E_w, cw[3], cs.E_dc) + cs.B * phi) * hdt;  // (k+3/2) dt
    const double c = cs.c_full, nu = cs.nu, xi = cs.xi, dt = cs.dt;

    const int ld = cs.ld;
    const T* __restrict__ aHs = A.src.a_h + m;
    const T* __restrict__ bHs = A.src.b_h + m;
    const T* __restrict__ aFs = A.src.a_f + m;
    const T* __restrict__ bFs = A.src.b_f + m;
    T* __restrict__ aHd = A.dst.a_h + m;
    T* __restrict__ bHd = A.dst.b_h + m;
    T* __restrict__ aFd = A.dst.a_f + m;
    T* __restrict__ bFd = A.dst.b_f + m;

    // Old fractional grid, own column, rows j-1 (0), j (1), j+1 (2); and its
    // left/right neighbours for rows j-1 and j+1.
    double fa0 = ld_state(aFs + (r0 - 2) * ld), fb0 = ld_state(bFs + (r0 - 2) * ld);
    double fa1 = ld_state(aFs + (r0 - 1) * ld), fb1 = ld_state(bFs + (r0 - 1) * ld);
    double fal0 = shfl_from_left(fa0), far0 = shfl_from_right(fa0);
    double fbl0 = shfl_from_left(fb0), fbr0 = shfl_from_right(fb0);
    double fal1 = shfl_from_left(fa1), far1 = shfl_from_right(fa1);
    double fbl1 = shfl_from_left(fb1), fbr1 = shfl_from_right(fb1);
    // New whole grid, neighbours only, rows j-2 (0), j-1 (1).
    double hal0 = 0, har0 = 0, hbl0 = 0, hbr0 = 0;
    double hal1 = 0, har1 = 0, hbl1 = 0, hbr1 = 0;

    for (int j = r0 - 1; j <= r1; ++j) {
        const double fa2 = ld_state(aFs + (j + 1) * ld);
        const double fb2 = ld_state(bFs + (j + 1) * ld);
        const double fal2 = shfl_from_left(fa2), far2 = shfl_from_right(fa2);
        const double fbl2 = shfl_from_left(fb2), fbr2 = shfl_from_right(fb2);

        // ---- whole grid, harmonic j: z^{k+1} = T(z^k; A, B from z^{k+1/2})
        const double nd = static_cast<double>(j);
        const int nc = min(max(j, 0), cs.nx - 1);
        const double s = A.s_n[nc];
        const double chi = (j == 1) ? 2.0 : 1.0;
        double ha, hb;
        {
            const double a = ld_state(aHs + j * ld);
            const double b = ld_state(bHs + j * ld);
            const double At = c * (chi * (far0 - fal0) - far2 + fal2);
            const double Bt = c * ((fbr2 - fbl2) - fbr0 + fbl0);
            op_T(a, b, At, Bt, s * gm * dt, nd * q0h, nd * q1h, nu, xi, ha, hb);
        }
        const bool row_a = (j >= 0) && (j < cs.nx) && col_ok;
        const bool row_b = row_a && (j >= 1);
        ha = row_a ? ha : 0.0;
        hb = row_b ? hb : 0.0;
        if (out_lane && j >= r0 && j < r1) {
            st_state(aHd + j * ld, ha);
            st_state(bHd + j * ld, hb);
            if (j == 1 && acc_step) {                // drift-velocity window sums
                A.acc_v[m] += hb;
                A.acc_vc[m] += hb * cw[2];
            }
        }
        const double hal2 = shfl_from_left(ha), har2 = shfl_from_right(ha);
        const double hbl2 = shfl_from_left(hb), hbr2 = shfl_from_right(hb);

        // ---- fractional grid, harmonic j-1: z^{k+3/2} = T(z^{k+1/2}; A, B from z^{k+1})
        const int n = j - 1;
        if (n >= r0) {
            const double nd1 = static_cast<double>(n);
            const double s1 = A.s_n[min(max(n, 0), cs.nx - 1)];
            const double chi1 = (n == 1) ? 2.0 : 1.0;
            const double At = c * (chi1 * (har0 - hal0) - har2 + hal2);
            const double Bt = c * ((hbr2 - hbl2) - hbr0 + hbl0);
            double fa, fb;
            op_T(fa0, fb0, At, Bt, s1 * gm * dt, nd1 * q0f, nd1 * q1f, nu, xi, fa, fb);
            if (out_lane) {
                st_state(aFd + n * ld, fa);
                st_state(bFd + n * ld, n >= 1 ? fb : 0.0);
            }
        }
        // rotate the register window
        fa0 = fa1; fb0 = fb1; fa1 = fa2; fb1 = fb2;
        fal0 = fal1; far0 = far1; fbl0 = fbl1; fbr0 = fbr1;
        fal1 = fal2; far1 = far2; fbl1 = fbl2; fbr1 = fbr2;
        hal0 = hal1; har0 = har1; hbl0 = hbl1; hbr0 = hbr1;
        hal1 = hal2; har1 = har2; hbl1 = hbl2; hbr1 = hbr2;
    }
}

template <typename T>
struct HalfArgs {
    T* xa;
    T* xb;
    const T* ya;
    const T* yb;
    const double* s_n;
    const double* g_m;
    double* acc_v;
    double* acc_vc;
    const Ctl* ctl;
    Consts cs;
    double h;
    int off0, off1;
    int accumulate;
    int j_off;
    int R;
    int nchunks;
    int ntiles;
};

// One half-step of the paper's two-kernel structure, in place on X (a cell of
// X reads only its own old value; all neighbour reads hit Y).
template <typename T>
__global__ __launch_bounds__(512) void k_half_step(HalfArgs<T> A)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    const int tile = xcd_block() * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (tile >= A.ntiles) return;
    const int ct = tile / A.nchunks;
    const int r0 = (tile - ct * A.nchunks) * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kHalfCols - 1 + lane;
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 1) && (lane < kWave - 1) && col_ok;

    const Ctl ctl = *A.ctl;
    const int64_t k = ctl.k + A.j_off;
    const int lane_off = (lane & 1) ? A.off1 : A.off0;
    const double tt = static_cast<double>(2 * k + lane_off) * cs.half_dt;
    const double cv = cos(cs.omega * tt);
    const double c0 = __shfl(cv, 0), c1 = __shfl(cv, 1);
    const bool acc_step = A.accumulate && (k + 1 > ctl.win_lo) && (k + 1 <= ctl.win_hi);
    const double cw_acc = cos(cs.omega * static_cast<double>(2 * k + 2) * cs.half_dt);

    const double h = A.h;
    const double nu = 1.0 + 0.5 * h, xi = 1.0 - 0.5 * h;
    const double c = cs.B * h / (4.0 * cs.dphi);
    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gm = col_ok ? A.g_m[m] : 0.0;
    const double q0 = (fma(cs.E_w, c0, cs.E_dc) + cs.B * phi) * (0.5 * h);
    const double q1 = (fma(cs.E_w, c1, cs.E_dc) + cs.B * phi) * (0.5 * h);

    const int ld = cs.ld;
    T* __restrict__ xa = A.xa + m;
    T* __restrict__ xb = A.xb + m;
    const T* __restrict__ ya = A.ya + m;
    const T* __restrict__ yb = A.yb + m;

    double ya0 = ld_state(ya + (r0 - 1) * ld), yb0 = ld_state(yb + (r0 - 1) * ld);
    double yal0 = shfl_from_left(ya0), yar0 = shfl_from_right(ya0);
    double ybl0 = shfl_from_left(yb0), ybr0 = shfl_from_right(yb0);
    double ya1 = ld_state(ya + r0 * ld), yb1 = ld_state(yb + r0 * ld);
    double yal1 = shfl_from_left(ya1), yar1 = shfl_from_right(ya1);
    double ybl1 = shfl_from_left(yb1), ybr1 = shfl_from_right(yb1);

    for (int n = r0; n < r1; ++n) {
        const double ya2 = ld_state(ya + (n + 1) * ld), yb2 = ld_state(yb + (n + 1) * ld);
        const double yal2 = shfl_from_left(ya2), yar2 = shfl_from_right(ya2);
        const double ybl2 = shfl_from_left(yb2), ybr2 = shfl_from_right(yb2);
        const double chi = (n == 1) ? 2.0 : 1.0;
        const double At = c * (chi * (yar0 - yal0) - yar2 + yal2);
        const double Bt = c * ((ybr2 - ybl2) - ybr0 + ybl0);
        const double nd = static_cast<double>(n);
        double an, bn;
        const double a = ld_state(xa + n * ld);
        const double b = ld_state(xb + n * ld);
        op_T(a, b, At, Bt, A.s_n[n] * gm * h, nd * q0, nd * q1, nu, xi, an, bn);
        if (out_lane) {
            st_state(xa + n * ld, an);
            st_state(xb + n * ld, n >= 1 ? bn : 0.0);
            if (n == 1 && acc_step) {
                A.acc_v[m] += bn;
                A.acc_vc[m] += bn * cw_acc;
            }
        }
        yal0 = yal1; yar0 = yar1; ybl0 = ybl1; ybr0 = ybr1;
        yal1 = yal2; yar1 = yar2; ybl1 = ybl2; ybr1 = ybr2;
    }
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

constexpr int kReduceThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_obs(Consts cs, const T* a_h,
                                                               const T* b_h,
                                                               const double* acc_v,
                                                               const double* acc_vc, double* out)
{
    __shared__ double sh[4][kReduceThreads];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int m = threadIdx.x; m < cs.ny; m += kReduceThreads) {
        s0 += static_cast<double>(a_h[m]);
        s1 += static_cast<double>(b_h[cs.ld + m]);
        s2 += acc_v[m];
        s3 += acc_vc[m];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    sh[3][threadIdx.x] = s3;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

inline int round_up8(int x) { return (x + 7) & ~7; }

}  // namespace

template <typename T>
hipError_t launch_fused_step(const Consts& cs, const Shape& sh, Planes<T> src, Planes<T> dst,
                             const double* s_n, const double* g_m, double* acc_v,
                             double* acc_vc, const Ctl* ctl, int j_off, hipStream_t st)
{
    FusedArgs<T> A;
    A.src = src;
    A.dst = dst;
    A.s_n = s_n;
    A.g_m = g_m;
    A.acc_v = acc_v;
    A.acc_vc = acc_vc;
    A.ctl = ctl;
    A.cs = cs;
    A.j_off = j_off;
    A.R = sh.rows_per_wave;
    A.nchunks = (cs.nx + A.R - 1) / A.R;
    A.ntiles = A.nchunks * ((cs.ny + kFusedCols - 1) / kFusedCols);
    const int wpb = sh.waves_per_block;
    const int blocks = round_up8((A.ntiles + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_fused_step<T>, dim3(blocks), dim3(wpb * kWave), 0, st, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_half_step(const Consts& cs, const Shape& sh, T* xa, T* xb, const T* ya,
                            const T* yb, const double* s_n, const double* g_m, double h,
                            int off0, int off1, int accumulate, double* acc_v, double* acc_vc,
                            const Ctl* ctl, int j_off, hipStream_t st)
{
    HalfArgs<T> A;
    A.xa = xa;
    A.xb = xb;
    A.ya = ya;
    A.yb = yb;
    A.s_n = s_n;
    A.g_m = g_m;
    A.acc_v = acc_v;
    A.acc_vc = acc_vc;
    A.ctl = ctl;
    A.cs = cs;
    A.h = h;
    A.off0 = off0;
    A.off1 = off1;
    A.accumulate = accumulate;
    A.j_off = j_off;
    A.R = sh.rows_per_wave;
    A.nchunks = (cs.nx + A.R - 1) / A.R;
    A.ntiles = A.nchunks * ((cs.ny + kHalfCols - 1) / kHalfCols);
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
                             const double* acc_vc, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_obs<T>, dim3(1), dim3(kReduceThreads), 0, st, cs, a_h, b_h, acc_v,
                       acc_vc, out);
    return hipGetLastError();
}

#define BTE_INSTANTIATE(T)                                                                     \
    template hipError_t launch_fused_step<T>(const Consts&, const Shape&, Planes<T>, Planes<T>, \
                                             const double*, const double*, double*, double*,   \
                                             const Ctl*, int, hipStream_t);                    \
    template hipError_t launch_half_step<T>(const Consts&, const Shape&, T*, T*, const T*,      \
                                            const T*, const double*, const double*, double,    \
                                            int, int, int, double*, double*, const Ctl*, int,  \
                                            hipStream_t);                                      \
    template hipError_t launch_init_equilibrium<T>(const Consts&, T*, T*, const double*,        \
                                                   const double*, hipStream_t);                \
    template hipError_t launch_reduce_obs<T>(const Consts&, const T*, const T*, const double*,  \
                                             const double*, double*, hipStream_t);

BTE_INSTANTIATE(double)
BTE_INSTANTIATE(float)

}  // namespace bte
