// Batched parameter sweep: many independent instances of the superlattice
// BTE run to per-period convergence, in one of two schedules (the wide one
// is described above its kernels further down).
//
// Persistent schedule: one graph-captured launch; each workgroup owns a state slot (two ping-pong sets of the four planes,
// sized for the largest N_y of the batch, plus the phi_y envelope and the
// per-phi_y window sums) and loops: take the next instance from a device work
// queue, initialise it (equilibrium or warm start, then the start-up
// half-step), run whole ac periods with the one- or two-step tile kernels and
// a workgroup barrier between passes, reduce the period's drift velocity and
// absorption, and stop on convergence of the period-to-period absorption.
// The tiles of one pass are spread over the workgroup's wavefronts; the
// per-cell arithmetic is the single-instance solver's (same device code).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bte.h"
#include "bte_device.h"

namespace bte {
namespace {

using namespace detail;

constexpr int kMaxWavesPerGroup = 8;
constexpr int kWarmRows = 64;       // warm-start coefficient rows (32 a + 32 b)
constexpr int kWarmCols = 128;      // warm-start phi_y samples
constexpr int kWarmHarmonics = 32;

// Per-instance constants, prepared on the host.
struct BatchInst {
    double E_dc, E_w, omega, B, mu;
    double dphi;          // phi_y spacing of this instance
    int64_t period_steps; // L = round(T / dt): steps per period window
    double two_over_ratio1;   // 2 I_0(mu) / I_1(mu)
    double v_norm;        // pi sqrt(alpha) dphi: v_dr = v_norm sum_m b_1(m)
    int32_t ny;
    int32_t pad;
};

template <typename T>
struct BatchArgs {
    const BatchInst* inst;
    const double* s_all;      // [n][nx] source coefficients
    const int32_t* order;     // work order (instance indices)
    const float* warm;        // [n][64][128] or null
    float* state_out;         // [n][64][128] or null: encoded final state
    bte_result* results;
    int32_t* queue;           // next-instance counter
    char* slots;              // per-workgroup state slots
    size_t slot_bytes;
    size_t plane_bytes;       // bytes of one padded plane (256-aligned)
    size_t off_g, off_accv, off_accvc;   // offsets inside a slot
    Consts base;              // nx, ld, dt, phimin, nu, xi (per-instance fields filled in-kernel)
    int n;
    int R;                    // harmonics per wave
    int form;                 // BTE_KERNEL_FUSED or BTE_KERNEL_FUSED2
    double tol;
    int min_periods, max_periods, confirm;
};

__global__ void k_batch_reset(int32_t* queue)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) queue[0] = 0;
}

// Values every lane agrees on, made provably uniform (scalar registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ double uni(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of one wavefront (fixed butterfly order).
__device__ __forceinline__ void wave_sum3(double& x, double& y, double& z)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        x += __shfl_xor(x, o);
        y += __shfl_xor(y, o);
        z += __shfl_xor(z, o);
    }
}

// A state slot: two ping-pong sets of the four planes, the phi_y envelope and
// the per-phi_y window sums.
template <typename T>
struct SlotView {
    char* base;
    size_t plane_bytes;
    double* g_m;
    double* acc_v;
    double* acc_vc;
    __device__ T* plane(int set, int which) const
    {
        return reinterpret_cast<T*>(base + (set * 4 + which) * plane_bytes);   // physical base
    }
    __device__ Planes<T> planes(int set) const
    {
        return Planes<T>{plane(set, 0), plane(set, 1), plane(set, 2), plane(set, 3)};
    }
};

template <typename T>
__device__ SlotView<T> slot_view(const BatchArgs<T>& B, int s)
{
    char* slot = B.slots + static_cast<size_t>(s) * B.slot_bytes;
    return SlotView<T>{slot, B.plane_bytes, reinterpret_cast<double*>(slot + B.off_g),
                       reinterpret_cast<double*>(slot + B.off_accv),
                       reinterpret_cast<double*>(slot + B.off_accvc)};
}

// Instance constants, made provably uniform, and the solver constants.
template <typename T>
__device__ void load_instance(const BatchArgs<T>& B, int idx, BatchInst& I, Consts& cs)
{
    I = B.inst[idx];
    I.E_dc = uni(I.E_dc);
    I.E_w = uni(I.E_w);
    I.omega = uni(I.omega);
    I.B = uni(I.B);
    I.mu = uni(I.mu);
    I.dphi = uni(I.dphi);
    I.period_steps = uni(I.period_steps);
    I.two_over_ratio1 = uni(I.two_over_ratio1);
    I.v_norm = uni(I.v_norm);
    I.ny = uni(I.ny);
    cs = B.base;
    cs.ny = I.ny;
    cs.dphi = I.dphi;
    cs.B = I.B;
    cs.E_dc = I.E_dc;
    cs.E_w = I.E_w;
    cs.omega = I.omega;
    cs.c_full = I.B * cs.dt / (4.0 * I.dphi);
}

__device__ __forceinline__ uint32_t instance_salt(int idx) { return 16u * static_cast<uint32_t>(idx + 1); }

// Initial state of instance idx in slot S (every cell of all eight planes,
// which clears what a previous instance left; whole and fractional grid of
// set 0 = z^0), then the start-up half-step z^{1/2} = T_{dt/2}(z^0).  Called
// by a whole workgroup.
template <typename T>
__device__ void init_slot(const BatchArgs<T>& B, const SlotView<T>& S, int idx, const BatchInst& I,
                          const Consts& cs, int wave, int nwaves)
{
    const int nx = B.base.nx, ld = B.base.ld;
    const int rows = nx + 2 * kPadRows;
    const double* s_n = B.s_all + static_cast<size_t>(idx) * nx;
    const float* warm = B.warm ? B.warm + static_cast<size_t>(idx) * kWarmRows * kWarmCols : nullptr;
    for (int m = threadIdx.x; m < ld; m += blockDim.x) {
        const double phi = cs.phimin + m * cs.dphi;
        S.g_m[m] = (m < I.ny) ? exp(-0.5 * I.mu * phi * phi) : 0.0;
    }
    __syncthreads();
    const double box = (I.ny - 1) * I.dphi;
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(rows) * ld; e += blockDim.x) {
        const int row = static_cast<int>(e / ld), col = static_cast<int>(e - static_cast<int64_t>(row) * ld);
        const int n = row - kPadRows, m = col - kPadCols;
        double a = 0.0, b = 0.0;
        if (n >= 0 && n < nx && m >= 0 && m < I.ny) {
            const double g = S.g_m[m];
            a = s_n[n] * g;
            if (warm && n < kWarmHarmonics) {
                // linear interpolation of the coefficient rows in phi_y
                const double u = (m * I.dphi) / box * (kWarmCols - 1);
                const int j0 = min(static_cast<int>(u), kWarmCols - 2);
                const double w = u - j0;
                const float* ra = warm + n * kWarmCols;
                a += (1.0 - w) * ra[j0] + w * ra[j0 + 1];
                if (n >= 1) {
                    const float* rb = warm + (kWarmHarmonics + n - 1) * kWarmCols;
                    b = (1.0 - w) * rb[j0] + w * rb[j0 + 1];
                }
            }
        }
        const T ta = static_cast<T>(a), tb = static_cast<T>(b), zero = static_cast<T>(0.0);
        S.plane(0, 0)[e] = ta;
        S.plane(0, 1)[e] = tb;
        S.plane(0, 2)[e] = ta;
        S.plane(0, 3)[e] = tb;
        S.plane(1, 0)[e] = zero;
        S.plane(1, 1)[e] = zero;
        S.plane(1, 2)[e] = zero;
        S.plane(1, 3)[e] = zero;
    }
    __syncthreads();
    HalfEnv<T> E{};
    E.xa = S.plane(0, 2);
    E.xb = S.plane(0, 3);
    E.ya = S.plane(0, 0);
    E.yb = S.plane(0, 1);
    E.s_n = s_n;
    E.g_m = S.g_m;
    E.acc_v = S.acc_v;
    E.acc_vc = S.acc_vc;
    E.cs = cs;
    E.h = 0.5 * cs.dt;
    E.off0 = 0;
    E.off1 = 1;
    E.k = 0;
    E.acc1 = false;
    E.salt = instance_salt(idx);
    E.R = min(B.R, kWave);
    E.nchunks = (nx + E.R - 1) / E.R;
    const int ntiles = E.nchunks * ((I.ny + kHalfCols - 1) / kHalfCols);
    for (int t = wave; t < ntiles; t += nwaves) half_tile<T>(E, t);
    __syncthreads();
}

// Period sums over phi_y, and of the cosine at the period's steps (the times
// the step kernels use), by one wavefront in a fixed order; every lane ends
// with the totals.
__device__ void period_sums(const double* acc_v, const double* acc_vc, int ny, const Consts& cs,
                            int64_t pstart, int64_t pend, double& sv, double& svc, double& sc)
{
    const int lane = threadIdx.x & (kWave - 1);
    sv = 0.0;
    svc = 0.0;
    sc = 0.0;
    for (int m = lane; m < ny; m += kWave) {
        sv += acc_v[m];
        svc += acc_vc[m];
    }
    for (int64_t kk = pstart + 1 + lane; kk <= pend; kk += kWave)
        sc += cos(cs.omega * (static_cast<double>(2 * kk) * cs.half_dt));
    wave_sum3(sv, svc, sc);
}

// The converged whole-grid state (phase 0 of the last period) in the
// warm-start encoding: a_n - a^(0)_n and b_n at 128 uniform phi_y points,
// linear interpolation between grid points.
template <typename T>
__device__ void export_state(const BatchArgs<T>& B, const SlotView<T>& S, int cur, int idx,
                             const BatchInst& I)
{
    const int nx = B.base.nx, ld = B.base.ld;
    const double* s_n = B.s_all + static_cast<size_t>(idx) * nx;
    float* out = B.state_out + static_cast<size_t>(idx) * kWarmRows * kWarmCols;
    const T* pa = S.plane(cur, 0);
    const T* pb = S.plane(cur, 1);
    for (int e = threadIdx.x; e < kWarmRows * kWarmCols; e += blockDim.x) {
        const int row = e / kWarmCols, j = e - row * kWarmCols;
        const int n = row < kWarmHarmonics ? row : row - kWarmHarmonics + 1;
        double v = 0.0;
        if (n < nx) {
            const double u = static_cast<double>(j) * (I.ny - 1) / (kWarmCols - 1);
            const int m0 = min(static_cast<int>(u), I.ny - 2);
            const double w = u - m0;
            const size_t o = static_cast<size_t>(n + kPadRows) * ld + (m0 + kPadCols);
            if (row < kWarmHarmonics) {
                const double d0 = static_cast<double>(pa[o]) - s_n[n] * S.g_m[m0];
                const double d1 = static_cast<double>(pa[o + 1]) - s_n[n] * S.g_m[m0 + 1];
                v = (1.0 - w) * d0 + w * d1;
            } else {
                v = (1.0 - w) * static_cast<double>(pb[o]) + w * static_cast<double>(pb[o + 1]);
            }
        }
        out[e] = static_cast<float>(v);
    }
}

// Harmonic chunking of the one- and two-step tiles.
struct Chunking {
    int R1, R2, n1, n2;
};
__host__ __device__ inline Chunking chunking(int nx, int R)
{
    Chunking c;
    c.R1 = R < kWave - 2 ? R : kWave - 2;
    c.R2 = R < kWave - 6 ? R : kWave - 6;
    c.n1 = (nx + c.R1 - 1) / c.R1;
    c.n2 = (nx + c.R2 - 1) / c.R2;
    return c;
}

template <typename T>
__global__ __launch_bounds__(kMaxWavesPerGroup * kWave) void k_batch(BatchArgs<T> B)
{
    __shared__ int s_q;
    __shared__ double s_red[2 * kMaxWavesPerGroup];
    __shared__ double s_tab[kMaxWavesPerGroup][kWave];
    const int nwaves = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const SlotView<T> S = slot_view(B, blockIdx.x);
    const int nx = B.base.nx;

    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_q = atomicAdd(&B.queue[0], 1);
        __syncthreads();
        const int q = uni(s_q);
        if (q >= B.n) break;
        const int idx = uni(B.order[q]);
        BatchInst I;
        Consts cs;
        load_instance(B, idx, I, cs);
        const double* s_n = B.s_all + static_cast<size_t>(idx) * nx;
        init_slot(B, S, idx, I, cs, wave, nwaves);

        // ---- whole ac periods until the absorption settles
        TileEnv<T> E{};
        E.s_n = s_n;
        E.g_m = S.g_m;
        E.acc_v = S.acc_v;
        E.acc_vc = S.acc_vc;
        E.cs = cs;
        E.acc1 = true;
        E.acc2 = true;
        E.salt = instance_salt(idx);
        const Chunking ch = chunking(nx, B.R);
        const int tiles1 = ch.n1 * ((I.ny + kFusedCols - 1) / kFusedCols);
        E.cgroup = nwaves;
        const int tiles2 = fused2_tile_count(I.ny, ch.n2, nwaves);
        int64_t k = 0;
        int cur = 0, p = 0, converged = 0, run_ok = 0;
        int32_t status = BTE_OK;
        double A_prev = 0.0, A_p = 0.0, v_p = 0.0, dA = 0.0;
        while (true) {
            ++p;
            const int64_t pstart = k;
            const int64_t pend = static_cast<int64_t>(p) * I.period_steps;
            for (int m = threadIdx.x; m < I.ny; m += blockDim.x) {
                S.acc_v[m] = 0.0;
                S.acc_vc[m] = 0.0;
            }
            __syncthreads();
            while (k < pend) {
                E.src = S.planes(cur);
                E.dst = S.planes(1 - cur);
                E.k = k;
                if (B.form == BTE_KERNEL_FUSED2 && pend - k >= 2) {
                    E.R = ch.R2;
                    E.nchunks = ch.n2;
                    for (int t = wave; t < tiles2; t += nwaves) fused2_tile<T>(E, t, &s_tab[wave][0]);
                    k += 2;
                } else {
                    E.R = ch.R1;
                    E.nchunks = ch.n1;
                    for (int t = wave; t < tiles1; t += nwaves) fused_tile<T>(E, t);
                    k += 1;
                }
                cur = 1 - cur;
                __syncthreads();
            }
            // period reduction by wavefront 0 in a fixed order whatever the
            // group size
            double sv = 0.0, svc = 0.0, sc = 0.0;
            if (wave == 0) {
                period_sums(S.acc_v, S.acc_vc, I.ny, cs, pstart, pend, sv, svc, sc);
                if (threadIdx.x == 0) {
                    s_red[0] = sv;
                    s_red[1] = svc;
                    s_red[2] = sc;
                }
            }
            __syncthreads();
            sv = s_red[0];
            svc = s_red[1];
            sc = s_red[2];
            __syncthreads();
            const double K = static_cast<double>(pend - pstart);
            v_p = I.v_norm * sv / K;
            // mean of v cos(w t) with the mean of v taken out: a period window
            // of whole steps is not exactly one period, and the dc drift would
            // otherwise leak into A_p by up to |v| dt / T
            A_p = I.two_over_ratio1 * I.v_norm * (svc - (sv / K) * sc) / K;
            dA = (p > 1) ? fabs(A_p - A_prev) : 0.0;
            if (!isfinite(A_p) || !isfinite(v_p)) {
                status = BTE_EUNSTABLE;
                break;
            }
            // a run of `confirm` consecutive small changes: a transient that
            // rotates (complex eigenvalues of the period map) can make two
            // periods agree by accident while both are still off
            run_ok = (p > 1 && dA < B.tol) ? run_ok + 1 : 0;
            if (p >= B.min_periods && run_ok >= B.confirm) {
                converged = 1;
                break;
            }
            if (p >= B.max_periods) break;
            A_prev = A_p;
        }
        if (B.state_out) export_state(B, S, cur, idx, I);
        if (threadIdx.x == 0) {
            bte_result r{};
            r.absorption = A_p;
            r.v_avg = v_p;
            r.dA = dA;
            r.steps = k;
            r.periods = p;
            r.converged = converged;
            r.status = status;
            B.results[idx] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// Wide schedule: every instance has its own slot, and each pass is one launch
// over the tiles of all instances still running (one or two steps each), so
// that a few long instances are spread over the whole GPU instead of running
// on one workgroup each.  Between passes a bookkeeping kernel (one wavefront
// per instance) advances the step counters, closes periods with the same
// fixed-order reduction and stopping rule as k_batch, and sizes the next
// pass; a one-block scan turns the per-instance block counts into the pass's
// block -> instance table.  Per-cell arithmetic, step sequence and
// reductions are those of k_batch, so both schedules give identical bits.
// ---------------------------------------------------------------------------
struct WideState {
    int64_t k;          // whole step of the current state
    int64_t pend;       // last step of the current period
    double A_prev, A_p, v_p, dA;
    int32_t p;          // current period (1-based)
    int32_t cur;        // ping-pong set holding the state
    int32_t run_ok, converged, status, done;
    int32_t form;       // steps of the next pass: 1 or 2
    int32_t nblocks;    // workgroups of the next pass (0 when done)
};

struct WideArgs {
    WideState* st;
    int32_t* first;     // [n + 1]: first block of each instance in the pass; first[n] = total
    int32_t* owner;     // [pass blocks]: instance of each block of the pass
    int32_t* remaining; // instances still running
    int wpg;            // wavefronts per workgroup
};

__host__ __device__ inline int wide_blocks(int form, int ny, const Chunking& ch, int wpg)
{
    const int tiles = form == 2 ? fused2_tile_count(ny, ch.n2, wpg)
                                : ch.n1 * ((ny + kFusedCols - 1) / kFusedCols);
    return (tiles + wpg - 1) / wpg;
}

template <typename T>
__device__ void wide_next(const BatchArgs<T>& B, const WideArgs& W, const BatchInst& I, WideState& s)
{
    s.form = (B.form == BTE_KERNEL_FUSED2 && s.pend - s.k >= 2) ? 2 : 1;
    s.nblocks = s.done ? 0 : wide_blocks(s.form, I.ny, chunking(B.base.nx, B.R), W.wpg);
}

// One workgroup per instance: initial state, start-up half-step, counters.
template <typename T>
__global__ __launch_bounds__(kMaxWavesPerGroup * kWave) void k_wide_setup(BatchArgs<T> B, WideArgs W)
{
    const int idx = blockIdx.x;
    const int nwaves = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    BatchInst I;
    Consts cs;
    load_instance(B, idx, I, cs);
    const SlotView<T> S = slot_view(B, idx);
    init_slot(B, S, idx, I, cs, wave, nwaves);
    for (int m = threadIdx.x; m < I.ny; m += blockDim.x) {
        S.acc_v[m] = 0.0;
        S.acc_vc[m] = 0.0;
    }
    if (threadIdx.x == 0) {
        WideState s{};
        s.k = 0;
        s.p = 1;
        s.pend = I.period_steps;
        s.cur = 0;
        wide_next(B, W, I, s);
        W.st[idx] = s;
    }
}

// Block -> instance table of the next pass, and the count still running.
// One block of kScanThreads: each thread sums a contiguous run of instances,
// the runs are scanned with wavefront shuffles and the wavefront totals
// through LDS (integer sums, so the order does not matter).
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_wide_scan(WideArgs W, int n)
{
    constexpr int kWaves = kScanThreads / kWave;
    __shared__ int s_wsum[kWaves];
    __shared__ int s_wleft[kWaves];
    const int t = threadIdx.x;
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int lo = min(t * per, n), hi = min(lo + per, n);
    int sum = 0, left = 0;
    for (int i = lo; i < hi; ++i) {
        sum += W.st[i].nblocks;
        left += W.st[i].done ? 0 : 1;
    }
    const int lane = t & (kWave - 1), w = t / kWave;
    int x = sum;                                  // inclusive scan within the wavefront
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    int l = left;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == kWave - 1) s_wsum[w] = x;
    if (lane == 0) s_wleft[w] = l;
    __syncthreads();
    int base = 0;
    for (int j = 0; j < w; ++j) base += s_wsum[j];
    if (t == kScanThreads - 1) W.first[n] = base + x;
    int acc = base + x - sum;                     // exclusive prefix of this thread's run
    for (int i = lo; i < hi; ++i) {
        W.first[i] = acc;
        const int nb = W.st[i].nblocks;
        for (int j = 0; j < nb; ++j) W.owner[acc + j] = i;
        acc += nb;
    }
    if (t == 0) {
        int L = 0;
        for (int j = 0; j < kWaves; ++j) L += s_wleft[j];
        W.remaining[0] = L;
    }
}

// One pass: workgroup b runs tiles of the instance whose block range holds b.
template <typename T>
__global__ __launch_bounds__(kMaxWavesPerGroup * kWave) void k_wide_pass(BatchArgs<T> B, WideArgs W)
{
    __shared__ double s_tab[kMaxWavesPerGroup][kWave];
    const int b = blockIdx.x;
    const int total = uni(W.first[B.n]);
    if (b >= total) return;
    const int idx = uni(W.owner[b]);
    const int nwaves = blockDim.x / kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int tile = (b - uni(W.first[idx])) * nwaves + wave;
    const WideState& s = W.st[idx];
    const int form = uni(s.form), cur = uni(s.cur);
    const int64_t k = uni(s.k);
    BatchInst I;
    Consts cs;
    load_instance(B, idx, I, cs);
    const SlotView<T> S = slot_view(B, idx);
    const Chunking ch = chunking(B.base.nx, B.R);
    TileEnv<T> E{};
    E.src = S.planes(cur);
    E.dst = S.planes(1 - cur);
    E.s_n = B.s_all + static_cast<size_t>(idx) * B.base.nx;
    E.g_m = S.g_m;
    E.acc_v = S.acc_v;
    E.acc_vc = S.acc_vc;
    E.cs = cs;
    E.k = k;
    E.acc1 = true;
    E.acc2 = true;
    E.salt = instance_salt(idx);
    E.cgroup = nwaves;
    if (form == 2) {
        E.R = ch.R2;
        E.nchunks = ch.n2;
        if (tile < fused2_tile_count(I.ny, ch.n2, nwaves)) fused2_tile<T>(E, tile, &s_tab[wave][0]);
    } else {
        E.R = ch.R1;
        E.nchunks = ch.n1;
        if (tile < ch.n1 * ((I.ny + kFusedCols - 1) / kFusedCols)) fused_tile<T>(E, tile);
    }
}

// After a pass: one wavefront per instance.
template <typename T>
__global__ __launch_bounds__(kWave) void k_wide_book(BatchArgs<T> B, WideArgs W)
{
    const int idx = blockIdx.x;
    WideState s = W.st[idx];
    if (s.done) return;
    BatchInst I;
    Consts cs;
    load_instance(B, idx, I, cs);
    const SlotView<T> S = slot_view(B, idx);
    s.k += s.form;
    s.cur = 1 - s.cur;
    if (s.k == s.pend) {
        const int64_t pstart = s.pend - I.period_steps;
        double sv, svc, sc;
        period_sums(S.acc_v, S.acc_vc, I.ny, cs, pstart, s.pend, sv, svc, sc);
        const double K = static_cast<double>(s.pend - pstart);
        s.v_p = I.v_norm * sv / K;
        s.A_p = I.two_over_ratio1 * I.v_norm * (svc - (sv / K) * sc) / K;
        s.dA = (s.p > 1) ? fabs(s.A_p - s.A_prev) : 0.0;
        if (!isfinite(s.A_p) || !isfinite(s.v_p)) {
            s.status = BTE_EUNSTABLE;
            s.done = 1;
        } else {
            s.run_ok = (s.p > 1 && s.dA < B.tol) ? s.run_ok + 1 : 0;
            if (s.p >= B.min_periods && s.run_ok >= B.confirm) {
                s.converged = 1;
                s.done = 1;
            } else if (s.p >= B.max_periods) {
                s.done = 1;
            }
        }
        if (!s.done) {
            s.A_prev = s.A_p;
            s.p += 1;
            s.pend = static_cast<int64_t>(s.p) * I.period_steps;
            for (int m = threadIdx.x; m < I.ny; m += blockDim.x) {
                S.acc_v[m] = 0.0;
                S.acc_vc[m] = 0.0;
            }
        }
    }
    if (s.done) {
        if (B.state_out) export_state(B, S, s.cur, idx, I);
        if (threadIdx.x == 0) {
            bte_result r{};
            r.absorption = s.A_p;
            r.v_avg = s.v_p;
            r.dA = s.dA;
            r.steps = s.k;
            r.periods = s.p;
            r.converged = s.converged;
            r.status = s.status;
            B.results[idx] = r;
        }
    }
    wide_next(B, W, I, s);
    if (threadIdx.x == 0) W.st[idx] = s;
}

}  // namespace
}  // namespace bte

// ---------------------------------------------------------------------------
// host runtime
// ---------------------------------------------------------------------------
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }


struct BatchLayout {
    int ld = 0;
    size_t elem = 8;
    size_t plane_bytes = 0, slot_bytes = 0;
    size_t off_g = 0, off_accv = 0, off_accvc = 0;
    size_t off_inst = 0, off_s = 0, off_order = 0, off_results = 0, off_queue = 0, off_slots = 0;
    size_t off_wstate = 0, off_first = 0, off_owner = 0, off_remaining = 0;   // wide schedule
    size_t total = 0;
    int groups = 0;
    int slots = 0;
};

// The wide schedule holds a state slot per instance; it is the default while
// those slots stay below this many bytes.
constexpr double kWideDefaultBytes = 64.0 * (1u << 30);

// Measured on 192 sweep draws (N_x 128, N_y 401-1601, FP32 bulk, wide):
// 58 harmonics per wave and 4 wavefronts per group ran 37.4 s; 25 / 4 and
// 40 / 4 40.7 s; 58 / 8 41.8 s; the 5 harmonics the single-instance tuner
// picks for the largest grid (it fills the GPU with one instance) 63.6 s.
bte_batch_tuning default_batch_tuning()
{
    bte_batch_tuning t{};
    t.kernel = BTE_KERNEL_FUSED2;
    t.rows_per_wave = 58;
    t.waves_per_group = 4;
    t.groups = 0;
    t.schedule = BTE_BATCH_WIDE;
    return t;
}

int device_cus()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}

BatchLayout batch_layout(const bte_batch_config& c, int n, int ny_max, const bte_batch_tuning& t)
{
    using namespace bte;
    BatchLayout L;
    int need = std::max({col_extent(ny_max, kHalfCols, 1), col_extent(ny_max, kFusedCols, 2),
                         col_extent(ny_max, kFused2Cols, 4), ny_max + 2 * kPadCols});
    L.ld = (need + 63) / 64 * 64;
    L.elem = c.precision == BTE_FP32_BULK ? 4 : 8;
    L.plane_bytes = align_up(static_cast<size_t>(c.n_x + 2 * kPadRows) * L.ld * L.elem);
    size_t o = 8 * L.plane_bytes;
    L.off_g = o; o += align_up(sizeof(double) * L.ld);
    L.off_accv = o; o += align_up(sizeof(double) * L.ld);
    L.off_accvc = o; o += align_up(sizeof(double) * L.ld);
    L.slot_bytes = o;
    L.groups = t.groups > 0 ? t.groups : device_cus() * std::max(1, kMaxWavesPerGroup / t.waves_per_group);
    // persistent: one slot per workgroup; wide: one per instance
    L.slots = t.schedule == BTE_BATCH_WIDE ? n : L.groups;
    size_t g = 0;
    L.off_queue = g; g += align_up(64);
    L.off_inst = g; g += align_up(sizeof(bte::BatchInst) * n);
    L.off_s = g; g += align_up(sizeof(double) * static_cast<size_t>(n) * c.n_x);
    L.off_order = g; g += align_up(sizeof(int32_t) * n);
    L.off_results = g; g += align_up(sizeof(bte_result) * n);
    if (t.schedule == BTE_BATCH_WIDE) {
        L.off_wstate = g; g += align_up(sizeof(bte::WideState) * n);
        L.off_first = g; g += align_up(sizeof(int32_t) * (static_cast<size_t>(n) + 1));
        // block -> instance table: at most every instance's largest pass
        const bte::Chunking ch = bte::chunking(c.n_x, t.rows_per_wave);
        const size_t per = static_cast<size_t>(std::max(bte::wide_blocks(1, ny_max, ch, t.waves_per_group),
                                                        bte::wide_blocks(2, ny_max, ch, t.waves_per_group)));
        L.off_owner = g; g += align_up(sizeof(int32_t) * per * n);
        L.off_remaining = g; g += align_up(64);
    }
    L.off_slots = g; g += L.slot_bytes * L.slots;
    L.total = g;
    return L;
}

// The default tuning for a batch: the wide schedule unless its per-instance
// slots would exceed kWideDefaultBytes.
bte_batch_tuning default_tuning_for(const bte_batch_config& c, int n, int ny_max)
{
    bte_batch_tuning t = default_batch_tuning();
    if (static_cast<double>(batch_layout(c, n, ny_max, t).slot_bytes) * n > kWideDefaultBytes)
        t.schedule = BTE_BATCH_PERSISTENT;
    return t;
}

bte_status bfail(bte_status st, const std::string& msg)
{
    bte::set_last_error(msg.c_str());
    return st;
}

bte_status validate_batch(const bte_batch_config* c, int n, const bte_instance* in,
                          const bte_batch_tuning* t, int* ny_max)
{
    if (!c || !in || n <= 0) return bfail(BTE_EINVAL, "config, instances and n > 0 required");
    if (c->n_x < 2 || c->n_x > 4096) return bfail(BTE_EINVAL, "n_x must be in 2..4096");
    if (!(c->phiy_max > c->phiy_min) || !std::isfinite(c->phiy_min) || !std::isfinite(c->phiy_max))
        return bfail(BTE_EINVAL, "need finite phiy_min < phiy_max");
    if (!(c->dt > 0) || !(c->alpha > 0) || !(c->tol > 0))
        return bfail(BTE_EINVAL, "dt, alpha and tol must be > 0");
    if (c->precision != BTE_FP64 && c->precision != BTE_FP32_BULK)
        return bfail(BTE_EINVAL, "unknown precision");
    if (c->min_periods < 2 || c->max_periods < c->min_periods)
        return bfail(BTE_EINVAL, "need 2 <= min_periods <= max_periods");
    if (c->confirm < 1 || c->confirm > 64) return bfail(BTE_EINVAL, "confirm must be in 1..64");
    if (c->reserved != 0) return bfail(BTE_EINVAL, "reserved must be 0");
    if (t) {
        if (t->kernel != BTE_KERNEL_FUSED && t->kernel != BTE_KERNEL_FUSED2)
            return bfail(BTE_EINVAL, "batch kernel must be FUSED or FUSED2");
        if (t->rows_per_wave < 1 || t->rows_per_wave > bte::kWave - 2)
            return bfail(BTE_EINVAL, "rows_per_wave out of range");
        if (t->waves_per_group != 2 && t->waves_per_group != 4 && t->waves_per_group != 8)
            return bfail(BTE_EINVAL, "waves_per_group must be 2, 4 or 8");
        if (t->groups < 0) return bfail(BTE_EINVAL, "groups must be >= 0");
        if (t->schedule != BTE_BATCH_PERSISTENT && t->schedule != BTE_BATCH_WIDE)
            return bfail(BTE_EINVAL, "schedule must be BTE_BATCH_PERSISTENT or BTE_BATCH_WIDE");
    }
    int mx = 0;
    for (int i = 0; i < n; ++i) {
        const bte_instance& I = in[i];
        const double v[] = {I.E_dc, I.E_w, I.omega, I.B, I.mu};
        for (double x : v)
            if (!std::isfinite(x)) return bfail(BTE_EINVAL, "instance " + std::to_string(i) + ": non-finite parameter");
        if (!(I.omega > 0) || !(I.mu > 0) || I.n_y < 3 || I.n_y > (1 << 20) || I.reserved != 0)
            return bfail(BTE_EINVAL, "instance " + std::to_string(i) + ": need omega > 0, mu > 0, n_y >= 3");
        const double dphi = (c->phiy_max - c->phiy_min) / (I.n_y - 1);
        if (!(c->dt * std::fabs(I.B) / (2.0 * dphi) < 1.0))
            return bfail(BTE_EINVAL, "instance " + std::to_string(i) + ": leap-frog bound dt |B| / (2 dphi) >= 1");
        mx = std::max(mx, I.n_y);
    }
    *ny_max = mx;
    return BTE_OK;
}

}  // namespace

struct bte_batch {
    bte_batch_config cfg{};
    bte_batch_tuning tune{};
    int n = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    char* ws = nullptr;
    bool owns = false;
    BatchLayout L;
    const float* warm = nullptr;
    float* state_out = nullptr;
    hipGraphExec_t graph = nullptr;       // persistent: the whole sweep; wide: set-up
    hipGraphExec_t pass_graph = nullptr;  // wide: kWidePasses passes
    const float* graph_warm = nullptr;
    float* graph_out = nullptr;
    bool ran = false;
    bool wide_running = false;            // wide: set up, not finished
    int64_t wide_replays = 0, wide_max_replays = 0;
    int wide_pass_blocks = 0;
    int32_t* remaining_host = nullptr;    // pinned landing word
};

namespace {

constexpr int kWidePasses = 64;    // passes per replay of the wide pass graph

template <typename T>
bte::BatchArgs<T> batch_args(bte_batch* b)
{
    bte::BatchArgs<T> A{};
    char* ws = b->ws;
    A.inst = reinterpret_cast<const bte::BatchInst*>(ws + b->L.off_inst);
    A.s_all = reinterpret_cast<const double*>(ws + b->L.off_s);
    A.order = reinterpret_cast<const int32_t*>(ws + b->L.off_order);
    A.warm = b->warm;
    A.state_out = b->state_out;
    A.results = reinterpret_cast<bte_result*>(ws + b->L.off_results);
    A.queue = reinterpret_cast<int32_t*>(ws + b->L.off_queue);
    A.slots = ws + b->L.off_slots;
    A.slot_bytes = b->L.slot_bytes;
    A.plane_bytes = b->L.plane_bytes;
    A.off_g = b->L.off_g;
    A.off_accv = b->L.off_accv;
    A.off_accvc = b->L.off_accvc;
    bte::Consts& c = A.base;
    c.nx = b->cfg.n_x;
    c.ld = b->L.ld;
    c.dt = b->cfg.dt;
    c.half_dt = 0.5 * b->cfg.dt;
    c.phimin = b->cfg.phiy_min;
    c.nu = 1.0 + 0.5 * b->cfg.dt;
    c.xi = 1.0 - 0.5 * b->cfg.dt;
    A.n = b->n;
    A.R = b->tune.rows_per_wave;
    A.form = b->tune.kernel;
    A.tol = b->cfg.tol;
    A.min_periods = b->cfg.min_periods;
    A.max_periods = b->cfg.max_periods;
    A.confirm = b->cfg.confirm;
    return A;
}

bte::WideArgs wide_args(bte_batch* b)
{
    bte::WideArgs W{};
    W.st = reinterpret_cast<bte::WideState*>(b->ws + b->L.off_wstate);
    W.first = reinterpret_cast<int32_t*>(b->ws + b->L.off_first);
    W.owner = reinterpret_cast<int32_t*>(b->ws + b->L.off_owner);
    W.remaining = reinterpret_cast<int32_t*>(b->ws + b->L.off_remaining);
    W.wpg = b->tune.waves_per_group;
    return W;
}

template <typename T>
hipError_t capture_batch(bte_batch* b)
{
    const bte::BatchArgs<T> A = batch_args<T>(b);
    hipLaunchKernelGGL(bte::k_batch_reset, dim3(1), dim3(64), 0, b->capture_stream, A.queue);
    hipLaunchKernelGGL(bte::k_batch<T>, dim3(b->L.groups), dim3(b->tune.waves_per_group * bte::kWave),
                       0, b->capture_stream, A);
    return hipGetLastError();
}

template <typename T>
hipError_t capture_wide_setup(bte_batch* b)
{
    const bte::BatchArgs<T> A = batch_args<T>(b);
    const bte::WideArgs W = wide_args(b);
    hipLaunchKernelGGL(bte::k_wide_setup<T>, dim3(b->n), dim3(b->tune.waves_per_group * bte::kWave),
                       0, b->capture_stream, A, W);
    hipLaunchKernelGGL(bte::k_wide_scan, dim3(1), dim3(bte::kScanThreads), 0, b->capture_stream, W, b->n);
    return hipGetLastError();
}

template <typename T>
hipError_t capture_wide_passes(bte_batch* b)
{
    const bte::BatchArgs<T> A = batch_args<T>(b);
    const bte::WideArgs W = wide_args(b);
    for (int i = 0; i < kWidePasses; ++i) {
        hipLaunchKernelGGL(bte::k_wide_pass<T>, dim3(b->wide_pass_blocks),
                           dim3(b->tune.waves_per_group * bte::kWave), 0, b->capture_stream, A, W);
        hipLaunchKernelGGL(bte::k_wide_book<T>, dim3(b->n), dim3(bte::kWave), 0, b->capture_stream,
                           A, W);
        hipLaunchKernelGGL(bte::k_wide_scan, dim3(1), dim3(bte::kScanThreads), 0, b->capture_stream, W, b->n);
    }
    return hipGetLastError();
}

// Capture `fn` on the batch's capture stream and instantiate it into *out.
bte_status capture_graph(bte_batch* b, hipError_t (*fn)(bte_batch*), hipGraphExec_t* out)
{
    if (*out) {
        (void)hipGraphExecDestroy(*out);
        *out = nullptr;
    }
    if (!b->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
    hipError_t e1 = fn(b);
    hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(BTE_EDEVICE, std::string("batch capture: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e));
    return BTE_OK;
}

bte_status build_wide_graphs(bte_batch* b)
{
    const bool f32 = b->cfg.precision == BTE_FP32_BULK;
    bte_status st = capture_graph(b, f32 ? capture_wide_setup<float> : capture_wide_setup<double>,
                                  &b->graph);
    if (st != BTE_OK) return st;
    st = capture_graph(b, f32 ? capture_wide_passes<float> : capture_wide_passes<double>,
                       &b->pass_graph);
    if (st != BTE_OK) return st;
    b->graph_warm = b->warm;
    b->graph_out = b->state_out;
    return BTE_OK;
}

bte_status build_batch_graph(bte_batch* b)
{
    bte_status st = capture_graph(
        b, b->cfg.precision == BTE_FP32_BULK ? capture_batch<float> : capture_batch<double>, &b->graph);
    if (st != BTE_OK) return st;
    b->graph_warm = b->warm;
    b->graph_out = b->state_out;
    return BTE_OK;
}

}  // namespace

extern "C" {

bte_status bte_batch_workspace_bytes(const bte_batch_config* cfg, int32_t n,
                                     const bte_instance* inst, const bte_batch_tuning* tuning,
                                     size_t* bytes)
{
    int ny_max = 0;
    bte_status st = validate_batch(cfg, n, inst, tuning, &ny_max);
    if (st != BTE_OK) return st;
    if (!bytes) return bfail(BTE_EINVAL, "bytes must not be NULL");
    const bte_batch_tuning t = tuning ? *tuning : default_tuning_for(*cfg, n, ny_max);
    const BatchLayout L = batch_layout(*cfg, n, ny_max, t);
    if (4.0 * static_cast<double>(L.plane_bytes) >= 2147483648.0)
        return bfail(BTE_EINVAL, "grid too large: a set of four state planes must stay below 2 GiB");
    *bytes = L.total;
    return BTE_OK;
}

bte_status bte_batch_create(const bte_batch_config* cfg, int32_t n, const bte_instance* inst,
                            const bte_batch_tuning* tuning, void* workspace,
                            size_t workspace_bytes, void* hip_stream, bte_batch** out)
{
    if (!out) return bfail(BTE_EINVAL, "out must not be NULL");
    *out = nullptr;
    int ny_max = 0;
    bte_status st = validate_batch(cfg, n, inst, tuning, &ny_max);
    if (st != BTE_OK) return st;
    const bte_batch_tuning t = tuning ? *tuning : default_tuning_for(*cfg, n, ny_max);
    BatchLayout L = batch_layout(*cfg, n, ny_max, t);
    if (4.0 * static_cast<double>(L.plane_bytes) >= 2147483648.0)
        return bfail(BTE_EINVAL, "grid too large: a set of four state planes must stay below 2 GiB");
    if (workspace && workspace_bytes < L.total)
        return bfail(BTE_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    if (workspace && reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return bfail(BTE_EINVAL, "workspace must be 256-byte aligned");

    bte_batch* b = new bte_batch();
    b->cfg = *cfg;
    b->tune = t;
    b->n = n;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->L = L;
    if (workspace) {
        b->ws = static_cast<char*>(workspace);
    } else {
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->ws), L.total);
        if (e != hipSuccess) {
            delete b;
            return bfail(BTE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        b->owns = true;
    }

    // per-instance tables
    std::vector<bte::BatchInst> I(n);
    std::vector<double> S(static_cast<size_t>(n) * cfg->n_x);
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) {
        const bte_instance& x = inst[i];
        bte::BatchInst& y = I[i];
        y.E_dc = x.E_dc;
        y.E_w = x.E_w;
        y.omega = x.omega;
        y.B = x.B;
        y.mu = x.mu;
        y.ny = x.n_y;
        y.dphi = (cfg->phiy_max - cfg->phiy_min) / (x.n_y - 1);
        y.period_steps = std::max<int64_t>(1, std::llround(2.0 * kPi / (x.omega * cfg->dt)));
        std::vector<double> r = bte::bessel_ratio_table(x.mu, cfg->n_x);
        y.two_over_ratio1 = 2.0 / r[1];
        y.v_norm = kPi * std::sqrt(cfg->alpha) * y.dphi;
        const double norm = std::sqrt(x.mu / (2.0 * kPi * cfg->alpha)) / kPi;
        for (int k = 0; k < cfg->n_x; ++k)
            S[static_cast<size_t>(i) * cfg->n_x + k] = (k == 0 ? 0.5 : 1.0) * r[k] * norm;
        // expected cost: cells x steps of the first min_periods periods or ~14
        // relaxation times, whichever is longer
        const double t_run = std::max(cfg->min_periods * 2.0 * kPi / x.omega, 14.0);
        cost[i] = static_cast<double>(x.n_y) * cfg->n_x * t_run / cfg->dt;
    }
    if (t.schedule == BTE_BATCH_WIDE) {
        // pass grid: every instance's largest block count; the longest
        // possible run (max_periods periods of one-step passes) bounds the
        // replays
        const bte::Chunking ch = bte::chunking(cfg->n_x, t.rows_per_wave);
        int64_t blocks = 0, steps = 0;
        for (int i = 0; i < n; ++i) {
            const int b1 = bte::wide_blocks(1, I[i].ny, ch, t.waves_per_group);
            const int b2 = t.kernel == BTE_KERNEL_FUSED2 ? bte::wide_blocks(2, I[i].ny, ch, t.waves_per_group) : 0;
            blocks += std::max(b1, b2);
            steps = std::max<int64_t>(steps, I[i].period_steps * cfg->max_periods);
        }
        if (blocks > (int64_t{1} << 30)) {
            bte_batch_destroy(b);
            return bfail(BTE_EINVAL, "batch too large for the wide schedule");
        }
        b->wide_pass_blocks = static_cast<int>(std::max<int64_t>(blocks, 1));
        b->wide_max_replays = steps / kWidePasses + 2;
        hipError_t eh = hipHostMalloc(reinterpret_cast<void**>(&b->remaining_host), sizeof(int32_t));
        if (eh != hipSuccess) {
            b->remaining_host = nullptr;
            bte_batch_destroy(b);
            return bfail(BTE_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(eh));
        }
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });

    hipError_t e = hipMemcpyAsync(b->ws + L.off_inst, I.data(), sizeof(bte::BatchInst) * n,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_s, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_order, order.data(), sizeof(int32_t) * n,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws + L.off_results, 0, sizeof(bte_result) * n, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        bte_batch_destroy(b);
        return bfail(BTE_EDEVICE, std::string("batch tables: ") + hipGetErrorString(e));
    }
    *out = b;
    return BTE_OK;
}

bte_status bte_batch_set_warm_start(bte_batch* b, const float* dev_coeffs)
{
    if (!b) return bfail(BTE_EINVAL, "batch is NULL");
    b->warm = dev_coeffs;
    return BTE_OK;
}

bte_status bte_batch_set_state_output(bte_batch* b, float* dev_coeffs)
{
    if (!b) return bfail(BTE_EINVAL, "batch is NULL");
    b->state_out = dev_coeffs;
    return BTE_OK;
}

bte_status bte_batch_advance(bte_batch* b, int32_t max_replays, int32_t* remaining)
{
    if (!b || !remaining) return bfail(BTE_EINVAL, "batch and remaining must not be NULL");
    if (b->tune.schedule != BTE_BATCH_WIDE) return bfail(BTE_ESTATE, "bte_batch_advance needs the wide schedule");
    if (max_replays < 1) return bfail(BTE_EINVAL, "max_replays must be >= 1");
    if (!b->wide_running) {
        if (!b->graph || !b->pass_graph || b->graph_warm != b->warm || b->graph_out != b->state_out) {
            bte_status st = build_wide_graphs(b);
            if (st != BTE_OK) return st;
        }
        hipError_t e = hipGraphLaunch(b->graph, b->stream);
        if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        b->wide_running = true;
        b->wide_replays = 0;
        b->ran = false;
    }
    for (int32_t r = 0; r < max_replays; ++r) {
        if (b->wide_replays >= b->wide_max_replays) {
            b->wide_running = false;
            return bfail(BTE_EDEVICE, "wide sweep did not finish within its pass bound");
        }
        hipError_t e = hipGraphLaunch(b->pass_graph, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->remaining_host, b->ws + b->L.off_remaining, sizeof(int32_t),
                               hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) {
            b->wide_running = false;
            return bfail(BTE_EDEVICE, std::string("wide pass: ") + hipGetErrorString(e));
        }
        ++b->wide_replays;
        *remaining = *b->remaining_host;
        if (*remaining == 0) {
            b->wide_running = false;
            b->ran = true;
            return BTE_OK;
        }
    }
    return BTE_OK;
}

bte_status bte_batch_run(bte_batch* b)
{
    if (!b) return bfail(BTE_EINVAL, "batch is NULL");
    if (b->tune.schedule == BTE_BATCH_WIDE) {
        b->wide_running = false;     // a run always starts from the set-up
        int32_t left = 1;
        while (true) {
            bte_status st = bte_batch_advance(b, 1 << 20, &left);
            if (st != BTE_OK) return st;
            if (left == 0) return BTE_OK;
        }
    }
    if (!b->graph || b->graph_warm != b->warm || b->graph_out != b->state_out) {
        bte_status st = build_batch_graph(b);
        if (st != BTE_OK) return st;
    }
    hipError_t e = hipGraphLaunch(b->graph, b->stream);
    if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    b->ran = true;
    return BTE_OK;
}

bte_status bte_batch_results(bte_batch* b, bte_result* out)
{
    if (!b || !out) return bfail(BTE_EINVAL, "batch and out must not be NULL");
    if (!b->ran) return bfail(BTE_ESTATE, "bte_batch_run has not been called");
    hipError_t e = hipMemcpyAsync(out, b->ws + b->L.off_results, sizeof(bte_result) * b->n,
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(BTE_EDEVICE, std::string("results: ") + hipGetErrorString(e));
    return BTE_OK;
}

bte_status bte_batch_get_tuning(const bte_batch* b, bte_batch_tuning* t)
{
    if (!b || !t) return bfail(BTE_EINVAL, "batch and tuning must not be NULL");
    *t = b->tune;
    t->groups = b->L.groups;
    return BTE_OK;
}

}  // extern "C"

// ---- sweep autotuner ------------------------------------------------------------
// The per-step cost of an instance depends only on its grid (N_x shared, its
// own N_y) and the tile shape, not on its fields: the tuner runs samples of
// the batch whose N_y values follow the batch's share of cells, with omega
// raised so that every instance runs exactly `kTunePeriods` periods of
// `kTunePeriodSteps` steps (a fixed, known amount of work), through the wide
// schedule, and times them.  Stage one ranks every candidate on a small
// sample; stage two re-times the best few on a sample as large as the batch
// (up to kTuneLarge instances), since a shape's rate can change once the
// passes carry thousands of instances (ties at a hundred instances have come
// apart by a tenth at four thousand).
namespace {
constexpr int kTuneSample = 128;        // instances in the stage-one sample (at most)
constexpr int kTuneLarge = 4096;        // instances in the stage-two sample (at most)
constexpr int kTuneFinalists = 3;       // candidates re-timed in stage two
constexpr int kTunePeriodSteps = 400;   // steps per period of a sample instance
constexpr int kTunePeriods = 2;

struct TuneKey {
    int n_x, precision;
    int size_class;                     // smallest power of two >= min(n, kTuneLarge)
    std::vector<int> ny;                // distinct N_y values of the batch, sorted
    bool operator<(const TuneKey& o) const
    {
        if (n_x != o.n_x) return n_x < o.n_x;
        if (precision != o.precision) return precision < o.precision;
        if (size_class != o.size_class) return size_class < o.size_class;
        return ny < o.ny;
    }
};

int size_class(int n)
{
    int c = 1;
    while (c < std::min(n, kTuneLarge)) c <<= 1;
    return c;
}
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<bte_batch_tuning, double>> g_tune_cache;

// Harmonics per wave that split N_x into c equal chunks (c = 1 .. 8), up to
// the form's limit.
std::vector<int> balanced_rows(int nx, int rmax)
{
    std::vector<int> r;
    for (int c = 1; c <= 8; ++c) {
        const int R = (nx + c - 1) / c;
        if (R <= rmax && (r.empty() || r.back() != R)) r.push_back(R);
    }
    return r;
}

// m sample instances (about; at least one per class): each N_y class in
// proportion to its share of the batch's cells, with a representative's
// fields and omega set for periods of kTunePeriodSteps steps.
std::vector<bte_instance> tune_sample(const bte_batch_config* cfg, int n, const bte_instance* inst,
                                      const std::map<int, double>& cells, int m)
{
    double total = 0.0;
    for (const auto& kv : cells) total += kv.second;
    std::vector<bte_instance> sample;
    for (const auto& kv : cells) {
        const int k = std::max(1, static_cast<int>(std::lround(m * kv.second / total)));
        const bte_instance* rep = nullptr;
        for (int i = 0; i < n && !rep; ++i)
            if (inst[i].n_y == kv.first) rep = &inst[i];
        bte_instance x = *rep;
        x.omega = 2.0 * kPi / (kTunePeriodSteps * cfg->dt);
        for (int j = 0; j < k; ++j) sample.push_back(x);
    }
    return sample;
}

// Cell-steps per second of the sample under tuning t (the second of two runs:
// the first captures the graphs), or an error status.
bte_status time_sample(const bte_batch_config& c, const std::vector<bte_instance>& sample,
                       const bte_batch_tuning& t, void* hip_stream, double* rate)
{
    double work = 0.0;
    for (const bte_instance& x : sample)
        work += static_cast<double>(x.n_y) * c.n_x * kTunePeriods * kTunePeriodSteps;
    bte_batch* b = nullptr;
    bte_status st = bte_batch_create(&c, static_cast<int32_t>(sample.size()), sample.data(), &t,
                                     nullptr, 0, hip_stream, &b);
    if (st != BTE_OK) return st;
    double secs = 1e300;
    for (int rep = 0; rep < 2 && st == BTE_OK; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        st = bte_batch_run(b);
        const auto t1 = std::chrono::steady_clock::now();
        secs = std::chrono::duration<double>(t1 - t0).count();
    }
    bte_batch_destroy(b);
    if (st != BTE_OK) return st;
    *rate = work / secs;
    return BTE_OK;
}
}  // namespace

extern "C" {

bte_status bte_batch_tune(const bte_batch_config* cfg, int32_t n, const bte_instance* inst,
                          void* hip_stream, int32_t use_cache, bte_batch_tuning* out,
                          double* cell_steps_per_s)
{
    if (!out) return bfail(BTE_EINVAL, "out must not be NULL");
    int ny_max = 0;
    bte_status st = validate_batch(cfg, n, inst, nullptr, &ny_max);
    if (st != BTE_OK) return st;
    // cells per distinct N_y, and the cache key
    std::map<int, double> cells;
    for (int i = 0; i < n; ++i) cells[inst[i].n_y] += static_cast<double>(inst[i].n_y) * cfg->n_x;
    TuneKey key{cfg->n_x, cfg->precision, size_class(n), {}};
    for (const auto& kv : cells) key.ny.push_back(kv.first);
    if (use_cache) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second.first;
            if (cell_steps_per_s) *cell_steps_per_s = it->second.second;
            return BTE_OK;
        }
    }
    bte_batch_config c = *cfg;
    c.min_periods = c.max_periods = kTunePeriods;
    c.confirm = 1;

    std::vector<bte_batch_tuning> cand;
    for (int form : {BTE_KERNEL_FUSED2, BTE_KERNEL_FUSED})
        for (int R : balanced_rows(c.n_x, form == BTE_KERNEL_FUSED2 ? 58 : bte::kWave - 2))
            for (int w : {2, 4, 8}) {
                bte_batch_tuning t{};
                t.kernel = form;
                t.rows_per_wave = R;
                t.waves_per_group = w;
                t.groups = 0;
                t.schedule = BTE_BATCH_WIDE;
                cand.push_back(t);
            }
    // the samples' state slots stay within the wide schedule's default budget
    const double slot = static_cast<double>(batch_layout(c, 1, ny_max, cand[0]).slot_bytes);
    const int cap = std::max(1, static_cast<int>(std::min(kWideDefaultBytes / slot, 1e9)));
    // stage one: every candidate on the small sample
    const int m1 = std::min({n, kTuneSample, cap});
    const std::vector<bte_instance> small = tune_sample(cfg, n, inst, cells, m1);
    std::vector<std::pair<double, int>> ranked;      // (rate, candidate), best first
    for (int i = 0; i < static_cast<int>(cand.size()); ++i) {
        double rate = 0.0;
        st = time_sample(c, small, cand[i], hip_stream, &rate);
        if (st != BTE_OK) return st;
        ranked.push_back({rate, i});
    }
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
    bte_batch_tuning best = cand[ranked[0].second];
    double best_rate = ranked[0].first;
    // stage two: the finalists on a sample as large as the batch
    const int m2 = std::min({n, kTuneLarge, cap});
    if (m2 > m1) {
        const std::vector<bte_instance> large = tune_sample(cfg, n, inst, cells, m2);
        best_rate = -1.0;
        const int f = std::min<int>(kTuneFinalists, static_cast<int>(ranked.size()));
        for (int j = 0; j < f; ++j) {
            const bte_batch_tuning& t = cand[ranked[j].second];
            double rate = 0.0;
            st = time_sample(c, large, t, hip_stream, &rate);
            if (st != BTE_OK) return st;
            if (rate > best_rate) {
                best_rate = rate;
                best = t;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = {best, best_rate};
    }
    *out = best;
    if (cell_steps_per_s) *cell_steps_per_s = best_rate;
    return BTE_OK;
}

void bte_batch_destroy(bte_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->pass_graph) (void)hipGraphExecDestroy(b->pass_graph);
    if (b->remaining_host) (void)hipHostFree(b->remaining_host);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->owns && b->ws) (void)hipFree(b->ws);
    delete b;
}

}  // extern "C"
