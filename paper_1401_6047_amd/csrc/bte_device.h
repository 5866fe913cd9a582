// Device-side building blocks of the superlattice BTE kernels: cross-lane
// moves, the pointwise Crank-Nicolson operator, FP32 stochastic rounding,
// buffer row access, and the per-tile bodies of the step kernels.  Included by
// the single-instance kernels and by the batched sweep so that both run the
// same arithmetic.  Internal to the library.
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
// adjacent lanes through cross-lane shuffles, not from memory.  A tile that
// chains several half-steps recomputes the earlier ones on halo columns and
// harmonics, so tiles never wait for each other within a launch; reads and
// writes then go to different (ping-pong) buffers.
#pragma once

#include <algorithm>
#include <type_traits>

#include "bte_internal.h"

namespace bte {
namespace detail {


// ---- cross-lane moves --------------------------------------------------------
// DPP wave shifts move a value one lane up or down the whole 64-lane wave in a
// single VALU instruction per 32-bit half (no LDS round trip).  Lane l holds
// phi_y column m, so "from left" is column m-1 and "from right" column m+1.
// The two edge lanes receive garbage and are never used for output.
constexpr int kDppWaveShr1 = 0x138;   // lane l <- lane l-1
constexpr int kDppWaveShl1 = 0x130;   // lane l <- lane l+1

__device__ __forceinline__ double dpp_move(double v, int ctrl_is_shr)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int rlo, rhi;
    if (ctrl_is_shr) {
        rlo = __builtin_amdgcn_mov_dpp(lo, kDppWaveShr1, 0xF, 0xF, true);
        rhi = __builtin_amdgcn_mov_dpp(hi, kDppWaveShr1, 0xF, 0xF, true);
    } else {
        rlo = __builtin_amdgcn_mov_dpp(lo, kDppWaveShl1, 0xF, 0xF, true);
        rhi = __builtin_amdgcn_mov_dpp(hi, kDppWaveShl1, 0xF, 0xF, true);
    }
    return __hiloint2double(rhi, rlo);
}

// Centred difference across phi_y of a row held one column per lane:
// v(m+1) - v(m-1).  The coupling terms A^t and B^t of Sec. 3 only ever use
// the other grid through these differences, at harmonics n-1 and n+1.
__device__ __forceinline__ double dphi_diff(double v)
{
    return dpp_move(v, 0) - dpp_move(v, 1);
}

// Broadcast lane `l` (wave-uniform) of a per-lane double to the whole wave.
__device__ __forceinline__ double lane_bcast(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 1/d for d >= 1: hardware reciprocal refined by two Newton steps (the error
// is within a couple of ulp of the correctly rounded quotient).
__device__ __forceinline__ double recip(double d)
{
    double x = __builtin_amdgcn_rcp(d);
    double e = fma(-d, x, 1.0);
    x = fma(x, e, x);
    e = fma(-d, x, 1.0);
    return fma(x, e, x);
}

// Operator T of Sec. 3 for one cell: Crank-Nicolson over a step h.
//   g = a xi - b mu0 + B^t + a0 h,   h' = b xi + a mu0 + A^t,
//   nu a' + mu1 b' = g,  nu b' - mu1 a' = h'  =>  Cramer's rule.
__device__ __forceinline__ void op_T(double a, double b, double At, double Bt, double a0h,
                                     double mu0, double mu1, double nu, double xi, double& an,
                                     double& bn)
{
    const double g = fma(a, xi, fma(-b, mu0, Bt + a0h));
    const double hh = fma(b, xi, fma(a, mu0, At));
    const double inv = recip(fma(mu1, mu1, nu * nu));
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

// Tile of this wavefront, made provably wave-uniform so that everything derived
// from it (rows, loop bounds, row addresses) lives in scalar registers.
__device__ __forceinline__ int wave_tile()
{
    const int t = xcd_block() * (blockDim.x / kWave) + (threadIdx.x / kWave);
    return __builtin_amdgcn_readfirstlane(t);
}

// Row access through a buffer resource: the row offset is a scalar (SGPR)
// operand and the lane's column a 32-bit VGPR offset, so no vector address
// arithmetic is spent per access.  The descriptor's record count is the
// extent it covers (a plane, or the four planes of a state set): an access
// outside it reads 0 and a store is dropped.
constexpr int kBufferWord3 = 0x00020000;   // gfx9 raw buffer, no format conversion

// ---- FP32 storage with stochastic rounding -------------------------------------
// In FP32-bulk mode every cell update is computed in FP64 and stored in FP32.
// Round-to-nearest would make the storage error of a slowly drifting state
// systematic: a step changes a value by ~dt of itself, only a few float ulp,
// and the same rounding direction repeats step after step.  Stochastic
// rounding (round up with probability equal to the discarded fraction) makes
// each storage error zero-mean and independent, so the errors average out in
// the drift velocity and absorption.  The random bits come from a
// counter-based hash of (step, plane, cell), so runs are reproducible.
// mix32 is the published "lowbias32" integer hash (xor-shift 16, multiply,
// xor-shift 15, multiply, xor-shift 16, with the two multipliers found by
// C. Wellons' hash-prospector search).
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Per-launch, per-plane seed.  The odd constants only spread the step and
// plane indices over the word before hashing: 0x9E3779B9 is 2^32 divided by
// the golden ratio (Knuth's multiplicative hashing), 0x85EBCA6B a multiplier
// of the MurmurHash3 finaliser and 0x27D4EB2F one of the xxHash32 primes.
__device__ __forceinline__ uint32_t plane_seed(int64_t k, uint32_t tag)
{
    const uint32_t lo = static_cast<uint32_t>(k), hi = static_cast<uint32_t>(static_cast<uint64_t>(k) >> 32);
    return mix32(mix32(lo * 0x9E3779B9U + hi) ^ (tag * 0x85EBCA6BU + 0x27D4EB2FU));
}

// FP64 -> FP32 with stochastic rounding: add 29 random bits below the float
// mantissa of the double's bit pattern, truncate them, convert (now exact).
__device__ __forceinline__ float round_stochastic(double x, uint32_t rnd)
{
    uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    b += static_cast<uint64_t>(rnd >> 3);
    b &= ~((static_cast<uint64_t>(1) << 29) - 1);
    return static_cast<float>(__longlong_as_double(static_cast<long long>(b)));
}

template <typename T>
struct RowAddr {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t row_bytes;   // ld * sizeof(T)
    uint32_t col_bytes;   // (m + kPadCols) * sizeof(T), per lane
    uint32_t seed;        // stochastic-rounding seed of this plane and launch (FP32 only)
    uint32_t poff;        // byte offset of this plane from the descriptor's base
    __device__ __forceinline__ RowAddr(const T* base, uint32_t bytes, uint32_t rb, uint32_t cb,
                                       uint32_t sd = 0, uint32_t po = 0)
        : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), static_cast<short>(0),
                                                 static_cast<int>(bytes), kBufferWord3)),
          row_bytes(rb), col_bytes(cb), seed(sd), poff(po)
    {
    }
    __device__ __forceinline__ int soff(int j) const
    {
        return static_cast<int>(static_cast<uint32_t>(j + kPadRows) * row_bytes + poff);
    }
    __device__ __forceinline__ double load(int j) const
    {
        if constexpr (sizeof(T) == 8) {
            auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, col_bytes, soff(j), 0);
            return __builtin_bit_cast(double, v);
        } else {
            auto v = __builtin_amdgcn_raw_buffer_load_b32(rsrc, col_bytes, soff(j), 0);
            return static_cast<double>(__builtin_bit_cast(float, v));
        }
    }
    __device__ __forceinline__ void store(int j, double x) const
    {
        if constexpr (sizeof(T) == 8) {
            using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc, 0u, 0, 0));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), rsrc, col_bytes, soff(j), 0);
        } else {
            using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(rsrc, 0u, 0, 0));
            const uint32_t cell = static_cast<uint32_t>(soff(j)) - poff + col_bytes;
            const float f = round_stochastic(x, mix32(seed ^ cell));
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, f), rsrc, col_bytes, soff(j), 0);
        }
    }
};

// The four planes of a state set lie at one stride, in the order a_h, b_h,
// a_f, b_f (both the single-instance workspace and the batch slots are laid
// out so, and the launchers check it): one buffer descriptor then covers the
// set and a plane is a fixed byte offset into it, which leaves the march far
// fewer scalar registers to hold than a descriptor per plane.
template <typename T>
__device__ __forceinline__ uint32_t plane_stride(const Planes<T>& P)
{
    return static_cast<uint32_t>(reinterpret_cast<const char*>(P.b_h) -
                                 reinterpret_cast<const char*>(P.a_h));
}

// Everything a tile of a step kernel reads besides its tile index.  The
// single-instance kernels fill it from the device control block; the batched
// sweep fills it per instance and step.
template <typename T>
struct TileEnv {
    Planes<T> src;            // physical plane bases (row -kPadRows, column -kPadCols)
    Planes<T> dst;
    const double* s_n;        // source coefficients sigma(n) I_n/(pi I_0) sqrt(mu/(2 pi alpha))
    const double* g_m;        // exp(-mu phi_y(m)^2 / 2)
    double* acc_v;            // per-phi_y window sums of b_1 and b_1 cos(w t)
    double* acc_vc;
    Consts cs;
    int64_t k;                // step of the source state
    bool acc1, acc2, acc3;    // steps k+1, k+2, k+3 enter the window sums
    uint32_t salt;            // stochastic-rounding seed offset (instance)
    int R;                    // harmonics per wave
    int nchunks;              // ceil(nx / R)
    int cgroup;               // two-step tiles: phi_y strips per column group (see fused2_tile)
    bool even_progress;       // the whole launch is resident at once (see march_priority)
};

// Issue priority by progress through the march.  Two wavefronts sharing a
// SIMD otherwise run oldest-first: one finishes about as fast as if it were
// alone, and the other then runs its remainder alone, at the lower issue rate
// of a single wavefront.  Lowering a wavefront's priority as it advances (four
// levels over its iterations) keeps the progress of the wavefronts on a SIMD
// even, so that they overlap for most of the launch.  Only used when every
// wavefront of the launch is resident at once (with more wavefronts than
// slots it would hold back the wavefronts that free a slot for the next) and
// they fill a good part of the device.
__device__ __forceinline__ void march_priority(int i, int iters)
{
    const int lvl = (i * 4) / iters;
    if (lvl == 0) __builtin_amdgcn_s_setprio(3);
    else if (lvl == 1) __builtin_amdgcn_s_setprio(2);
    else if (lvl == 2) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Tiles of the two-step kernel for a grid of `ncol` phi_y strips, in column
// groups of `cgroup` strips (the last group padded): the kernels launch or
// loop over this many tile indices and fused2_tile skips the padding.
__host__ __device__ inline int fused2_tile_count(int ny, int nchunks, int cgroup)
{
    const int ncol = (ny + kFused2Cols - 1) / kFused2Cols;
    return nchunks * ((ncol + cgroup - 1) / cgroup) * cgroup;
}

__host__ __device__ inline int fused3_tile_count(int ny, int nchunks, int cgroup)
{
    const int ncol = (ny + kFused3Cols - 1) / kFused3Cols;
    return nchunks * ((ncol + cgroup - 1) / cgroup) * cgroup;
}

template <typename T>
struct HalfEnv {
    T* xa;                    // updated in place (physical bases)
    T* xb;
    const T* ya;              // coupling source
    const T* yb;
    const double* s_n;
    const double* g_m;
    double* acc_v;
    double* acc_vc;
    Consts cs;
    double h;                 // step length (dt, or dt/2 for the start-up)
    int off0, off1;           // half-step time indices relative to 2k
    int64_t k;
    bool acc1;                // the new b_1 row enters the window sums at step k+1
    uint32_t salt;
    int R;
    int nchunks;
};

// Registers of one slot of the sliding window (see k_fused_step).
struct RowRegs {
    double fa, fb;     // old fractional grid, own column
    double dfa, dfb;   // its phi_y differences
    double dha, dhb;   // phi_y differences of the new whole grid (row r or r-3)
    double nfa, nfb;   // in flight: inputs of the iteration that next uses this
    double nha, nhb;   //   slot as its centre row (old fractional row j+1, old whole row j)
};

// One fused leap-frog step on one tile (see the file comment of the kernels).
template <typename T>
__device__ __forceinline__ void fused_tile(const TileEnv<T>& A, int tile)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    const int ct = tile / A.nchunks;
    const int r0 = (tile - ct * A.nchunks) * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kFusedCols - 2 + lane;        // this lane's phi_y column
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 2) && (lane < kWave - 2) && col_ok;

    const int64_t k = A.k;
    double cw[4];
    field_cosines(cs, k, cw);
    const bool acc_step = A.acc1;

    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gdt = (col_ok ? A.g_m[m] : 0.0) * cs.dt;
    // s_n of harmonics r0-1 .. r1 (at most 64 of them), one per lane; row j's
    // value is broadcast from lane j - (r0 - 1).
    const double s_lane = A.s_n[min(max(r0 - 1 + lane, 0), cs.nx - 1)];
    const double hdt = 0.5 * cs.dt;
    // mu^t = n beta^t dt/2 with beta^t = E(t) + B phi: per-lane factor q, mu = n q.
    const double q0h = (fma(cs.E_w, cw[0], cs.E_dc) + cs.B * phi) * hdt;  // t = k dt
    const double q1h = (fma(cs.E_w, cw[2], cs.E_dc) + cs.B * phi) * hdt;  // t = (k+1) dt
    const double q0f = (fma(cs.E_w, cw[1], cs.E_dc) + cs.B * phi) * hdt;  // (k+1/2) dt
    const double q1f = (fma(cs.E_w, cw[3], cs.E_dc) + cs.B * phi) * hdt;  // (k+3/2) dt
    const double c = cs.c_full, nu = cs.nu, xi = cs.xi;

    const uint32_t rb = static_cast<uint32_t>(cs.ld) * sizeof(T);
    const uint32_t cb = static_cast<uint32_t>(m + kPadCols) * sizeof(T);
    const uint32_t pb = static_cast<uint32_t>(cs.nx + 2 * kPadRows) * rb;
    const uint32_t ss = plane_stride(A.src), sd = plane_stride(A.dst);
    const RowAddr<T> aHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 0);
    const RowAddr<T> bHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, ss);
    const RowAddr<T> aFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 2 * ss);
    const RowAddr<T> bFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 3 * ss);
    const RowAddr<T> aHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 0 + A.salt), 0);
    const RowAddr<T> bHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 1 + A.salt), sd);
    const RowAddr<T> aFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 2 + A.salt), 2 * sd);
    const RowAddr<T> bFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 3 + A.salt), 3 * sd);

    // Sliding window over harmonics.  Iteration j computes the new whole grid
    // at harmonic j (needs old fractional rows j-1, j+1) and the new
    // fractional grid at harmonic j-1 (needs new whole rows j-2, j).  Row r's
    // registers live in slot r mod 3; the slot of row j+1 still holds the new
    // whole-grid differences of row j-2 when iteration j reads them.
    RowRegs S[3];
    S[0] = S[1] = S[2] = RowRegs{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int jlo = r0 - 1;
    // Loads run three iterations ahead: iteration j consumes old fractional
    // row j+1 and old whole row j from the slot of row j and refills that slot
    // with the inputs of iteration j+3.  Clamped rows stay inside the plane;
    // the values loaded for iterations past the end are never used.
    auto issue = [&](RowRegs& P, int j) {
        const int jf = min(j + 1, r1 + 1);
        const int jh = min(j, r1);
        P.nfa = aFs.load(jf);
        P.nfb = bFs.load(jf);
        P.nha = aHs.load(jh);
        P.nhb = bHs.load(jh);
    };
    // prime: old fractional rows r0-2 (slot of jlo-1) and r0-1 (slot of jlo)
    {
        RowRegs& a = S[0];
        a.fa = aFs.load(r0 - 2);
        a.fb = bFs.load(r0 - 2);
        RowRegs& b = S[1];
        b.fa = aFs.load(r0 - 1);
        b.fb = bFs.load(r0 - 1);
        issue(S[1], jlo);
        issue(S[2], jlo + 1);
        issue(S[0], jlo + 2);
        a.dfa = dphi_diff(a.fa);
        a.dfb = dphi_diff(a.fb);
        b.dfa = dphi_diff(b.fa);
        b.dfb = dphi_diff(b.fb);
    }

    auto iter = [&](int j, RowRegs& Pm, RowRegs& P0, RowRegs& Pp) {
        // old fractional row j+1 and old whole row j, loaded three iterations ago
        Pp.fa = P0.nfa;
        Pp.fb = P0.nfb;
        const double ha_old = P0.nha, hb_old = P0.nhb;
        issue(P0, j + 3);
        Pp.dfa = dphi_diff(Pp.fa);
        Pp.dfb = dphi_diff(Pp.fb);

        // ---- whole grid, harmonic j: z^{k+1} = T(z^k; A, B from z^{k+1/2})
        const double sdt = lane_bcast(s_lane, min(j - (r0 - 1), kWave - 1)) * gdt;
        const double chi = (j == 1) ? 2.0 : 1.0;
        const double nd = static_cast<double>(j);
        double ha, hb;
        op_T(ha_old, hb_old, c * (chi * Pm.dfa - Pp.dfa), c * (Pp.dfb - Pm.dfb), sdt, nd * q0h,
             nd * q1h, nu, xi, ha, hb);
        const bool row_a = (j >= 0) && (j < cs.nx) && col_ok;
        ha = row_a ? ha : 0.0;
        hb = (row_a && j >= 1) ? hb : 0.0;
        if (j >= r0 && j < r1) {
            if (out_lane) {
                aHd.store(j, ha);
                bHd.store(j, hb);
                if (j == 1 && acc_step) {            // drift-velocity window sums
                    A.acc_v[m] += hb;
                    A.acc_vc[m] += hb * cw[2];
                }
            }
        }
        P0.dha = dphi_diff(ha);
        P0.dhb = dphi_diff(hb);

        // ---- fractional grid, harmonic j-1: z^{k+3/2} = T(z^{k+1/2}; A, B from z^{k+1})
        const int n = j - 1;
        if (n >= r0 && n < r1) {
            const double sdt1 = lane_bcast(s_lane, n - (r0 - 1)) * gdt;
            const double chi1 = (n == 1) ? 2.0 : 1.0;
            const double nd1 = static_cast<double>(n);
            double fa, fb;
            // new whole rows n-1 = j-2 (held in the slot of j+1) and n+1 = j
            op_T(Pm.fa, Pm.fb, c * (chi1 * Pp.dha - P0.dha), c * (P0.dhb - Pp.dhb), sdt1,
                 nd1 * q0f, nd1 * q1f, nu, xi, fa, fb);
            if (out_lane) {
                aFd.store(n, fa);
                bFd.store(n, n >= 1 ? fb : 0.0);
            }
        }
    };

    // R + 2 iterations, padded to a multiple of 6; padding iterations store
    // nothing.  A loaded fractional row stays live for five iterations, so a
    // body of six (two turns of the slot rotation) lets the register
    // assignment repeat without copies of loads in flight at the back edge.
    // The start-up loads land before the loop so that the wait counts at the
    // loop head are those of the steady state.
    const int jend = jlo + (r1 - jlo + 1 + 5) / 6 * 6;
    __builtin_amdgcn_s_waitcnt(0);
    for (int j = jlo; j < jend; j += 6) {
        iter(j, S[0], S[1], S[2]);
        iter(j + 1, S[1], S[2], S[0]);
        iter(j + 2, S[2], S[0], S[1]);
        iter(j + 3, S[0], S[1], S[2]);
        iter(j + 4, S[1], S[2], S[0]);
        iter(j + 5, S[2], S[0], S[1]);
    }
}

// ---- two steps per pass ------------------------------------------------------
// Registers of one slot (rows congruent mod 3) of the two-step pipeline.
struct Row2Regs {
    double f0a, f0b, f0da, f0db;   // old fractional grid z^{k+1/2}: own, phi_y differences
    double h1a, h1b, h1da, h1db;   // whole grid z^{k+1}: own, differences
    double f1a, f1b, f1da, f1db;   // fractional grid z^{k+3/2}: own, differences
    double h2da, h2db;             // whole grid z^{k+2}: differences
    double nfa, nfb, nha, nhb;     // loads in flight (old fractional row j+1, old whole row j)
};

// Two leap-frog steps in one pass over the state.  Iteration j of the march
// along the harmonics computes
//   W1: z^{k+1}   at harmonic j    (old fractional rows j-1, j+1; old whole row j)
//   F1: z^{k+3/2} at harmonic j-1  (z^{k+1} rows j-2, j; old fractional row j-1)
//   W2: z^{k+2}   at harmonic j-2  (z^{k+3/2} rows j-3, j-1; z^{k+1} row j-2)
//   F2: z^{k+5/2} at harmonic j-3  (z^{k+2} rows j-4, j-2; z^{k+3/2} row j-3)
// and writes z^{k+2} and z^{k+5/2}: the state is read and written once per two
// steps.  Every quantity a later stage needs lives in the slot of its row mod
// 3.  The tile keeps four halo lanes and three or four halo harmonics on each
// side; each stage is valid one lane further in, and the 56 lanes 4..59 hold
// outputs.  Per cell the arithmetic is exactly that of the one-step kernel.
// Operator T with nu^2 supplied (constant over the grid).
__device__ __forceinline__ void op_T2(double a, double b, double At, double Bt, double a0h,
                                      double mu0, double mu1, double nu, double nu2, double xi,
                                      double& an, double& bn)
{
    const double g = fma(a, xi, fma(-b, mu0, Bt + a0h));
    const double hh = fma(b, xi, fma(a, mu0, At));
    const double inv = recip(fma(mu1, mu1, nu2));
    an = fma(g, nu, -hh * mu1) * inv;
    bn = fma(g, mu1, hh * nu) * inv;
}

// Two leap-frog steps on one tile.  `s_tab` is this wave's 64-double slice of
// LDS: the source coefficients s_n of the tile's harmonics, read with a
// wave-uniform index (an LDS broadcast, no vector ALU work).
template <typename T>
__device__ __forceinline__ void fused2_tile(const TileEnv<T>& A, int tile, double* s_tab)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    // Tile order: groups of `cgroup` neighbouring phi_y strips (the waves of
    // one block) of one harmonic chunk, then the next chunk of the same
    // strips, then the next group.  The waves of a block march in step over
    // neighbouring strips, so the halo columns they share are read once from
    // L2; the chunks of a group follow each other closely, so the halo
    // harmonics neighbouring chunks share are too.
    const int ncol_tiles = (cs.ny + kFused2Cols - 1) / kFused2Cols;
    const int cg = A.cgroup;
    const int within = tile % cg;
    const int rest = tile / cg;
    const int chunk = rest % A.nchunks;
    const int ct = (rest / A.nchunks) * cg + within;
    if (ct >= ncol_tiles) return;                     // padding of the last group
    const int r0 = chunk * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kFused2Cols - 4 + lane;
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 4) && (lane < kWave - 4) && col_ok;

    const int64_t k = A.k;
    // cos(omega t) at the half-step times 2k .. 2k+5, lane i holds time 2k+i
    double cw[6];
    {
        const double t = static_cast<double>(2 * k + min(lane, 5)) * cs.half_dt;
        const double v = cos(cs.omega * t);
#pragma unroll
        for (int i = 0; i < 6; ++i) cw[i] = __shfl(v, i);
    }
    const bool acc1 = A.acc1;
    const bool acc2 = A.acc2;

    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gdt = (col_ok ? A.g_m[m] : 0.0) * cs.dt;
    const double hdt = 0.5 * cs.dt;
    double q[6];                                      // (E(t_i) + B phi) dt/2
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = (fma(cs.E_w, cw[i], cs.E_dc) + cs.B * phi) * hdt;
    const double c = cs.c_full, nu = cs.nu, xi = cs.xi, nu2 = cs.nu * cs.nu;
    // s_n of harmonics r0-3 .. r0+60, one per lane; a0 dt = s_n (g_m dt) as
    // in the other kernel forms
    const int sbase = r0 - 3;
    s_tab[lane] = A.s_n[min(max(sbase + lane, 0), cs.nx - 1)];
    __builtin_amdgcn_wave_barrier();
    auto a0dt = [&](int n) { return s_tab[min(max(n - sbase, 0), kWave - 1)] * gdt; };

    const uint32_t rb = static_cast<uint32_t>(cs.ld) * sizeof(T);
    const uint32_t cb = static_cast<uint32_t>(m + kPadCols) * sizeof(T);
    const uint32_t pb = static_cast<uint32_t>(cs.nx + 2 * kPadRows) * rb;
    const uint32_t ss = plane_stride(A.src), sd = plane_stride(A.dst);
    const RowAddr<T> aHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 0);
    const RowAddr<T> bHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, ss);
    const RowAddr<T> aFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 2 * ss);
    const RowAddr<T> bFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 3 * ss);
    const RowAddr<T> aHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 0 + A.salt), 0);
    const RowAddr<T> bHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 1 + A.salt), sd);
    const RowAddr<T> aFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 2 + A.salt), 2 * sd);
    const RowAddr<T> bFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 3 + A.salt), 3 * sd);

    const int jlo = r0 - 3;                           // first W1 row
    const int jhi = r1 + 2;                           // last W1 row
    // A tile is "interior" when every row its stages compute is a harmonic
    // >= 2 inside the grid and every lane a phi_y column inside the box: no
    // boundary masks, chi = 1 and no b_0 row.
    const bool interior = (jlo >= 2) && (jhi < cs.nx) && (ct > 0) && (ct < ncol_tiles - 1) &&
                          (ct * kFused2Cols - 4 >= 0) && (ct * kFused2Cols + kWave - 5 < cs.ny);

    // The march over the harmonics alternates direction from one chunk to the
    // next (even chunks upward in n, odd chunks downward), so that the halo
    // harmonics two neighbouring chunks share are read by both at about the
    // same time and the second read hits in L2.  Stage rows move with the
    // direction D: W1 at j, F1 at j - D, W2 at j - 2D, F2 at j - 3D.
    auto run = [&](auto edge_tag, auto dir_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        constexpr int D = decltype(dir_tag)::value;
        auto valid = [&](int n) { return (n >= 0) && (n < cs.nx) && col_ok; };
        // coupling terms of Sec. 3 from the other grid's phi_y differences
        // at harmonics n-1 (lo) and n+1 (hi): A = c (chi lo_a - hi_a),
        // B = c (hi_b - lo_b).  Slot "behind" holds row n - D, "ahead" n + D.
        auto coupling = [&](int n, double behind_a, double ahead_a, double behind_b,
                            double ahead_b, double& At, double& Bt) {
            const double lo_a = D > 0 ? behind_a : ahead_a, hi_a = D > 0 ? ahead_a : behind_a;
            const double lo_b = D > 0 ? behind_b : ahead_b, hi_b = D > 0 ? ahead_b : behind_b;
            if constexpr (EDGE)
                At = c * ((n == 1 ? 2.0 * lo_a : lo_a) - hi_a);
            else
                At = c * (lo_a - hi_a);
            Bt = c * (hi_b - lo_b);
        };
        auto mask = [&](int n, double& a, double& b) {
            if constexpr (EDGE) {
                const bool v = valid(n);
                a = v ? a : 0.0;
                b = (v && n >= 1) ? b : 0.0;
            }
        };

        const int jfirst = D > 0 ? jlo : jhi;         // first W1 row of the march
        Row2Regs S[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) S[i] = Row2Regs{};
        auto issue = [&](Row2Regs& P, int j) {
            const int jf = min(max(j + D, r0 - 4), r1 + 3);
            const int jh = min(max(j, jlo), jhi);
            P.nfa = aFs.load(jf);
            P.nfb = bFs.load(jf);
            P.nha = aHs.load(jh);
            P.nhb = bHs.load(jh);
        };
        {
            Row2Regs& a = S[0];                       // slot of jfirst - D
            a.f0a = aFs.load(jfirst - D);
            a.f0b = bFs.load(jfirst - D);
            Row2Regs& b = S[1];                       // slot of jfirst
            b.f0a = aFs.load(jfirst);
            b.f0b = bFs.load(jfirst);
            issue(S[1], jfirst);
            issue(S[2], jfirst + D);
            issue(S[0], jfirst + 2 * D);
            a.f0da = dphi_diff(a.f0a);
            a.f0db = dphi_diff(a.f0b);
            b.f0da = dphi_diff(b.f0a);
            b.f0db = dphi_diff(b.f0b);
        }

        // Pm: slot of row j - D, P0: row j, Pp: row j + D (= j - 2D mod 3)
        auto iter = [&](int j, Row2Regs& Pm, Row2Regs& P0, Row2Regs& Pp) {
            // inputs loaded three iterations ago
            Pp.f0a = P0.nfa;
            Pp.f0b = P0.nfb;
            const double ha0 = P0.nha, hb0 = P0.nhb;
            issue(P0, j + 3 * D);
            Pp.f0da = dphi_diff(Pp.f0a);
            Pp.f0db = dphi_diff(Pp.f0b);

            // W1: whole grid k -> k+1 at harmonic j
            {
                const double nd = static_cast<double>(j);
                double At, Bt, ha, hb;
                coupling(j, Pm.f0da, Pp.f0da, Pm.f0db, Pp.f0db, At, Bt);
                op_T2(ha0, hb0, At, Bt, a0dt(j), nd * q[0], nd * q[2], nu, nu2, xi, ha, hb);
                mask(j, ha, hb);
                P0.h1a = ha;
                P0.h1b = hb;
                P0.h1da = dphi_diff(ha);
                P0.h1db = dphi_diff(hb);
                if constexpr (EDGE) {
                    if (j == 1 && j >= r0 && j < r1 && out_lane && acc1) {
                        A.acc_v[m] += hb;
                        A.acc_vc[m] += hb * cw[2];
                    }
                }
            }
            // F1: fractional grid k+1/2 -> k+3/2 at harmonic j - D
            {
                const int n = j - D;
                const double nd = static_cast<double>(n);
                double At, Bt, fa, fb;
                // z^{k+1} at n - D = j - 2D (slot Pp) and n + D = j (slot P0)
                coupling(n, Pp.h1da, P0.h1da, Pp.h1db, P0.h1db, At, Bt);
                op_T2(Pm.f0a, Pm.f0b, At, Bt, a0dt(n), nd * q[1], nd * q[3], nu, nu2, xi, fa, fb);
                mask(n, fa, fb);
                Pm.f1a = fa;
                Pm.f1b = fb;
                Pm.f1da = dphi_diff(fa);
                Pm.f1db = dphi_diff(fb);
            }
            // W2: whole grid k+1 -> k+2 at harmonic j - 2D
            {
                const int n = j - 2 * D;
                const double nd = static_cast<double>(n);
                double At, Bt, ha, hb;
                // z^{k+3/2} at n - D = j - 3D (slot P0) and n + D = j - D (slot Pm)
                coupling(n, P0.f1da, Pm.f1da, P0.f1db, Pm.f1db, At, Bt);
                op_T2(Pp.h1a, Pp.h1b, At, Bt, a0dt(n), nd * q[2], nd * q[4], nu, nu2, xi, ha, hb);
                mask(n, ha, hb);
                Pp.h2da = dphi_diff(ha);
                Pp.h2db = dphi_diff(hb);
                if (n >= r0 && n < r1 && out_lane) {
                    aHd.store(n, ha);
                    bHd.store(n, hb);
                    if constexpr (EDGE) {
                        if (n == 1 && acc2) {
                            A.acc_v[m] += hb;
                            A.acc_vc[m] += hb * cw[4];
                        }
                    }
                }
            }
            // F2: fractional grid k+3/2 -> k+5/2 at harmonic j - 3D
            {
                const int n = j - 3 * D;
                if (n >= r0 && n < r1) {
                    const double nd = static_cast<double>(n);
                    double At, Bt, fa, fb;
                    // z^{k+2} at n - D = j - 4D (slot Pm) and n + D = j - 2D (slot Pp)
                    coupling(n, Pm.h2da, Pp.h2da, Pm.h2db, Pp.h2db, At, Bt);
                    op_T2(P0.f1a, P0.f1b, At, Bt, a0dt(n), nd * q[3], nd * q[5], nu, nu2, xi, fa, fb);
                    if (out_lane) {
                        aFd.store(n, fa);
                        bFd.store(n, (!EDGE || n >= 1) ? fb : 0.0);
                    }
                }
            }
        };

        // W1 rows jlo .. jhi (R + 6 iterations), padded to a multiple of 6;
        // padding iterations store nothing.  A loaded row stays live for five
        // iterations, so a body of six (two turns of the slot rotation) lets
        // the register assignment repeat without copies of rows still in
        // flight at the loop's back edge (a copy would wait for the load).
        const int iters = (jhi - jlo + 1 + 5) / 6 * 6;
        // Let the start-up loads land before the loop: otherwise the wait
        // counts at the loop head are those of the entry path (few younger
        // operations in flight) on every turn, and each turn drains the
        // memory pipeline.
        __builtin_amdgcn_s_waitcnt(0);
        for (int i = 0; i < iters; i += 6) {
            if (A.even_progress) march_priority(i, iters);
            const int j = jfirst + D * i;
            iter(j, S[0], S[1], S[2]);
            iter(j + D, S[1], S[2], S[0]);
            iter(j + 2 * D, S[2], S[0], S[1]);
            iter(j + 3 * D, S[0], S[1], S[2]);
            iter(j + 4 * D, S[1], S[2], S[0]);
            iter(j + 5 * D, S[2], S[0], S[1]);
        }
    };
    using Up = std::integral_constant<int, 1>;
    using Down = std::integral_constant<int, -1>;
    const bool up = (chunk & 1) == 0;
    if (interior) {
        if (up) run(std::false_type{}, Up{});
        else run(std::false_type{}, Down{});
    } else {
        if (up) run(std::true_type{}, Up{});
        else run(std::true_type{}, Down{});
    }
}

// ---- three steps per pass ----------------------------------------------------
// Registers of one slot (rows congruent mod 3) of the three-step pipeline.
struct Row3Regs {
    double f0a, f0b, f0da, f0db;   // old fractional grid z^{k+1/2}: own, phi_y differences
    double h1a, h1b, h1da, h1db;   // whole grid z^{k+1}
    double f1a, f1b, f1da, f1db;   // fractional grid z^{k+3/2}
    double h2a, h2b, h2da, h2db;   // whole grid z^{k+2}
    double f2a, f2b, f2da, f2db;   // fractional grid z^{k+5/2}
    double h3da, h3db;             // whole grid z^{k+3}: differences
    double nfa, nfb, nha, nhb;     // loads in flight (old fractional row j+D, old whole row j)
};

// Three leap-frog steps in one pass over the state: the two-step pipeline
// extended by two more stages.  Iteration j of the march computes
//   W1: z^{k+1} at j,  F1: z^{k+3/2} at j-D,  W2: z^{k+2} at j-2D,
//   F2: z^{k+5/2} at j-3D,  W3: z^{k+3} at j-4D,  F3: z^{k+7/2} at j-5D
// (D = +1 or -1, the march direction) and writes z^{k+3} and z^{k+7/2}: the
// state is read and written once per three steps.  Each stage is valid one
// lane further in, so a tile keeps six halo lanes on each side (52 output
// lanes, 6..57) and five or six halo harmonics.  Per cell the arithmetic is
// exactly that of the one-step kernel.
template <typename T>
__device__ __forceinline__ void fused3_tile(const TileEnv<T>& A, int tile, double* s_tab)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    // tile order as in fused2_tile: column groups of `cgroup` strips
    const int ncol_tiles = (cs.ny + kFused3Cols - 1) / kFused3Cols;
    const int cg = A.cgroup;
    const int within = tile % cg;
    const int rest = tile / cg;
    const int chunk = rest % A.nchunks;
    const int ct = (rest / A.nchunks) * cg + within;
    if (ct >= ncol_tiles) return;                     // padding of the last group
    const int r0 = chunk * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kFused3Cols - 6 + lane;
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 6) && (lane < kWave - 6) && col_ok;

    const int64_t k = A.k;
    // cos(omega t) at the half-step times 2k .. 2k+7, lane i holds time 2k+i
    double cw[8];
    {
        const double t = static_cast<double>(2 * k + min(lane, 7)) * cs.half_dt;
        const double v = cos(cs.omega * t);
#pragma unroll
        for (int i = 0; i < 8; ++i) cw[i] = __shfl(v, i);
    }
    const bool acc1 = A.acc1, acc2 = A.acc2, acc3 = A.acc3;

    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gdt = (col_ok ? A.g_m[m] : 0.0) * cs.dt;
    const double hdt = 0.5 * cs.dt;
    double q[8];                                      // (E(t_i) + B phi) dt/2
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = (fma(cs.E_w, cw[i], cs.E_dc) + cs.B * phi) * hdt;
    const double c = cs.c_full, nu = cs.nu, xi = cs.xi, nu2 = cs.nu * cs.nu;
    // s_n of harmonics r0-5 .. r0+58, one per lane
    const int sbase = r0 - 5;
    s_tab[lane] = A.s_n[min(max(sbase + lane, 0), cs.nx - 1)];
    __builtin_amdgcn_wave_barrier();
    auto a0dt = [&](int n) { return s_tab[min(max(n - sbase, 0), kWave - 1)] * gdt; };

    const uint32_t rb = static_cast<uint32_t>(cs.ld) * sizeof(T);
    // the two leftmost halo lanes of the first column tile lie left of the
    // zero border: they read its outermost (zero) column
    const uint32_t cb = static_cast<uint32_t>(max(m, -kPadCols) + kPadCols) * sizeof(T);
    const uint32_t pb = static_cast<uint32_t>(cs.nx + 2 * kPadRows) * rb;
    const uint32_t ss = plane_stride(A.src), sd = plane_stride(A.dst);
    const RowAddr<T> aHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 0);
    const RowAddr<T> bHs(A.src.a_h, 3 * ss + pb, rb, cb, 0, ss);
    const RowAddr<T> aFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 2 * ss);
    const RowAddr<T> bFs(A.src.a_h, 3 * ss + pb, rb, cb, 0, 3 * ss);
    const RowAddr<T> aHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 0 + A.salt), 0);
    const RowAddr<T> bHd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 1 + A.salt), sd);
    const RowAddr<T> aFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 2 + A.salt), 2 * sd);
    const RowAddr<T> bFd(A.dst.a_h, 3 * sd + pb, rb, cb, plane_seed(k, 3 + A.salt), 3 * sd);
    // rows beyond the zero border read its outermost (zero) row
    const int rmin = -kPadRows, rmax = cs.nx + kPadRows - 1;

    const int jlo = r0 - 5;                           // first W1 row
    const int jhi = r1 + 4;                           // last W1 row
    // interior: every stage row a harmonic >= 2 inside the grid and every
    // lane a phi_y column inside the box (no masks, chi = 1, no b_0 row)
    const bool interior = (jlo >= 2) && (jhi < cs.nx) && (ct * kFused3Cols - 6 >= 0) &&
                          (ct * kFused3Cols - 6 + kWave - 1 < cs.ny);

    auto run = [&](auto edge_tag, auto dir_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        constexpr int D = decltype(dir_tag)::value;
        auto valid = [&](int n) { return (n >= 0) && (n < cs.nx) && col_ok; };
        auto coupling = [&](int n, double behind_a, double ahead_a, double behind_b,
                            double ahead_b, double& At, double& Bt) {
            const double lo_a = D > 0 ? behind_a : ahead_a, hi_a = D > 0 ? ahead_a : behind_a;
            const double lo_b = D > 0 ? behind_b : ahead_b, hi_b = D > 0 ? ahead_b : behind_b;
            if constexpr (EDGE)
                At = c * ((n == 1 ? 2.0 * lo_a : lo_a) - hi_a);
            else
                At = c * (lo_a - hi_a);
            Bt = c * (hi_b - lo_b);
        };
        auto mask = [&](int n, double& a, double& b) {
            if constexpr (EDGE) {
                const bool v = valid(n);
                a = v ? a : 0.0;
                b = (v && n >= 1) ? b : 0.0;
            }
        };
        auto accumulate = [&](int n, double hb, double cwt, bool on) {
            if constexpr (EDGE) {
                if (n == 1 && n >= r0 && n < r1 && out_lane && on) {
                    A.acc_v[m] += hb;
                    A.acc_vc[m] += hb * cwt;
                }
            }
        };

        const int jfirst = D > 0 ? jlo : jhi;
        Row3Regs S[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) S[i] = Row3Regs{};
        auto issue = [&](Row3Regs& P, int j) {
            const int jf = min(max(min(max(j + D, r0 - 6), r1 + 5), rmin), rmax);
            const int jh = min(max(min(max(j, jlo), jhi), rmin), rmax);
            P.nfa = aFs.load(jf);
            P.nfb = bFs.load(jf);
            P.nha = aHs.load(jh);
            P.nhb = bHs.load(jh);
        };
        {
            const int j0 = min(max(jfirst - D, rmin), rmax);
            const int j1 = min(max(jfirst, rmin), rmax);
            Row3Regs& a = S[0];                       // slot of jfirst - D
            a.f0a = aFs.load(j0);
            a.f0b = bFs.load(j0);
            Row3Regs& b = S[1];                       // slot of jfirst
            b.f0a = aFs.load(j1);
            b.f0b = bFs.load(j1);
            issue(S[1], jfirst);
            issue(S[2], jfirst + D);
            issue(S[0], jfirst + 2 * D);
            a.f0da = dphi_diff(a.f0a);
            a.f0db = dphi_diff(a.f0b);
            b.f0da = dphi_diff(b.f0a);
            b.f0db = dphi_diff(b.f0b);
        }

        // Pm: slot of row j - D, P0: row j, Pp: row j + D.  Rows j - 2D and
        // j - 5D share Pp's slot, j - 3D shares P0's, j - 4D shares Pm's.
        auto iter = [&](int j, Row3Regs& Pm, Row3Regs& P0, Row3Regs& Pp) {
            Pp.f0a = P0.nfa;
            Pp.f0b = P0.nfb;
            const double ha0 = P0.nha, hb0 = P0.nhb;
            issue(P0, j + 3 * D);
            Pp.f0da = dphi_diff(Pp.f0a);
            Pp.f0db = dphi_diff(Pp.f0b);
            // W1: z^{k+1} at j (old fractional rows j -+ D in Pm, Pp)
            {
                const double nd = static_cast<double>(j);
                double At, Bt, ha, hb;
                coupling(j, Pm.f0da, Pp.f0da, Pm.f0db, Pp.f0db, At, Bt);
                op_T2(ha0, hb0, At, Bt, a0dt(j), nd * q[0], nd * q[2], nu, nu2, xi, ha, hb);
                mask(j, ha, hb);
                P0.h1a = ha;
                P0.h1b = hb;
                P0.h1da = dphi_diff(ha);
                P0.h1db = dphi_diff(hb);
                accumulate(j, hb, cw[2], acc1);
            }
            // F1: z^{k+3/2} at j - D (z^{k+1} at j - 2D in Pp, j in P0)
            {
                const int n = j - D;
                const double nd = static_cast<double>(n);
                double At, Bt, fa, fb;
                coupling(n, Pp.h1da, P0.h1da, Pp.h1db, P0.h1db, At, Bt);
                op_T2(Pm.f0a, Pm.f0b, At, Bt, a0dt(n), nd * q[1], nd * q[3], nu, nu2, xi, fa, fb);
                mask(n, fa, fb);
                Pm.f1a = fa;
                Pm.f1b = fb;
                Pm.f1da = dphi_diff(fa);
                Pm.f1db = dphi_diff(fb);
            }
            // W2: z^{k+2} at j - 2D (z^{k+3/2} at j - 3D in P0, j - D in Pm)
            {
                const int n = j - 2 * D;
                const double nd = static_cast<double>(n);
                double At, Bt, ha, hb;
                coupling(n, P0.f1da, Pm.f1da, P0.f1db, Pm.f1db, At, Bt);
                op_T2(Pp.h1a, Pp.h1b, At, Bt, a0dt(n), nd * q[2], nd * q[4], nu, nu2, xi, ha, hb);
                mask(n, ha, hb);
                Pp.h2a = ha;
                Pp.h2b = hb;
                Pp.h2da = dphi_diff(ha);
                Pp.h2db = dphi_diff(hb);
                accumulate(n, hb, cw[4], acc2);
            }
            // F2: z^{k+5/2} at j - 3D (z^{k+2} at j - 4D in Pm, j - 2D in Pp)
            {
                const int n = j - 3 * D;
                const double nd = static_cast<double>(n);
                double At, Bt, fa, fb;
                coupling(n, Pm.h2da, Pp.h2da, Pm.h2db, Pp.h2db, At, Bt);
                op_T2(P0.f1a, P0.f1b, At, Bt, a0dt(n), nd * q[3], nd * q[5], nu, nu2, xi, fa, fb);
                mask(n, fa, fb);
                P0.f2a = fa;
                P0.f2b = fb;
                P0.f2da = dphi_diff(fa);
                P0.f2db = dphi_diff(fb);
            }
            // W3: z^{k+3} at j - 4D (z^{k+5/2} at j - 5D in Pp, j - 3D in P0)
            {
                const int n = j - 4 * D;
                const double nd = static_cast<double>(n);
                double At, Bt, ha, hb;
                coupling(n, Pp.f2da, P0.f2da, Pp.f2db, P0.f2db, At, Bt);
                op_T2(Pm.h2a, Pm.h2b, At, Bt, a0dt(n), nd * q[4], nd * q[6], nu, nu2, xi, ha, hb);
                mask(n, ha, hb);
                Pm.h3da = dphi_diff(ha);
                Pm.h3db = dphi_diff(hb);
                if (n >= r0 && n < r1 && out_lane) {
                    aHd.store(n, ha);
                    bHd.store(n, hb);
                }
                accumulate(n, hb, cw[6], acc3);
            }
            // F3: z^{k+7/2} at j - 5D (z^{k+3} at j - 6D in P0, j - 4D in Pm)
            {
                const int n = j - 5 * D;
                if (n >= r0 && n < r1) {
                    const double nd = static_cast<double>(n);
                    double At, Bt, fa, fb;
                    coupling(n, P0.h3da, Pm.h3da, P0.h3db, Pm.h3db, At, Bt);
                    op_T2(Pp.f2a, Pp.f2b, At, Bt, a0dt(n), nd * q[5], nd * q[7], nu, nu2, xi, fa, fb);
                    if (out_lane) {
                        aFd.store(n, fa);
                        bFd.store(n, (!EDGE || n >= 1) ? fb : 0.0);
                    }
                }
            }
        };

        // W1 rows jlo .. jhi (R + 10 iterations), padded to a multiple of 6 (a
        // loaded row lives five iterations; see fused2_tile)
        const int iters = (jhi - jlo + 1 + 5) / 6 * 6;
        __builtin_amdgcn_s_waitcnt(0);
        for (int i = 0; i < iters; i += 6) {
            if (A.even_progress) march_priority(i, iters);
            const int j = jfirst + D * i;
            iter(j, S[0], S[1], S[2]);
            iter(j + D, S[1], S[2], S[0]);
            iter(j + 2 * D, S[2], S[0], S[1]);
            iter(j + 3 * D, S[0], S[1], S[2]);
            iter(j + 4 * D, S[1], S[2], S[0]);
            iter(j + 5 * D, S[2], S[0], S[1]);
        }
    };
    using Up = std::integral_constant<int, 1>;
    using Down = std::integral_constant<int, -1>;
    const bool up = (chunk & 1) == 0;
    if (interior) {
        if (up) run(std::false_type{}, Up{});
        else run(std::false_type{}, Down{});
    } else {
        if (up) run(std::true_type{}, Up{});
        else run(std::true_type{}, Down{});
    }
}

// One half-step of the paper's two-kernel structure, in place on X (a cell of
// X reads only its own old value; all neighbour reads hit Y).
template <typename T>
__device__ __forceinline__ void half_tile(const HalfEnv<T>& A, int tile)
{
    const Consts& cs = A.cs;
    const int lane = threadIdx.x & (kWave - 1);
    const int ct = tile / A.nchunks;
    const int r0 = (tile - ct * A.nchunks) * A.R;
    const int r1 = min(r0 + A.R, cs.nx);
    const int m = ct * kHalfCols - 1 + lane;
    const bool col_ok = (m >= 0) && (m < cs.ny);
    const bool out_lane = (lane >= 1) && (lane < kWave - 1) && col_ok;

    const int64_t k = A.k;
    const int lane_off = (lane & 1) ? A.off1 : A.off0;
    const double tt = static_cast<double>(2 * k + lane_off) * cs.half_dt;
    const double cv = cos(cs.omega * tt);
    const double c0 = __shfl(cv, 0), c1 = __shfl(cv, 1);
    const bool acc_step = A.acc1;
    const double cw_acc = acc_step ? cos(cs.omega * static_cast<double>(2 * k + 2) * cs.half_dt) : 0.0;

    const double h = A.h;
    const double nu = 1.0 + 0.5 * h, xi = 1.0 - 0.5 * h;
    const double c = cs.B * h / (4.0 * cs.dphi);
    const double phi = fma(static_cast<double>(m), cs.dphi, cs.phimin);
    const double gh = (col_ok ? A.g_m[m] : 0.0) * h;
    const double s_lane = A.s_n[min(r0 + lane, cs.nx - 1)];   // harmonics r0 .. r1-1
    const double q0 = (fma(cs.E_w, c0, cs.E_dc) + cs.B * phi) * (0.5 * h);
    const double q1 = (fma(cs.E_w, c1, cs.E_dc) + cs.B * phi) * (0.5 * h);

    const uint32_t rb = static_cast<uint32_t>(cs.ld) * sizeof(T);
    const uint32_t cb = static_cast<uint32_t>(m + kPadCols) * sizeof(T);
    const uint32_t pb = static_cast<uint32_t>(cs.nx + 2 * kPadRows) * rb;
    // distinct per half-step kind: start-up (0,1), whole (0,2), fractional (1,3)
    const uint32_t tag = 4u + 2u * static_cast<uint32_t>(A.off0 + A.off1);
    const RowAddr<T> xa(A.xa, pb, rb, cb, plane_seed(k, tag + A.salt));
    const RowAddr<T> xb(A.xb, pb, rb, cb, plane_seed(k, tag + 1 + A.salt));
    const RowAddr<T> ya(A.ya, pb, rb, cb);
    const RowAddr<T> yb(A.yb, pb, rb, cb);

    // differences of Y for rows n-1 (0) and n (1); row n+1 loaded per iteration
    double da0 = dphi_diff(ya.load(r0 - 1)), db0 = dphi_diff(yb.load(r0 - 1));
    double da1 = dphi_diff(ya.load(r0)), db1 = dphi_diff(yb.load(r0));
    double pf_ya = ya.load(r0 + 1), pf_yb = yb.load(r0 + 1);
    double pf_xa = xa.load(r0), pf_xb = xb.load(r0);

    for (int n = r0; n < r1; ++n) {
        const double da2 = dphi_diff(pf_ya), db2 = dphi_diff(pf_yb);
        const double a = pf_xa, b = pf_xb;
        {
            const int jn = min(n + 2, r1);
            pf_ya = ya.load(jn);
            pf_yb = yb.load(jn);
            const int jx = min(n + 1, r1 - 1);
            pf_xa = xa.load(jx);
            pf_xb = xb.load(jx);
        }
        const double chi = (n == 1) ? 2.0 : 1.0;
        const double nd = static_cast<double>(n);
        double an, bn;
        op_T(a, b, c * (chi * da0 - da2), c * (db2 - db0), lane_bcast(s_lane, n - r0) * gh, nd * q0, nd * q1, nu,
             xi, an, bn);
        if (out_lane) {
            xa.store(n, an);
            xb.store(n, n >= 1 ? bn : 0.0);
            if (n == 1 && acc_step) {
                A.acc_v[m] += bn;
                A.acc_vc[m] += bn * cw_acc;
            }
        }
        da0 = da1; db0 = db1;
        da1 = da2; db1 = db2;
    }
}

}  // namespace detail
}  // namespace bte
