// f(phi_x, phi_y) on a uniform phi_x grid from the Fourier state (Sec. 2,
// Eq. f_fourier):
//
//     f[j][m] = sum_{n < N_x} a_n(m) cos(n x_j) + b_n(m) sin(n x_j),
//     x_j = -pi + 2 pi j / M,  j = 0 .. M-1.
//
// This is a dense product F = T Z with T[j][k] the trigonometric matrix and
// Z[k][m] the coefficients, k = 2n for the cosine/a_n pair and 2n+1 for the
// sine/b_n pair (K = 2 N_x), so it runs on the FP64 matrix cores
// (16 x 16 x 4 instructions, FP64 products and sums).  The trigonometric
// operand is never stored: each lane produces its own entries of T.
//   - The A operand of an instruction is 16 samples j x 4 values of k; the
//     lane holding (j, k) carries e^{i n x_j} for its n = 2t + (k >> 1) and
//     advances it by the rotation e^{2 i x_j} per k step of 4 (4 FP64
//     operations on the vector unit, overlapping the matrix instructions),
//     reseeded exactly every 64 harmonics from the integer phase
//     (n j mod M) / M so that the rotation error stays near 64 ulp.
//   - The B operand (coefficients) is read straight from the state, 16
//     consecutive phi_y points per row, with the loads P steps ahead.
//   - A wavefront owns 16 TJ samples x 16 TM points; the four wavefronts of
//     a block share the points (the coefficient rows reach them through one
//     L1), and the blocks that share points are placed on the same XCD so
//     that one L2 holds their rows.
// Rows of the output are phi_x samples, columns phi_y points (phi_y
// contiguous, the state's own orientation).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bte_reconstruct.h"

namespace bte {

namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));

constexpr int kReconWaves = 4;
constexpr int kReseedSteps = 32;    // k steps of 4 = 64 harmonics
constexpr int kXcds = 8;

template <typename T, int TJ, int TM, int P>
__global__ __launch_bounds__(kReconWaves * 64) void k_reconstruct(const T* __restrict__ a,
                                                                   const T* __restrict__ b,
                                                                   int64_t ld, int nx, int ny,
                                                                   int M, int gx, int gy,
                                                                   double* __restrict__ out)
{
    // XCD-aware tile order: consecutive block ids go round-robin over the
    // XCDs, so block id -> (xcd = id mod 8, slot = id / 8) and each XCD takes
    // a contiguous run of tiles, in which the j tiles of one column tile are
    // adjacent.
    const int ntile = gx * gy;
    const int per_xcd = (ntile + kXcds - 1) / kXcds;
    const int id = blockIdx.x;
    const int tile = (id % kXcds) * per_xcd + id / kXcds;
    if (tile >= ntile) return;
    const int bx = tile / gy, by = tile % gy;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r16 = lane & 15;
    const int q = lane >> 4;                 // k offset inside an instruction
    const int half = q >> 1;                 // n = 2t + half
    const bool is_sin = (q & 1) != 0;        // odd k: sine / b_n
    const int m0 = bx * (16 * TM);
    const int jw = (by * kReconWaves + wave) * (16 * TJ);

    int jj[TJ];
    double c[TJ], s[TJ], c2[TJ], s2[TJ];
#pragma unroll
    for (int i = 0; i < TJ; ++i) {
        const int j = jw + 16 * i + r16;
        jj[i] = j < M ? j : M - 1;           // rows past the end shadow the last sample
        // rotation by 2 x_j = -2 pi + 2 pi (2 j) / M
        const int64_t p2 = (2 * static_cast<int64_t>(jj[i])) % M;
        sincospi(2.0 * static_cast<double>(p2) / static_cast<double>(M), &s2[i], &c2[i]);
        c[i] = 0.0;
        s[i] = 0.0;
    }
    const T* src = is_sin ? b : a;
    int64_t col[TM];
#pragma unroll
    for (int u = 0; u < TM; ++u) {
        const int m = m0 + 16 * u + r16;
        col[u] = m < ny ? m : ny - 1;
    }
    // Coefficient of k step t (rows n = 2t + half), with the guards: rows
    // past N_x and b_0 (not part of the series) give 0 and are not read.
    auto coef = [&](int t, int u) -> double {
        const int n = 2 * t + half;
        if (n >= nx || (is_sin && n == 0)) return 0.0;
        return static_cast<double>(src[n * ld + col[u]]);
    };

    f64x4 acc[TJ][TM];
#pragma unroll
    for (int i = 0; i < TJ; ++i)
#pragma unroll
        for (int u = 0; u < TM; ++u) acc[i][u] = f64x4{0.0, 0.0, 0.0, 0.0};

    auto reseed = [&](int t) {
        const int n = 2 * t + half;
#pragma unroll
        for (int i = 0; i < TJ; ++i) {
            const int64_t k = (static_cast<int64_t>(n) * jj[i]) % M;
            double ss, cc;
            sincospi(2.0 * static_cast<double>(k) / static_cast<double>(M), &ss, &cc);
            const double sg = (n & 1) ? -1.0 : 1.0;   // n x_j = -n pi + 2 pi n j / M
            c[i] = sg * cc;
            s[i] = sg * ss;
        }
    };
    auto mma_rotate = [&](const double (&z)[TM]) {
#pragma unroll
        for (int i = 0; i < TJ; ++i) {
            const double av = is_sin ? s[i] : c[i];
#pragma unroll
            for (int u = 0; u < TM; ++u)
                acc[i][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, z[u], acc[i][u], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < TJ; ++i) {
            const double cn = fma(c[i], c2[i], -s[i] * s2[i]);
            const double sn = fma(s[i], c2[i], c[i] * s2[i]);
            c[i] = cn;
            s[i] = sn;
        }
    };

    // Steps 0 .. P-1 are fetched with guards.  In the main loop every row a
    // prefetch touches exists (2 (t + P) + 1 < N_x), so its loads go out
    // unconditionally, P steps ahead, through pointers that advance two rows
    // per step.  The last steps use what is left in the ring, then load
    // directly.
    const int nsteps = (nx + 1) / 2;
    const int full = nx / 2;                 // steps whose two rows both exist
    static_assert(kReseedSteps % P == 0, "reseeds fall on ring starts");
    double zb[P][TM];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < TM; ++u) zb[p][u] = coef(p, u);
    int64_t idx[TM];
#pragma unroll
    for (int u = 0; u < TM; ++u) idx[u] = (2 * P + half) * ld + col[u];
    const int64_t adv = 2 * ld;
    int t0 = 0;
    for (; t0 + 2 * P <= full; t0 += P) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (p == 0 && t0 % kReseedSteps == 0) reseed(t0);   // t0 is a multiple of P
            mma_rotate(zb[p]);
#pragma unroll
            for (int u = 0; u < TM; ++u) {
                zb[p][u] = static_cast<double>(src[idx[u]]);
                idx[u] += adv;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int t = t0 + p;
        if (t < nsteps) {
            if (p == 0 && t % kReseedSteps == 0) reseed(t);
            mma_rotate(zb[p]);
        }
    }
    for (int t = t0 + P; t < nsteps; ++t) {
        double z[TM];
#pragma unroll
        for (int u = 0; u < TM; ++u) z[u] = coef(t, u);
        if (t % kReseedSteps == 0) reseed(t);
        mma_rotate(z);
    }

    // accumulator of lane l: rows (l / 16) + 4 e, e = 0..3, of column l mod 16
    // (the FP64 16 x 16 x 4 layout)
#pragma unroll
    for (int i = 0; i < TJ; ++i) {
#pragma unroll
        for (int u = 0; u < TM; ++u) {
            const int m = m0 + 16 * u + r16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = jw + 16 * i + q + 4 * e;
                if (j < M && m < ny) out[static_cast<int64_t>(j) * ny + m] = acc[i][u][e];
            }
        }
    }
}

}  // namespace

template <typename T, int TJ, int TM, int P>
hipError_t launch_shape(hipStream_t stream, const T* a, const T* b, int64_t ld, int nx, int ny,
                        int M, double* out)
{
    const int gx = (ny + 16 * TM - 1) / (16 * TM);
    const int gy = (M + kReconWaves * 16 * TJ - 1) / (kReconWaves * 16 * TJ);
    const int64_t ntile = static_cast<int64_t>(gx) * gy;
    if (ntile > (int64_t{1} << 30)) return hipErrorInvalidValue;
    const int per_xcd = static_cast<int>((ntile + kXcds - 1) / kXcds);
    k_reconstruct<T, TJ, TM, P><<<per_xcd * kXcds, kReconWaves * 64, 0, stream>>>(
        a, b, ld, nx, ny, M, gx, gy, out);
    return hipGetLastError();
}

// Tile shapes by measurement at 512 harmonics x 8193 points: one 16-sample
// row of instructions per wavefront (more rows cost occupancy); 32 points
// with loads 8 steps ahead up to ~768 samples (43.6 TFLOP/s at 512), 64
// points 4 steps ahead beyond (50.1 TFLOP/s at 1024).
// ---- power-of-two sample counts: one FFT per phi_y column ------------------------
// With x_j = -pi + 2 pi j / M, e^{i n x_j} = (-1)^n w^{n j}, w = e^{2 pi i / M},
// so f[j][m] = Re sum_k C_k(m) w^{j k} with the folded coefficients
//     C_k(m) = sum_{n < N_x, n = k mod M} (-1)^n (a_n(m) - i b_n(m)),
// an inverse DFT of length M per column.  f is real, so two columns share one
// complex transform: with H_k = (C_k + conj(C_{-k})) / 2 (the Hermitian part,
// whose transform is Re of C's), the transform of H(m) + i H(m') is
// f(m) + i f(m').  A workgroup owns 2P consecutive columns (P pairs; P = 8
// up to M = 256, then 4 and 2, so that the sequences and the twiddles stay
// within 64 KiB of LDS): it builds the P sequences in LDS in bit-reversed
// order, runs log2 M radix-2 decimation-in-time stages over them with a
// shared twiddle table (each stage's e^{2 pi i t / 2^s} contiguous, sincospi
// of an exact fraction), and writes each sample row as 2P consecutive
// doubles.  O(M log M) work per column instead of O(M N_x); each coefficient
// row is read once per column group, the groups sharing cache lines run on
// one XCD, and the output is written once.
constexpr int kFftThreads = 256;
constexpr int kFftMaxM = 1024;

__device__ __forceinline__ int bit_reverse(int k, int bits)
{
    return static_cast<int>(__builtin_bitreverse32(static_cast<uint32_t>(k)) >> (32 - bits));
}

// LDS position of entry i of a sequence: one 16-byte gap after every 8
// entries, so that entries a multiple of 8 apart (the bit-reversed stores, the
// early butterfly stages) fall in different banks.
__device__ __forceinline__ int fft_pad(int i) { return i + (i >> 3); }

template <typename T, int kFftPairs>
__global__ __launch_bounds__(kFftThreads) void k_reconstruct_fft(const T* __restrict__ a,
                                                                 const T* __restrict__ b,
                                                                 int64_t ld, int nx, int ny,
                                                                 int M, int logM,
                                                                 double* __restrict__ out)
{
    constexpr int kFftCols = 2 * kFftPairs;
    extern __shared__ double lds[];
    const int Mp = M + M / 8;                                  // padded sequence length
    double2* z = reinterpret_cast<double2*>(lds);              // [kFftPairs][Mp]
    double2* tw = z + static_cast<size_t>(kFftPairs) * Mp;     // [M - 1]
    // blocks are dispatched round-robin over the 8 XCDs: give each XCD a
    // contiguous run of column groups, so that the halves of a cache line two
    // neighbouring groups read meet in one L2
    const int nb = gridDim.x, per = (nb + kXcds - 1) / kXcds;
    const int grp = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    if (grp * kFftCols >= ny) return;
    const int m0 = grp * kFftCols;
    const int tid = threadIdx.x;

    // twiddles of stage s (butterfly span 2^s) stored contiguously from
    // 2^{s-1} - 1: e^{2 pi i t / 2^s} for t < 2^{s-1}, so that the lanes of a
    // stage read consecutive entries
    for (int e = tid; e < M - 1; e += kFftThreads) {
        const int sm1 = 31 - __builtin_clz(static_cast<unsigned>(e + 1));   // s - 1
        const int t = e + 1 - (1 << sm1);
        double sn, cs;
        sincospi(static_cast<double>(t) / static_cast<double>(1 << sm1), &sn, &cs);
        tw[e] = make_double2(cs, sn);
    }
    // Hermitian parts of both columns of a pair, bit-reversed into place.
    // H is Hermitian (H_{-k} = conj(H_k)), so thread (k, p) for k = 0 .. M/2
    // reads the rows n = k and n = -k (mod M) once and writes both Z_k and
    // Z_{-k}; all of its loads are independent of each other.
    for (int idx = tid; idx < (M / 2 + 1) * kFftPairs; idx += kFftThreads) {
        const int p = idx % kFftPairs;
        const int k = idx / kFftPairs;
        const int km = (M - k) & (M - 1);
        const int c0 = m0 + 2 * p;
        // C_k = sum_{n = k mod M} (-1)^n (a_n - i b_n), for both columns
        double ck[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, cm[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = c0 + q;
            if (c >= ny) continue;
            for (int n = k; n < nx; n += M) {
                const double s = (n & 1) ? -1.0 : 1.0;
                ck[q][0] += s * static_cast<double>(a[n * ld + c]);
                if (n > 0) ck[q][1] -= s * static_cast<double>(b[n * ld + c]);
            }
            if (km != k) {
                for (int n = km; n < nx; n += M) {
                    const double s = (n & 1) ? -1.0 : 1.0;
                    cm[q][0] += s * static_cast<double>(a[n * ld + c]);
                    if (n > 0) cm[q][1] -= s * static_cast<double>(b[n * ld + c]);
                }
            } else {
                cm[q][0] = ck[q][0];
                cm[q][1] = ck[q][1];
            }
        }
        // H_k = (C_k + conj(C_{-k})) / 2 for both columns; Z = H(m) + i H(m')
        const double h0r = 0.5 * (ck[0][0] + cm[0][0]), h0i = 0.5 * (ck[0][1] - cm[0][1]);
        const double h1r = 0.5 * (ck[1][0] + cm[1][0]), h1i = 0.5 * (ck[1][1] - cm[1][1]);
        z[p * Mp + fft_pad(bit_reverse(k, logM))] = make_double2(h0r - h1i, h0i + h1r);
        if (km != k)   // Z_{-k} = conj(H_k(m)) + i conj(H_k(m'))
            z[p * Mp + fft_pad(bit_reverse(km, logM))] = make_double2(h0r + h1i, h1r - h0i);
    }
    __syncthreads();
    // radix-2 decimation in time, in place
    // (all sizes are powers of two: index arithmetic by shifts and masks)
    for (int s = 1; s <= logM; ++s) {
        const int half = 1 << (s - 1);
        const double2* tws = tw + (half - 1);                // this stage's twiddles
        for (int idx = tid; idx < kFftPairs * (M / 2); idx += kFftThreads) {
            const int p = idx >> (logM - 1);
            const int r = idx & (M / 2 - 1);
            const int g = (r >> (s - 1)) << s;
            const int t = r & (half - 1);
            double2* zp = z + p * Mp;
            const double2 u = zp[fft_pad(g + t)];
            const double2 v0 = zp[fft_pad(g + t + half)];
            const double2 w = tws[t];
            const double2 v = make_double2(v0.x * w.x - v0.y * w.y, v0.x * w.y + v0.y * w.x);
            zp[fft_pad(g + t)] = make_double2(u.x + v.x, u.y + v.y);
            zp[fft_pad(g + t + half)] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    // row j of the output: 16 consecutive columns (real and imaginary parts
    // of the 8 transforms)
    for (int idx = tid; idx < M * kFftCols; idx += kFftThreads) {
        const int c = idx % kFftCols;
        const int j = idx / kFftCols;
        const int m = m0 + c;
        if (m >= ny) continue;
        const double2 v = z[(c >> 1) * Mp + fft_pad(j)];
        out[static_cast<int64_t>(j) * ny + m] = (c & 1) ? v.y : v.x;
    }
}

template <typename T>
hipError_t launch_reconstruct(hipStream_t stream, const T* a, const T* b, int64_t ld, int nx,
                              int ny, int M, double* out)
{
    if (M >= 8 && M <= kFftMaxM && (M & (M - 1)) == 0) {
        const int logM = __builtin_ctz(static_cast<unsigned>(M));
        const int pairs = M <= 256 ? 8 : (M == 512 ? 4 : 2);
        const size_t lds = (static_cast<size_t>(pairs) * (M + M / 8) + M - 1) * sizeof(double2);
        const int groups = (ny + 2 * pairs - 1) / (2 * pairs);
        const int blocks = (groups + kXcds - 1) / kXcds * kXcds;   // whole rounds over the XCDs
        if (pairs == 8)
            hipLaunchKernelGGL((k_reconstruct_fft<T, 8>), dim3(blocks), dim3(kFftThreads), lds,
                               stream, a, b, ld, nx, ny, M, logM, out);
        else if (pairs == 4)
            hipLaunchKernelGGL((k_reconstruct_fft<T, 4>), dim3(blocks), dim3(kFftThreads), lds,
                               stream, a, b, ld, nx, ny, M, logM, out);
        else
            hipLaunchKernelGGL((k_reconstruct_fft<T, 2>), dim3(blocks), dim3(kFftThreads), lds,
                               stream, a, b, ld, nx, ny, M, logM, out);
        return hipGetLastError();
    }
    if (M >= 768) return launch_shape<T, 1, 4, 4>(stream, a, b, ld, nx, ny, M, out);
    return launch_shape<T, 1, 2, 8>(stream, a, b, ld, nx, ny, M, out);
}

template hipError_t launch_reconstruct<float>(hipStream_t, const float*, const float*, int64_t,
                                              int, int, int, double*);
template hipError_t launch_reconstruct<double>(hipStream_t, const double*, const double*, int64_t,
                                               int, int, int, double*);

}  // namespace bte
