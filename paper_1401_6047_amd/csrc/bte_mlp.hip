// Warm-start network: forward pass, loss gradient and Adam on the GPU.
//
// The two large layers are "NT" products C[M][N] = sum_k A[m][k] B[n][k] with
// both operands stored K-contiguous, the layout the 16x16 matrix-core
// instructions read directly from memory: every producer (layer epilogues,
// the loss kernel, the Adam step) also writes the transposed copy the next
// product needs, so no product transposes on the fly.  Batch rows are padded
// to a multiple of 64 with zero gradient, so every product dimension is a
// multiple of the 64 x 64 block tile and no kernel needs a bounds test.
//
// Forward (rows m of the batch, features x):
//   x'  = (x - shift) / scale                      (layer-1 kernel, FP32)
//   Z1  = x' W1^T + b1,  H1 = gelu(Z1)             (layer-1 kernel, FP32)
//   Z2  = H1 W2^T + b2,  H2 = gelu(Z2)             (matrix cores)
//   Y   = H2 W3^T + b3                             (matrix cores)
// Loss L = mean over n x 8192 of (Y - out_scale c)^2; backward:
//   dY  = 2 (Y - out_scale c) / (8192 n)           (loss kernel; 0 on padding)
//   dW3 = dY^T H2,  db3 = colsum dY,  dZ2 = (dY W3) * gelu'(Z2)
//   dW2 = dZ2^T H1, db2 = colsum dZ2, dZ1 = (dZ2 W2) * gelu'(Z1)
//   dW1 = dZ1^T x', db1 = colsum dZ1
// All reductions run in a fixed order, so results are reproducible.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/bte_mlp.h"
#include "bte_internal.h"

namespace bte {
namespace {

constexpr int kIn = BTE_MLP_IN;
constexpr int kHid = BTE_MLP_HIDDEN;
constexpr int kOut = BTE_MLP_OUT;
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + int64_t(kHid) * kIn;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + int64_t(kHid) * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + int64_t(kOut) * kHid;
constexpr int64_t kParams = kOffB3 + kOut;
static_assert(kParams == 2172672, "parameter count");

constexpr int kTile = 64;          // block tile of the products and the loss kernel
constexpr int kNorm = 11;          // shift[5], scale[5], out_scale

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// matrix-core fragments
// ---------------------------------------------------------------------------
// One 16 x 16 output tile per wavefront and instruction.  Lane l supplies row
// (l mod 16) of the A block and of the B block, with a run of consecutive k
// values starting at (l / 16) times the run length; A and B use the same k
// assignment, so the sum over the k block is complete whatever order the
// instruction takes it in.  The accumulator of lane l holds rows
// 4 (l / 16) + q, q = 0..3, of column l mod 16.
template <typename T>
struct Mma;

template <>
struct Mma<__bf16> {
    static constexpr int kK = 32;      // k values per step
    static constexpr int kRun = 8;     // per lane
    using Frag = bf16x8;
    __device__ static Frag load(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
    __device__ static f32x4 mma(const Frag& a, const Frag& b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Mma<float> {
    static constexpr int kK = 16;
    static constexpr int kRun = 4;
    using Frag = f32x4;
    __device__ static Frag load(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
    __device__ static f32x4 mma(const Frag& a, const Frag& b, f32x4 c)
    {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
        return c;
    }
};

template <typename T>
__device__ inline T to_op(float x)
{
    return static_cast<T>(x);   // round to nearest even for BF16
}

// GELU in the erf form and its derivative.
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epilogue {
    kEpiHidden = 0,    // Z = acc + bias -> Zf; H = gelu(Z) -> Ct and CtT
    kEpiOutput = 1,    // acc + bias -> Cf
    kEpiPlain = 2,     // acc -> Cf
    kEpiGeluBack = 3,  // d = acc * gelu'(Zin) -> Cf, and Ct / CtT when set
};

template <typename T>
struct GemmArgs {
    const T* A;        // [M][K]
    const T* B;        // [N][K]
    int M, N, K;
    const float* bias; // [N]
    const float* Zin;  // [M][N] pre-activations (kEpiGeluBack)
    float* Cf;         // [M][N]
    T* Ct;             // [M][N]
    T* CtT;            // [N][M]
};

// 64 x 64 block tile, four wavefronts of 32 x 32 (2 x 2 instruction tiles).
template <typename T, int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs<T> g)
{
    using M_ = Mma<T>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * kTile + (wave >> 1) * 32;
    const int n0 = blockIdx.x * kTile + (wave & 1) * 32;
    const int r = lane & 15;
    const int kq = (lane >> 4) * M_::kRun;
    const size_t K = static_cast<size_t>(g.K);
    const T* a0 = g.A + (m0 + r) * K + kq;
    const T* a1 = a0 + 16 * K;
    const T* b0 = g.B + (n0 + r) * K + kq;
    const T* b1 = b0 + 16 * K;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // fragments of the next k step load while the current step multiplies
    typename M_::Frag fa0 = M_::load(a0), fa1 = M_::load(a1);
    typename M_::Frag fb0 = M_::load(b0), fb1 = M_::load(b1);
    for (int k = M_::kK; k < g.K; k += M_::kK) {
        const typename M_::Frag na0 = M_::load(a0 + k), na1 = M_::load(a1 + k);
        const typename M_::Frag nb0 = M_::load(b0 + k), nb1 = M_::load(b1 + k);
        acc[0][0] = M_::mma(fa0, fb0, acc[0][0]);
        acc[0][1] = M_::mma(fa0, fb1, acc[0][1]);
        acc[1][0] = M_::mma(fa1, fb0, acc[1][0]);
        acc[1][1] = M_::mma(fa1, fb1, acc[1][1]);
        fa0 = na0;
        fa1 = na1;
        fb0 = nb0;
        fb1 = nb1;
    }
    acc[0][0] = M_::mma(fa0, fb0, acc[0][0]);
    acc[0][1] = M_::mma(fa0, fb1, acc[0][1]);
    acc[1][0] = M_::mma(fa1, fb0, acc[1][0]);
    acc[1][1] = M_::mma(fa1, fb1, acc[1][1]);
    const size_t N = static_cast<size_t>(g.N), M = static_cast<size_t>(g.M);
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + j * 16 + r;
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + i * 16 + (lane >> 4) * 4 + q;
                const size_t o = m * N + n;
                const float v = acc[i][j][q];
                if constexpr (EPI == kEpiHidden) {
                    const float z = v + g.bias[n];
                    g.Cf[o] = z;
                    const T h = to_op<T>(gelu(z));
                    g.Ct[o] = h;
                    g.CtT[n * M + m] = h;
                } else if constexpr (EPI == kEpiOutput) {
                    g.Cf[o] = v + g.bias[n];
                } else if constexpr (EPI == kEpiPlain) {
                    g.Cf[o] = v;
                } else {
                    const float d = v * gelu_grad(g.Zin[o]);
                    g.Cf[o] = d;
                    if (g.Ct) g.Ct[o] = to_op<T>(d);
                    if (g.CtT) g.CtT[n * M + m] = to_op<T>(d);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// first layer (5 inputs) on the vector ALUs
// ---------------------------------------------------------------------------
// One thread per (row, hidden unit).  Padding rows (m >= n) and rows whose
// index is out of range take zero features (their gradient is zero, see the
// loss kernel).
template <typename T>
__global__ __launch_bounds__(256) void k_layer1(const float* __restrict__ x,
                                                const int32_t* __restrict__ index, int n_rows,
                                                int n, int Mp,
                                                const float* __restrict__ theta,
                                                const float* __restrict__ norm,
                                                float* __restrict__ xn, float* __restrict__ Z1,
                                                T* __restrict__ H1, T* __restrict__ H1T)
{
    const int m = blockIdx.x;
    const int j = threadIdx.x;
    float f[kIn];
    for (int i = 0; i < kIn; ++i) {
        float v = 0.f;
        const int row = m < n ? (index ? index[m] : m) : -1;
        if (row >= 0 && row < n_rows)
            v = (x[static_cast<size_t>(row) * kIn + i] - norm[i]) / norm[kIn + i];
        f[i] = v;
    }
    if (j < kIn) xn[m * kIn + j] = f[j];
    float z = theta[kOffB1 + j];
    for (int i = 0; i < kIn; ++i) z += theta[kOffW1 + j * kIn + i] * f[i];
    Z1[static_cast<size_t>(m) * kHid + j] = z;
    const T h = to_op<T>(gelu(z));
    H1[static_cast<size_t>(m) * kHid + j] = h;
    H1T[static_cast<size_t>(j) * Mp + m] = h;
}

// dW1[j][i] = sum_m dZ1[m][j] x'[m][i], db1[j] = sum_m dZ1[m][j]
__global__ __launch_bounds__(256) void k_layer1_back(const float* __restrict__ dZ1,
                                                     const float* __restrict__ xn, int Mp,
                                                     float* __restrict__ grad)
{
    const int j = threadIdx.x;
    float sw[kIn] = {0.f, 0.f, 0.f, 0.f, 0.f};
    float sb = 0.f;
    for (int m = 0; m < Mp; ++m) {
        const float d = dZ1[static_cast<size_t>(m) * kHid + j];
        sb += d;
        for (int i = 0; i < kIn; ++i) sw[i] += d * xn[m * kIn + i];
    }
    for (int i = 0; i < kIn; ++i) grad[kOffW1 + j * kIn + i] = sw[i];
    grad[kOffB1 + j] = sb;
}

// out[c] = sum_m X[m][c] (one thread per column, rows in order)
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X, int M, int N,
                                                float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += X[static_cast<size_t>(m) * N + c];
    out[c] = s;
}

// ---------------------------------------------------------------------------
// loss and output gradient, 64 x 64 tiles of Y
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ Y,
                                              const float* __restrict__ coeffs,
                                              const int32_t* __restrict__ index, int n_rows,
                                              int n, int Mp,
                                              const float* __restrict__ norm, float* __restrict__ dYf,
                                              T* __restrict__ dY, T* __restrict__ dYT,
                                              double* __restrict__ partial)
{
    __shared__ float tile[kTile][kTile + 1];
    __shared__ double red[256];
    const int j0 = blockIdx.x * kTile, m0 = blockIdx.y * kTile;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    const float out_scale = norm[2 * kIn];
    const float g = 2.0f / (static_cast<float>(kOut) * static_cast<float>(n));
    double s = 0.0;
    for (int rr = r0; rr < kTile; rr += 4) {
        const int m = m0 + rr, j = j0 + c;
        const size_t o = static_cast<size_t>(m) * kOut + j;
        float d = 0.f;
        const int row = m < n ? (index ? index[m] : m) : -1;
        if (row >= 0 && row < n_rows) {
            const float res = Y[o] - out_scale * coeffs[static_cast<size_t>(row) * kOut + j];
            s += static_cast<double>(res) * res;
            d = g * res;
        }
        dYf[o] = d;
        dY[o] = to_op<T>(d);
        tile[rr][c] = d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int rr = r0; rr < kTile; rr += 4)
        dYT[static_cast<size_t>(j0 + rr) * Mp + m0 + c] = to_op<T>(tile[c][rr]);
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ partial, int np,
                                                    int n, float* __restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss)
        *loss = static_cast<float>(red[0] / (static_cast<double>(kOut) * n));
}

// Forward output back to coefficient units.
__global__ __launch_bounds__(256) void k_unscale(const float* __restrict__ Y, int64_t count,
                                                 const float* __restrict__ norm,
                                                 float* __restrict__ out)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < count) out[e] = Y[e] / norm[2 * kIn];
}

// ---------------------------------------------------------------------------
// normalisation statistics (one block, FP64, fixed order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stats(const float* __restrict__ x,
                                               const float* __restrict__ coeffs, int n,
                                               float* __restrict__ norm)
{
    __shared__ double red[256];
    auto block_sum = [&](double v) {
        __syncthreads();
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        return red[0];
    };
    for (int i = 0; i < kIn; ++i) {
        double s = 0.0;
        for (int m = threadIdx.x; m < n; m += 256) s += x[static_cast<size_t>(m) * kIn + i];
        const double mean = block_sum(s) / n;
        double q = 0.0;
        for (int m = threadIdx.x; m < n; m += 256) {
            const double d = x[static_cast<size_t>(m) * kIn + i] - mean;
            q += d * d;
        }
        const double sd = sqrt(block_sum(q) / n);
        if (threadIdx.x == 0) {
            norm[i] = static_cast<float>(mean);
            norm[kIn + i] = static_cast<float>(sd < 1e-6 * (1.0 + fabs(mean)) ? 1.0 : sd);
        }
    }
    double q = 0.0;
    const int64_t total = static_cast<int64_t>(n) * kOut;
    for (int64_t e = threadIdx.x; e < total; e += 256) {
        const double v = coeffs[e];
        q += v * v;
    }
    const double ms = block_sum(q) / static_cast<double>(total);
    if (threadIdx.x == 0) norm[2 * kIn] = static_cast<float>(ms > 0 ? 1.0 / sqrt(ms) : 1.0);
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master values, and the matrix-core copies of W2 and W3
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta,
                                              const float* __restrict__ grad,
                                              float* __restrict__ m1, float* __restrict__ m2,
                                              int update, float lr, float bc1, float bc2,
                                              T* __restrict__ W2, T* __restrict__ W2T,
                                              T* __restrict__ W3, T* __restrict__ W3T)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float t = theta[p];
    if (update) {
        const float g = grad[p];
        const float a = 0.9f * m1[p] + 0.1f * g;
        const float b = 0.999f * m2[p] + 0.001f * g * g;
        m1[p] = a;
        m2[p] = b;
        t -= lr * (a / bc1) / (sqrtf(b / bc2) + 1e-8f);
        theta[p] = t;
    }
    if (p >= kOffW2 && p < kOffB2) {
        const int64_t e = p - kOffW2, o = e / kHid, i = e % kHid;
        W2[e] = to_op<T>(t);
        W2T[i * kHid + o] = to_op<T>(t);
    } else if (p >= kOffW3 && p < kOffB3) {
        const int64_t e = p - kOffW3, o = e / kHid, i = e % kHid;
        W3[e] = to_op<T>(t);
        W3T[i * kOut + o] = to_op<T>(t);
    }
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int64_t count, float v)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < count) p[e] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
int pad64(int n) { return (n + kTile - 1) / kTile * kTile; }

struct Layout {
    size_t theta, grad, m1, m2, norm, partial;
    size_t W2, W2T, W3, W3T;
    size_t xn, Z1, H1, H1T, Z2, H2, H2T, Y, dYf, dY, dYT, dZ2f, dZ2, dZ2T, dZ1;
    size_t total;
};

Layout make_layout(int max_batch, int precision)
{
    const size_t e = precision == BTE_MLP_FP32 ? 4 : 2;   // operand bytes
    const size_t Mp = static_cast<size_t>(pad64(max_batch));
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.theta = take(4 * kParams);
    L.grad = take(4 * kParams);
    L.m1 = take(4 * kParams);
    L.m2 = take(4 * kParams);
    L.norm = take(4 * 16);
    L.partial = take(8 * (Mp / kTile) * (kOut / kTile));
    L.W2 = take(e * kHid * kHid);
    L.W2T = take(e * kHid * kHid);
    L.W3 = take(e * kOut * kHid);
    L.W3T = take(e * kOut * kHid);
    L.xn = take(4 * Mp * kIn);
    L.Z1 = take(4 * Mp * kHid);
    L.H1 = take(e * Mp * kHid);
    L.H1T = take(e * Mp * kHid);
    L.Z2 = take(4 * Mp * kHid);
    L.H2 = take(e * Mp * kHid);
    L.H2T = take(e * Mp * kHid);
    L.Y = take(4 * Mp * kOut);
    L.dYf = take(4 * Mp * kOut);
    L.dY = take(e * Mp * kOut);
    L.dYT = take(e * Mp * kOut);
    L.dZ2f = take(4 * Mp * kHid);
    L.dZ2 = take(e * Mp * kHid);
    L.dZ2T = take(e * Mp * kHid);
    L.dZ1 = take(4 * Mp * kHid);
    L.total = o;
    return L;
}

bte_status mfail(bte_status st, const std::string& msg)
{
    set_last_error(msg.c_str());
    return st;
}

bte_status launch_ok(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(BTE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return BTE_OK;
}

}  // namespace
}  // namespace bte

using namespace bte;

struct bte_mlp {
    int max_batch = 0;
    int precision = 0;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    Layout L{};
    int64_t adam_steps = 0;
    template <typename T>
    T* at(size_t off) const
    {
        return reinterpret_cast<T*>(ws + off);
    }
};

namespace {

template <typename T>
bte_status gemm(const bte_mlp* h, int epi, const T* A, const T* B, int M, int N, int K,
                const float* bias, const float* Zin, float* Cf, T* Ct, T* CtT)
{
    GemmArgs<T> g{A, B, M, N, K, bias, Zin, Cf, Ct, CtT};
    const dim3 grid(N / kTile, M / kTile);
    switch (epi) {
    case kEpiHidden: hipLaunchKernelGGL((k_gemm_nt<T, kEpiHidden>), grid, dim3(256), 0, h->stream, g); break;
    case kEpiOutput: hipLaunchKernelGGL((k_gemm_nt<T, kEpiOutput>), grid, dim3(256), 0, h->stream, g); break;
    case kEpiPlain: hipLaunchKernelGGL((k_gemm_nt<T, kEpiPlain>), grid, dim3(256), 0, h->stream, g); break;
    default: hipLaunchKernelGGL((k_gemm_nt<T, kEpiGeluBack>), grid, dim3(256), 0, h->stream, g); break;
    }
    return launch_ok("matrix-core product");
}

// Forward pass of rows 0..n-1 (n <= max_batch) up to Y.
template <typename T>
bte_status forward(bte_mlp* h, const float* x, int n_rows, const int32_t* index, int n)
{
    const int Mp = pad64(n);
    const Layout& L = h->L;
    const float* theta = h->at<float>(L.theta);
    hipLaunchKernelGGL((k_layer1<T>), dim3(Mp), dim3(kHid), 0, h->stream, x, index, n_rows, n, Mp,
                       theta,
                       h->at<float>(L.norm), h->at<float>(L.xn), h->at<float>(L.Z1),
                       h->at<T>(L.H1), h->at<T>(L.H1T));
    bte_status rc = launch_ok("layer 1");
    if (rc != BTE_OK) return rc;
    rc = gemm<T>(h, kEpiHidden, h->at<T>(L.H1), h->at<T>(L.W2), Mp, kHid, kHid, theta + kOffB2,
                 nullptr, h->at<float>(L.Z2), h->at<T>(L.H2), h->at<T>(L.H2T));
    if (rc != BTE_OK) return rc;
    return gemm<T>(h, kEpiOutput, h->at<T>(L.H2), h->at<T>(L.W3), Mp, kOut, kHid, theta + kOffB3,
                   nullptr, h->at<float>(L.Y), nullptr, nullptr);
}

template <typename T>
bte_status loss_grad(bte_mlp* h, const float* x, const float* c, int n_rows,
                     const int32_t* index, int n, float* loss)
{
    bte_status rc = forward<T>(h, x, n_rows, index, n);
    if (rc != BTE_OK) return rc;
    const int Mp = pad64(n);
    const Layout& L = h->L;
    float* grad = h->at<float>(L.grad);
    const dim3 lgrid(kOut / kTile, Mp / kTile);
    hipLaunchKernelGGL((k_loss<T>), lgrid, dim3(256), 0, h->stream, h->at<float>(L.Y), c, index,
                       n_rows, n, Mp, h->at<float>(L.norm), h->at<float>(L.dYf), h->at<T>(L.dY),
                       h->at<T>(L.dYT), h->at<double>(L.partial));
    if ((rc = launch_ok("loss")) != BTE_OK) return rc;
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, h->stream, h->at<double>(L.partial),
                       static_cast<int>(lgrid.x * lgrid.y), n, loss);
    if ((rc = launch_ok("loss reduction")) != BTE_OK) return rc;
    // output layer
    rc = gemm<T>(h, kEpiPlain, h->at<T>(L.dYT), h->at<T>(L.H2T), kOut, kHid, Mp, nullptr, nullptr,
                 grad + kOffW3, nullptr, nullptr);
    if (rc != BTE_OK) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(kOut / 256), dim3(256), 0, h->stream, h->at<float>(L.dYf), Mp,
                       kOut, grad + kOffB3);
    if ((rc = launch_ok("bias 3 gradient")) != BTE_OK) return rc;
    rc = gemm<T>(h, kEpiGeluBack, h->at<T>(L.dY), h->at<T>(L.W3T), Mp, kHid, kOut, nullptr,
                 h->at<float>(L.Z2), h->at<float>(L.dZ2f), h->at<T>(L.dZ2), h->at<T>(L.dZ2T));
    if (rc != BTE_OK) return rc;
    // second layer
    rc = gemm<T>(h, kEpiPlain, h->at<T>(L.dZ2T), h->at<T>(L.H1T), kHid, kHid, Mp, nullptr, nullptr,
                 grad + kOffW2, nullptr, nullptr);
    if (rc != BTE_OK) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, h->stream, h->at<float>(L.dZ2f), Mp, kHid,
                       grad + kOffB2);
    if ((rc = launch_ok("bias 2 gradient")) != BTE_OK) return rc;
    rc = gemm<T>(h, kEpiGeluBack, h->at<T>(L.dZ2), h->at<T>(L.W2T), Mp, kHid, kHid, nullptr,
                 h->at<float>(L.Z1), h->at<float>(L.dZ1), nullptr, nullptr);
    if (rc != BTE_OK) return rc;
    // first layer
    hipLaunchKernelGGL(k_layer1_back, dim3(1), dim3(kHid), 0, h->stream, h->at<float>(L.dZ1),
                       h->at<float>(L.xn), Mp, grad);
    return launch_ok("layer 1 gradient");
}

template <typename T>
bte_status adam(bte_mlp* h, int update, float lr)
{
    const Layout& L = h->L;
    float bc1 = 1.f, bc2 = 1.f;
    if (update) {
        ++h->adam_steps;
        bc1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(h->adam_steps)));
        bc2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(h->adam_steps)));
    }
    const int blocks = static_cast<int>((kParams + 255) / 256);
    hipLaunchKernelGGL((k_adam<T>), dim3(blocks), dim3(256), 0, h->stream, h->at<float>(L.theta),
                       h->at<float>(L.grad), h->at<float>(L.m1), h->at<float>(L.m2), update, lr,
                       bc1, bc2, h->at<T>(L.W2), h->at<T>(L.W2T), h->at<T>(L.W3), h->at<T>(L.W3T));
    return launch_ok("Adam step");
}

bte_status fill(bte_mlp* h, float* p, int64_t count, float v)
{
    hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0,
                       h->stream, p, count, v);
    return launch_ok("fill");
}

bte_status check_batch(const bte_mlp* h, const float* x, const float* c, int n_rows,
                       const int32_t* index, int n)
{
    if (!h) return mfail(BTE_EINVAL, "network handle is NULL");
    if (!x || !c) return mfail(BTE_EINVAL, "features and coefficients are required");
    if (n < 1 || n_rows < 1) return mfail(BTE_EINVAL, "n and n_rows must be >= 1");
    if (n > h->max_batch) return mfail(BTE_EINVAL, "n exceeds the network's max_batch");
    if (!index && n > n_rows) return mfail(BTE_EINVAL, "n exceeds n_rows");
    return BTE_OK;
}

}  // namespace

extern "C" {

int64_t bte_mlp_param_count(void) { return kParams; }

size_t bte_mlp_workspace_bytes(int32_t max_batch, int32_t precision)
{
    if (max_batch < 1 || max_batch > (1 << 20)) return 0;
    if (precision != BTE_MLP_BF16 && precision != BTE_MLP_FP32) return 0;
    return make_layout(max_batch, precision).total;
}

bte_status bte_mlp_create(int32_t max_batch, int32_t precision, void* workspace,
                          size_t workspace_bytes, void* hip_stream, bte_mlp** out)
{
    if (!out) return mfail(BTE_EINVAL, "out must not be NULL");
    *out = nullptr;
    const size_t need = bte_mlp_workspace_bytes(max_batch, precision);
    if (need == 0) return mfail(BTE_EINVAL, "max_batch must be in 1..2^20 and precision BF16 or FP32");
    if (!workspace) return mfail(BTE_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return mfail(BTE_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return mfail(BTE_EINVAL, "workspace too small");
    bte_mlp* h = new (std::nothrow) bte_mlp;
    if (!h) return mfail(BTE_ENOMEM, "out of host memory");
    h->max_batch = max_batch;
    h->precision = precision;
    h->ws = static_cast<char*>(workspace);
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->L = make_layout(max_batch, precision);
    // parameters, moments and the operand copies start at zero; identity
    // normalisation
    bte_status rc = fill(h, h->at<float>(0), static_cast<int64_t>(h->L.norm / 4), 0.f);
    if (rc == BTE_OK) rc = fill(h, h->at<float>(h->L.norm), 2 * kIn + 1, 1.f);
    if (rc == BTE_OK) rc = fill(h, h->at<float>(h->L.norm), kIn, 0.f);
    if (rc == BTE_OK)
        rc = precision == BTE_MLP_FP32 ? adam<float>(h, 0, 0.f) : adam<__bf16>(h, 0, 0.f);
    if (rc != BTE_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return BTE_OK;
}

bte_status bte_mlp_set_params(bte_mlp* h, const float* dev_params)
{
    if (!h || !dev_params) return mfail(BTE_EINVAL, "handle and parameters are required");
    if (hipMemcpyAsync(h->at<float>(h->L.theta), dev_params, 4 * kParams, hipMemcpyDeviceToDevice,
                       h->stream) != hipSuccess)
        return mfail(BTE_EDEVICE, "parameter copy failed");
    bte_status rc = fill(h, h->at<float>(h->L.m1), kParams, 0.f);
    if (rc == BTE_OK) rc = fill(h, h->at<float>(h->L.m2), kParams, 0.f);
    if (rc != BTE_OK) return rc;
    h->adam_steps = 0;
    return h->precision == BTE_MLP_FP32 ? adam<float>(h, 0, 0.f) : adam<__bf16>(h, 0, 0.f);
}

bte_status bte_mlp_get_params(bte_mlp* h, float* dev_params)
{
    if (!h || !dev_params) return mfail(BTE_EINVAL, "handle and output are required");
    if (hipMemcpyAsync(dev_params, h->at<float>(h->L.theta), 4 * kParams, hipMemcpyDeviceToDevice,
                       h->stream) != hipSuccess)
        return mfail(BTE_EDEVICE, "parameter copy failed");
    return BTE_OK;
}

bte_status bte_mlp_fit_normalization(bte_mlp* h, const float* dev_features, const float* dev_coeffs,
                                     int32_t n)
{
    if (!h) return mfail(BTE_EINVAL, "network handle is NULL");
    if (!dev_features || !dev_coeffs || n < 1)
        return mfail(BTE_EINVAL, "features, coefficients and n >= 1 are required");
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, h->stream, dev_features, dev_coeffs, n,
                       h->at<float>(h->L.norm));
    return launch_ok("normalisation statistics");
}

bte_status bte_mlp_get_normalization(bte_mlp* h, float* host11)
{
    if (!h || !host11) return mfail(BTE_EINVAL, "handle and output are required");
    if (hipMemcpyAsync(host11, h->at<float>(h->L.norm), 4 * kNorm, hipMemcpyDeviceToHost,
                       h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return mfail(BTE_EDEVICE, "normalisation copy failed");
    return BTE_OK;
}

bte_status bte_mlp_set_normalization(bte_mlp* h, const float* host11)
{
    if (!h || !host11) return mfail(BTE_EINVAL, "handle and values are required");
    for (int i = 0; i < kNorm; ++i)
        if (!std::isfinite(host11[i])) return mfail(BTE_EINVAL, "normalisation values must be finite");
    for (int i = kIn; i < kNorm; ++i)
        if (!(host11[i] > 0.f)) return mfail(BTE_EINVAL, "scales must be positive");
    // a synchronous copy: the host array need not outlive the call
    if (hipMemcpyAsync(h->at<float>(h->L.norm), host11, 4 * kNorm, hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return mfail(BTE_EDEVICE, "normalisation copy failed");
    return BTE_OK;
}

bte_status bte_mlp_forward(bte_mlp* h, const float* dev_features, int32_t n, float* dev_coeffs)
{
    if (!h) return mfail(BTE_EINVAL, "network handle is NULL");
    if (!dev_features || !dev_coeffs) return mfail(BTE_EINVAL, "features and output are required");
    if (n < 1) return mfail(BTE_EINVAL, "n must be >= 1");
    bte_status rc = BTE_OK;
    for (int32_t r0 = 0; r0 < n; r0 += h->max_batch) {
        const int nb = std::min(h->max_batch, n - r0);
        rc = h->precision == BTE_MLP_FP32
                 ? forward<float>(h, dev_features + static_cast<size_t>(r0) * kIn, nb, nullptr, nb)
                 : forward<__bf16>(h, dev_features + static_cast<size_t>(r0) * kIn, nb, nullptr, nb);
        if (rc != BTE_OK) return rc;
        const int64_t count = static_cast<int64_t>(nb) * kOut;
        hipLaunchKernelGGL(k_unscale, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0,
                           h->stream, h->at<float>(h->L.Y), count, h->at<float>(h->L.norm),
                           dev_coeffs + static_cast<size_t>(r0) * kOut);
        if ((rc = launch_ok("output scaling")) != BTE_OK) return rc;
    }
    return BTE_OK;
}

bte_status bte_mlp_loss_grad(bte_mlp* h, const float* dev_features, const float* dev_coeffs,
                             int32_t n_rows, const int32_t* dev_index, int32_t n, float* dev_grad,
                             float* dev_loss)
{
    bte_status rc = check_batch(h, dev_features, dev_coeffs, n_rows, dev_index, n);
    if (rc != BTE_OK) return rc;
    rc = h->precision == BTE_MLP_FP32
             ? loss_grad<float>(h, dev_features, dev_coeffs, n_rows, dev_index, n, dev_loss)
             : loss_grad<__bf16>(h, dev_features, dev_coeffs, n_rows, dev_index, n, dev_loss);
    if (rc != BTE_OK) return rc;
    if (dev_grad && hipMemcpyAsync(dev_grad, h->at<float>(h->L.grad), 4 * kParams,
                                   hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return mfail(BTE_EDEVICE, "gradient copy failed");
    return BTE_OK;
}

bte_status bte_mlp_train_step(bte_mlp* h, const float* dev_features, const float* dev_coeffs,
                              int32_t n_rows, const int32_t* dev_index, int32_t n, float lr,
                              float* dev_loss)
{
    bte_status rc = check_batch(h, dev_features, dev_coeffs, n_rows, dev_index, n);
    if (rc != BTE_OK) return rc;
    if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(BTE_EINVAL, "lr must be positive and finite");
    if (h->precision == BTE_MLP_FP32) {
        rc = loss_grad<float>(h, dev_features, dev_coeffs, n_rows, dev_index, n, dev_loss);
        if (rc == BTE_OK) rc = adam<float>(h, 1, lr);
    } else {
        rc = loss_grad<__bf16>(h, dev_features, dev_coeffs, n_rows, dev_index, n, dev_loss);
        if (rc == BTE_OK) rc = adam<__bf16>(h, 1, lr);
    }
    return rc;
}

void bte_mlp_destroy(bte_mlp* h) { delete h; }

}  // extern "C"
