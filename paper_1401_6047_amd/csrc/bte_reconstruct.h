// Launcher of the f(phi_x, phi_y) reconstruction kernel (bte_reconstruct.hip).
// Not part of the public C ABI (include/bte.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bte {

// out[j * ny + m] = sum_{n < nx} a[n][m] cos(n x_j) + b[n][m] sin(n x_j),
// x_j = -pi + 2 pi j / M; row stride ld elements, row 0 of b not read.
template <typename T>
hipError_t launch_reconstruct(hipStream_t stream, const T* a, const T* b, int64_t ld, int nx,
                              int ny, int M, double* out);

}  // namespace bte
