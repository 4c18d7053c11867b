// Reconstruction of the distribution function from its expansion
// coefficients (eq. spherical-harmonic-exp, App. A): at every basis node of
// every cell and every requested direction,
//     f(node, d) = sum_lms zeta[node][lms] Y_lms(d).
// A (rows x n) by (n x ndir) product with n <= 64: each workgroup stages a
// tile of 32 node rows and 32 directions of the Y table in LDS and writes the
// 32 x 32 outputs, direction index fastest (row-major [row][direction]).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kRecTile = 32;
constexpr int kRecThreads = 256;
constexpr int kRecMaxN = 64;

__global__ __launch_bounds__(kRecThreads) void reconstruct_kernel(const double* __restrict__ zeta, int64_t rows,
                                                                   int n, const double* __restrict__ Y,
                                                                   int64_t ndir, double* __restrict__ out) {
  __shared__ double zs[kRecTile][kRecMaxN + 1];
  __shared__ double ys[kRecTile][kRecMaxN + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kRecTile;
  const int64_t d0 = (int64_t)blockIdx.y * kRecTile;
  for (int e = threadIdx.x; e < kRecTile * n; e += kRecThreads) {
    const int i = e / n, j = e - (e / n) * n;
    zs[i][j] = (r0 + i < rows) ? zeta[(r0 + i) * n + j] : 0.0;
    ys[i][j] = (d0 + i < ndir) ? Y[(d0 + i) * n + j] : 0.0;
  }
  __syncthreads();
  // thread -> (direction column dc, rows rr, rr + 8, rr + 16, rr + 24)
  const int dc = threadIdx.x % kRecTile, rr = threadIdx.x / kRecTile;
  double acc[kRecTile / 8] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < n; ++j) {
    const double y = ys[dc][j];
#pragma unroll
    for (int q = 0; q < kRecTile / 8; ++q) acc[q] = fma(zs[rr + 8 * q][j], y, acc[q]);
  }
  if (d0 + dc < ndir) {
#pragma unroll
    for (int q = 0; q < kRecTile / 8; ++q) {
      const int64_t r = r0 + rr + 8 * q;
      if (r < rows) out[r * ndir + d0 + dc] = acc[q];
    }
  }
}

}  // namespace

int reconstruct_max_lms() { return kRecMaxN; }

void launch_reconstruct(const double* zeta, int64_t rows, int n, const double* Y, int64_t ndir, double* out,
                        hipStream_t s) {
  const dim3 grid((unsigned)((rows + kRecTile - 1) / kRecTile), (unsigned)((ndir + kRecTile - 1) / kRecTile));
  hipLaunchKernelGGL(reconstruct_kernel, grid, dim3(kRecThreads), 0, s, zeta, rows, n, Y, ndir, out);
}

}  // namespace vfp
