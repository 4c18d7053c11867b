// Reconstruction of the distribution function from its expansion
// coefficients (eq. spherical-harmonic-exp, App. A): at every basis node of
// every cell and every requested direction,
//     f(node, d) = sum_lms zeta[node][lms] Y_lms(d).
// A (rows x n) by (n x ndir) product with n <= 64: each workgroup keeps 64
// directions of the Y table in LDS, stages tiles of 32 node rows and writes
// 32 x 64 outputs per tile, direction index fastest (row-major
// [row][direction]); it walks a strided set of row tiles.  A lane computes
// two neighbouring directions of four rows and writes each pair with one
// 16-byte streaming store, so a wavefront stores two whole 64-direction rows
// per instruction (an odd ndir, or an output not 16-byte aligned, falls back
// to 8-byte stores).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kRecTile = 32;        // node rows per tile
constexpr int kRecDirs = 64;        // directions per workgroup
constexpr int kRecThreads = 256;
constexpr int kRecPairs = kRecDirs / 2;                 // direction pairs per workgroup
constexpr int kRecRowStep = kRecThreads / kRecPairs;    // rows between a lane's rows
constexpr int kRecMaxN = 64;

__global__ __launch_bounds__(kRecThreads) void reconstruct_kernel(const double* __restrict__ zeta, int64_t rows,
                                                                   int n, const double* __restrict__ Y,
                                                                   int64_t ndir, double* __restrict__ out) {
  __shared__ double zs[kRecTile][kRecMaxN + 1];
  __shared__ double ys[kRecDirs][kRecMaxN + 1];
  const int64_t d0 = (int64_t)blockIdx.y * kRecDirs;
  // the block's directions stay in LDS while it walks its row tiles
  for (int e = threadIdx.x; e < kRecDirs * n; e += kRecThreads) {
    const int i = e / n, j = e - (e / n) * n;
    ys[i][j] = (d0 + i < ndir) ? Y[(d0 + i) * n + j] : 0.0;
  }
  // thread -> (directions 2 dp and 2 dp + 1, rows rr + kRecRowStep q)
  const int dp = threadIdx.x % kRecPairs, rr = threadIdx.x / kRecPairs;
  const bool pairs = (ndir % 2) == 0 && (reinterpret_cast<uintptr_t>(out) % 16) == 0;   // 16-byte aligned pairs
  for (int64_t r0 = (int64_t)blockIdx.x * kRecTile; r0 < rows; r0 += (int64_t)gridDim.x * kRecTile) {
    __syncthreads();   // the previous tile's reads of zs are done
    for (int e = threadIdx.x; e < kRecTile * n; e += kRecThreads) {
      const int i = e / n, j = e - (e / n) * n;
      zs[i][j] = (r0 + i < rows) ? zeta[(r0 + i) * n + j] : 0.0;
    }
    __syncthreads();
    constexpr int NQ = kRecTile / kRecRowStep;
    double a0[NQ], a1[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a0[q] = a1[q] = 0.0;
    for (int j = 0; j < n; ++j) {
      const double y0 = ys[2 * dp][j], y1 = ys[2 * dp + 1][j];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double zv = zs[rr + kRecRowStep * q][j];
        a0[q] = fma(zv, y0, a0[q]);
        a1[q] = fma(zv, y1, a1[q]);
      }
    }
    // written once and not read again here: streaming stores
    const int64_t d = d0 + 2 * dp;
    if (pairs && d + 1 < ndir) {
      typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int64_t r = r0 + rr + kRecRowStep * q;
        if (r < rows) {
          d2v v;
          v.x = a0[q];
          v.y = a1[q];
          __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(&out[r * ndir + d]));
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int64_t r = r0 + rr + kRecRowStep * q;
        if (r < rows && d < ndir) __builtin_nontemporal_store(a0[q], &out[r * ndir + d]);
        if (r < rows && d + 1 < ndir) __builtin_nontemporal_store(a1[q], &out[r * ndir + d + 1]);
      }
    }
  }
}

}  // namespace

int reconstruct_max_lms() { return kRecMaxN; }

void launch_reconstruct(const double* zeta, int64_t rows, int n, const double* Y, int64_t ndir, double* out,
                        hipStream_t s) {
  const int64_t tiles = (rows + kRecTile - 1) / kRecTile;
  const dim3 grid((unsigned)(tiles < 2048 ? tiles : 2048), (unsigned)((ndir + kRecDirs - 1) / kRecDirs));
  hipLaunchKernelGGL(reconstruct_kernel, grid, dim3(kRecThreads), 0, s, zeta, rows, n, Y, ndir, out);
}

}  // namespace vfp
