// Reconstruction of the distribution function from its expansion
// coefficients (eq. spherical-harmonic-exp, App. A): at every basis node of
// every cell and every requested direction,
//     f(node, d) = sum_lms zeta[node][lms] Y_lms(d).
// A (rows x n) by (n x ndir) product with n <= 64, written row-major
// [row][direction].  Each workgroup keeps DIRS directions of the Y table in
// LDS (64, or 16 when there are at most 16 and n <= 49) and walks a strided set of row
// tiles (32 rows, or 128 with 16 directions), staging each tile's
// coefficients in LDS.  A lane computes two neighbouring directions of four
// rows and writes each pair with one 16-byte streaming store (8-byte stores
// for an odd ndir or an output not aligned to 16 bytes).  The 64-direction
// shape keeps its LDS in static arrays of pitch 65 (measured 186-189 us at
// 1024x128 against 195-212 us with launch-sized arrays); the 16-direction
// shape sizes its LDS at launch with pitch n + 1, since its 128-row tile
// would not fit at the widest pitch.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kRecThreads = 256;
constexpr int kRecMaxN = 64;        // LDS-tiled kernels
constexpr int kRecMaxWideN = 144;   // the plain kernel beyond (l_max <= 11)
constexpr int kRecRowsPerLane = 4;

template <int DIRS>
struct RecShape {
  static constexpr int kPairs = DIRS / 2;                    // direction pairs per workgroup
  static constexpr int kRowStep = kRecThreads / kPairs;      // rows between a lane's rows
  static constexpr int kTile = kRowStep * kRecRowsPerLane;   // node rows per tile
};

// NREG > 0 (n <= NREG): a lane keeps its two directions' table rows in
// registers, read from LDS once, so the inner loop reads only the tile
template <int DIRS, int NREG>
__global__ __launch_bounds__(kRecThreads) void reconstruct_kernel(const double* __restrict__ zeta, int64_t rows,
                                                                   int n, const double* __restrict__ Y,
                                                                   int64_t ndir, double* __restrict__ out) {
  using S = RecShape<DIRS>;
  // zs [kTile][pitch] and ys [DIRS][pitch]: static arrays at the widest
  // pitch for 64 directions, launch-sized for 16
  double* zs;
  double* ys;
  int pitch;
  if constexpr (DIRS == 64) {
    __shared__ double zs_s[S::kTile * (kRecMaxN + 1)];
    __shared__ double ys_s[DIRS * (kRecMaxN + 1)];
    zs = zs_s;
    ys = ys_s;
    pitch = kRecMaxN + 1;
  } else {
    extern __shared__ double rec_smem[];
    pitch = n + 1;
    zs = rec_smem;
    ys = rec_smem + S::kTile * pitch;
  }
  const int64_t d0 = (int64_t)blockIdx.y * DIRS;
  // the block's directions stay in LDS while it walks its row tiles
  for (int e = threadIdx.x; e < DIRS * n; e += kRecThreads) {
    const int i = e / n, j = e - (e / n) * n;
    ys[i * pitch + j] = (d0 + i < ndir) ? Y[(d0 + i) * n + j] : 0.0;
  }
  // thread -> (directions 2 dp and 2 dp + 1, rows rr + kRowStep q)
  const int dp = threadIdx.x % S::kPairs, rr = threadIdx.x / S::kPairs;
  const bool pairs = (ndir % 2) == 0 && (reinterpret_cast<uintptr_t>(out) % 16) == 0;   // 16-byte aligned pairs
  double y0r[NREG > 0 ? NREG : 1], y1r[NREG > 0 ? NREG : 1];
  if constexpr (NREG > 0) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      y0r[j] = j < n ? ys[(2 * dp) * pitch + j] : 0.0;
      y1r[j] = j < n ? ys[(2 * dp + 1) * pitch + j] : 0.0;
    }
  }
  for (int64_t r0 = (int64_t)blockIdx.x * S::kTile; r0 < rows; r0 += (int64_t)gridDim.x * S::kTile) {
    __syncthreads();   // the previous tile's reads of zs are done
    for (int e = threadIdx.x; e < S::kTile * n; e += kRecThreads) {
      const int i = e / n, j = e - (e / n) * n;
      zs[i * pitch + j] = (r0 + i < rows) ? zeta[(r0 + i) * n + j] : 0.0;
    }
    __syncthreads();
    double a0[kRecRowsPerLane], a1[kRecRowsPerLane];
#pragma unroll
    for (int q = 0; q < kRecRowsPerLane; ++q) a0[q] = a1[q] = 0.0;
    if constexpr (NREG > 0) {
#pragma unroll
      for (int j = 0; j < NREG; ++j) {
        if (j < n) {
#pragma unroll
          for (int q = 0; q < kRecRowsPerLane; ++q) {
            const double zv = zs[(rr + S::kRowStep * q) * pitch + j];
            a0[q] = fma(zv, y0r[j], a0[q]);
            a1[q] = fma(zv, y1r[j], a1[q]);
          }
        }
      }
    } else {
      const double* y0p = ys + (2 * dp) * pitch;
      const double* y1p = y0p + pitch;
      for (int j = 0; j < n; ++j) {
        const double y0 = y0p[j], y1 = y1p[j];
#pragma unroll
        for (int q = 0; q < kRecRowsPerLane; ++q) {
          const double zv = zs[(rr + S::kRowStep * q) * pitch + j];
          a0[q] = fma(zv, y0, a0[q]);
          a1[q] = fma(zv, y1, a1[q]);
        }
      }
    }
    // written once and not read again here: streaming stores
    const int64_t d = d0 + 2 * dp;
    if (pairs && d + 1 < ndir) {
      typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int q = 0; q < kRecRowsPerLane; ++q) {
        const int64_t r = r0 + rr + S::kRowStep * q;
        if (r < rows) {
          d2v v;
          v.x = a0[q];
          v.y = a1[q];
          __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(&out[r * ndir + d]));
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < kRecRowsPerLane; ++q) {
        const int64_t r = r0 + rr + S::kRowStep * q;
        if (r < rows && d < ndir) __builtin_nontemporal_store(a0[q], &out[r * ndir + d]);
        if (r < rows && d + 1 < ndir) __builtin_nontemporal_store(a1[q], &out[r * ndir + d + 1]);
      }
    }
  }
}

template <int DIRS>
void launch_t(const double* zeta, int64_t rows, int n, const double* Y, int64_t ndir, double* out, hipStream_t s) {
  using S = RecShape<DIRS>;
  const int64_t tiles = (rows + S::kTile - 1) / S::kTile;
  const dim3 grid((unsigned)(tiles < 2048 ? tiles : 2048), (unsigned)((ndir + DIRS - 1) / DIRS));
  const size_t lds = DIRS == 64 ? 0 : (size_t)(S::kTile + DIRS) * (n + 1) * sizeof(double);
  // the register rows only where the workgroup's LDS already limits the
  // occupancy (64 directions: 3 workgroups per CU either way)
  if (DIRS == 64 && n <= 16)
    hipLaunchKernelGGL((reconstruct_kernel<DIRS, 16>), grid, dim3(kRecThreads), lds, s, zeta, rows, n, Y, ndir, out);
  else
    hipLaunchKernelGGL((reconstruct_kernel<DIRS, 0>), grid, dim3(kRecThreads), lds, s, zeta, rows, n, Y, ndir, out);
}

// n > 64 (l_max 8..11): one output per lane, the row and the direction's
// table read through the caches (the LDS tiles above are sized for n <= 64).
__global__ __launch_bounds__(256) void reconstruct_wide_kernel(const double* __restrict__ zeta, int64_t rows, int n,
                                                              const double* __restrict__ Y, int64_t ndir,
                                                              double* __restrict__ out) {
  const int64_t total = rows * ndir;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int64_t r = t / ndir, d = t - r * ndir;
    const double* z = zeta + r * n;
    const double* y = Y + d * n;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(z[j], y[j], acc);
    out[t] = acc;
  }
}

}  // namespace

int reconstruct_max_lms() { return kRecMaxWideN; }

// LDS per workgroup stays within 64 KB: 64 directions need (32 + 64) 65
// doubles (50 KB); 16 directions need (128 + 16)(n + 1), taken up to n = 49
// (58 KB)
void launch_reconstruct(const double* zeta, int64_t rows, int n, const double* Y, int64_t ndir, double* out,
                        hipStream_t s) {
  if (n > kRecMaxN) {
    const int64_t total = rows * ndir;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(reconstruct_wide_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s,
                       zeta, rows, n, Y, ndir, out);
  } else if (ndir <= 16 && n <= 49)
    launch_t<16>(zeta, rows, n, Y, ndir, out, s);
  else
    launch_t<64>(zeta, rows, n, Y, ndir, out, s);
}

}  // namespace vfp
