// Vector kernels of the restarted GMRES that solves the Theta-method system
// (eq. system-matrix-rhs) for the implicit time step.  The operator of that
// system is applied by the fused stage kernels; these kernels provide the
// Krylov-basis arithmetic: several dot products against one vector in one
// pass, the matching multi-vector update, and plain linear combinations.
// Reductions are two-stage (fixed partial layout, then one block per result)
// so that every result is reproducible run to run.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kKryThreads = 256;
constexpr int kDotChunk = 8;          // basis vectors per block row of a multi-dot

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum of v over the workgroup (every thread gets it)
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kKryThreads / 64];
  __syncthreads();   // red is free again
  v = wave_sum(v);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kKryThreads / 64; ++q) s += red[q];
  return s;
}

// partial[j][blockIdx.x] = sum over this block's elements of V_j . w, for the
// kDotChunk vectors j = blockIdx.y kDotChunk + c < k; with self != 0 the
// first block row also writes w . w as row k (the norm that the Gram-Schmidt
// step needs, from the same pass over w).  C = the vectors of this block row
// (a compile-time count, so every load is unconditional); each thread takes
// its elements two strides at a time with all loads issued before the FMAs,
// in the same order as one at a time.
template <int C>
__device__ __forceinline__ void mdot_rows(const double* __restrict__ V, int64_t ldv, int j0,
                                          const double* __restrict__ w, int64_t n, bool do_self,
                                          double (&acc)[kDotChunk], double& ws) {
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x;
  const double* Vj = V + (int64_t)j0 * ldv;
  for (; i + stride < n; i += 2 * stride) {
    const double wa = w[i], wb = w[i + stride];
    double va[C], vb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      va[c] = Vj[(int64_t)c * ldv + i];
      vb[c] = Vj[(int64_t)c * ldv + i + stride];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fma(vb[c], wb, fma(va[c], wa, acc[c]));
    if (do_self) ws = fma(wb, wb, fma(wa, wa, ws));
  }
  if (i < n) {
    const double wa = w[i];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fma(Vj[(int64_t)c * ldv + i], wa, acc[c]);
    if (do_self) ws = fma(wa, wa, ws);
  }
}

__global__ __launch_bounds__(kKryThreads) void mdot_partial_kernel(const double* __restrict__ V, int64_t ldv,
                                                                    int k, const double* __restrict__ w,
                                                                    int64_t n, double* __restrict__ partial,
                                                                    int self, const double* __restrict__ enable) {
  if (enable && *enable == 0.0) return;   // a pass the device decided to skip
  const int j0 = blockIdx.y * kDotChunk;
  const bool do_self = self && blockIdx.y == 0;
  double acc[kDotChunk], ws = 0.0;
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) acc[c] = 0.0;
  switch (k - j0 < kDotChunk ? k - j0 : kDotChunk) {
    case 1: mdot_rows<1>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 2: mdot_rows<2>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 3: mdot_rows<3>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 4: mdot_rows<4>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 5: mdot_rows<5>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 6: mdot_rows<6>(V, ldv, j0, w, n, do_self, acc, ws); break;
    case 7: mdot_rows<7>(V, ldv, j0, w, n, do_self, acc, ws); break;
    default: mdot_rows<kDotChunk>(V, ldv, j0, w, n, do_self, acc, ws); break;
  }
  __shared__ double red[kDotChunk + 1][kKryThreads / 64];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) {
    const double s = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = s;
  }
  if (do_self) {
    const double s = wave_sum(ws);
    if (lane == 0) red[kDotChunk][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < kDotChunk && j0 + (int)threadIdx.x < k) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kKryThreads / 64; ++q) s += red[threadIdx.x][q];
    partial[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
  if (do_self && threadIdx.x == kDotChunk) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kKryThreads / 64; ++q) s += red[kDotChunk][q];
    partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
  }
}

// out[j] = sum_b partial[j][b]  (one block per j)
__global__ __launch_bounds__(kKryThreads) void mdot_final_kernel(const double* __restrict__ partial, int nblk,
                                                                  double* __restrict__ out,
                                                                  const double* __restrict__ enable) {
  if (enable && *enable == 0.0) return;
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kKryThreads) s += partial[(int64_t)j * nblk + b];
  __shared__ double red[kKryThreads / 64];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kKryThreads / 64; ++q) t += red[q];
    out[j] = t;
  }
}

// w += sign * sum_{j<k} coef[j] V_j; with partial != null also
// partial[blockIdx.x] = sum over this block's elements of the new w . w
__global__ __launch_bounds__(kKryThreads) void maxpy_kernel(double* __restrict__ w, const double* __restrict__ V,
                                                             int64_t ldv, int k, const double* __restrict__ coef,
                                                             double sign, int64_t n, double* __restrict__ partial,
                                                             const double* __restrict__ enable) {
  if (enable && *enable == 0.0) return;
  __shared__ double cs[kKryMaxVectors];
  for (int j = threadIdx.x; j < k; j += kKryThreads) cs[j] = sign * coef[j];
  __syncthreads();
  double ws = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  for (int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; i < n; i += stride) {
    double acc = w[i];
    for (int j = 0; j < k; ++j) acc = fma(cs[j], V[(int64_t)j * ldv + i], acc);
    w[i] = acc;
    ws = fma(acc, acc, ws);
  }
  if (partial) {
    const double s = block_sum(ws);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// out = a x + b y  (out may alias x or y)
__global__ __launch_bounds__(kKryThreads) void lincomb_kernel(double* out, double a, const double* x, double b,
                                                               const double* y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  for (int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; i < n; i += stride)
    out[i] = (b == 0.0) ? a * x[i] : fma(a, x[i], b * y[i]);
}

// out = in / (1 + s nu_c c_lms): the scattering part of I - dt Theta L0,
// which the inverse mass reduces to the exact per-DoF factor nu_c l(l+1)/2
// (in may alias out).  nu: per cell or null (nu0).
__global__ __launch_bounds__(kKryThreads) void coll_precond_kernel(double* out, const double* in,
                                                                    const double* __restrict__ nu, double nu0,
                                                                    const double* __restrict__ cval, double s,
                                                                    int64_t per_cell, int n, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  for (int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; i < total; i += stride) {
    const int64_t cell = i / per_cell;
    const int r = (int)(i % n);
    const double nc = nu ? nu[cell] : nu0;
    out[i] = in[i] / fma(s * nc, cval[r], 1.0);
  }
}

// The classical Gram-Schmidt step's decision on the device: a second pass
// where the first removed more than half of |w|^2 (d3[1] = |w_new|^2,
// d1[j + 1] = |w_old|^2); d3[4] = 1 or 0.
__global__ void decide_kernel(const double* __restrict__ d1, int j, double* __restrict__ d3) {
  if (threadIdx.x == 0) d3[4] = d3[1] < 0.5 * d1[j + 1] ? 1.0 : 0.0;
}

// hn = |w| after the Gram-Schmidt passes (d3[2] after a second pass, else
// d3[1]) into d3[3], and out = w / hn (out may be null)
__global__ __launch_bounds__(kKryThreads) void norm_scale_kernel(double* __restrict__ out,
                                                                  const double* __restrict__ w, int64_t n,
                                                                  double* __restrict__ d3) {
  const double hn2 = d3[4] != 0.0 ? d3[2] : d3[1];
  const double hn = sqrt(hn2 > 0.0 ? hn2 : 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) d3[3] = hn;
  if (!out) return;
  const double a = 1.0 / hn;
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  for (int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; i < n; i += stride) out[i] = a * w[i];
}

int grid_for(int64_t n) {
  const int64_t g = (n + kKryThreads - 1) / kKryThreads;
  return (int)(g < 1 ? 1 : (g > kKryBlocks ? kKryBlocks : g));
}

}  // namespace

void kry_mdot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial, double* out,
              hipStream_t s, bool self, const double* enable) {
  if (k <= 0) return;
  const dim3 grid(kKryBlocks, (k + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(mdot_partial_kernel, grid, dim3(kKryThreads), 0, s, V, ldv, k, w, n, partial, self ? 1 : 0,
                     enable);
  hipLaunchKernelGGL(mdot_final_kernel, dim3(k + (self ? 1 : 0)), dim3(kKryThreads), 0, s, partial, kKryBlocks,
                     out, enable);
}

void kry_maxpy(double* w, const double* V, int64_t ldv, int k, const double* coef, double sign, int64_t n,
               hipStream_t s, double* partial, double* norm2, const double* enable) {
  if (k <= 0) return;
  const int g = grid_for(n);
  hipLaunchKernelGGL(maxpy_kernel, dim3(g), dim3(kKryThreads), 0, s, w, V, ldv, k, coef, sign, n,
                     norm2 ? partial : nullptr, enable);
  if (norm2) hipLaunchKernelGGL(mdot_final_kernel, dim3(1), dim3(kKryThreads), 0, s, partial, g, norm2, enable);
}

void kry_decide(const double* d1, int j, double* d3, hipStream_t s) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(64), 0, s, d1, j, d3);
}

void kry_norm_scale(double* out, const double* w, int64_t n, double* d3, hipStream_t s) {
  hipLaunchKernelGGL(norm_scale_kernel, dim3(out ? grid_for(n) : 1), dim3(kKryThreads), 0, s, out, w, n, d3);
}

void kry_coll_precond(double* out, const double* in, const double* nu, double nu0, const double* cval, double s,
                      int64_t ncells, int nb, int n, hipStream_t st) {
  const int64_t per_cell = (int64_t)nb * n, total = ncells * per_cell;
  hipLaunchKernelGGL(coll_precond_kernel, dim3(grid_for(total)), dim3(kKryThreads), 0, st, out, in, nu, nu0, cval, s,
                     per_cell, n, total);
}

namespace {
// flag[0] = 1 if any x[i] is NaN or infinite (every writer stores the same
// value, so the race is benign)
__global__ __launch_bounds__(kKryThreads) void nonfinite_kernel(const double* __restrict__ x, int64_t n, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; i < n; i += stride) bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;
}
}  // namespace

void kry_nonfinite(const double* x, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n)), dim3(kKryThreads), 0, s, x, n, flag);
}

void kry_lincomb(double* out, double a, const double* x, double b, const double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n)), dim3(kKryThreads), 0, s, out, a, x, b, y ? y : x, n);
}

}  // namespace vfp
