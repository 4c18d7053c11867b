// Block-tridiagonal ("x-line") preconditioner for the Theta-method system
// A = I - dt Theta L0 (eq. system-matrix-rhs after the cell-wise inverse
// mass).  A couples a cell only to its face neighbours; keeping, for every
// cell, the block acting on its own unknowns and the two blocks acting on
// its neighbours along axis 0 gives a block-tridiagonal matrix per line of
// cells along axis 0 (cells ix = 0 .. nx-1 at fixed indices of the other
// axes), which a block Thomas recurrence inverts exactly.  Upwinding along
// axis 0 at large Courant numbers (the transport that makes the unpreconditioned
// GMRES slow) is then solved directly; the coupling along the other axes, and
// across a periodic wrap of axis 0, is left to the Krylov iteration.
//
// Blocks are extracted from the operator itself, with no assembly: with a
// unit vector e_j in the local unknown j of every cell of one colour (colour
// ix mod 3, so no two cells of one colour are neighbours along axis 0, and
// cells of one colour differ in ix from every neighbour along the other
// axes), A's output at a coloured cell is column j of its own block, and at
// its neighbours along axis 0 column j of their blocks towards it.
//
// Storage per cell, b = (k+1)^d n unknowns: three b x b blocks, column-major
// (entry (row, col) at col b + row): D (own), L (towards ix - 1), U (towards
// ix + 1).  xl_factor overwrites D with S^{-1}, U with G = S^{-1} U and,
// past the first cell of each line, L with M = S^{-1} L, where
// S_i = D_i - L_i G_{i-1} (block LU along the line, pivoting inside each
// block by Gauss-Jordan with partial pivoting).  The solve is then
// y_i = S_i^{-1} r_i - M_i y_{i-1} forward and x_i = y_i - G_i x_{i+1}
// backward: one block product per cell on each recurrence chain, the
// products S_i^{-1} r_i standing apart from it.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kXlThreads = 256;
constexpr int kXlApplyThreads = 64;

__device__ __forceinline__ int xl_color(int ix, int nx, int wrapc) { return (wrapc && ix == nx - 1) ? 3 : ix % 3; }

__global__ __launch_bounds__(kXlThreads) void xl_probe_set_kernel(double* v, int64_t ndofs, int nx, int b, int wrapc,
                                                                 int color, int j) {
  const int64_t t = (int64_t)blockIdx.x * kXlThreads + threadIdx.x;
  if (t >= ndofs) return;
  const int64_t cell = t / b;
  const int loc = (int)(t - cell * b);
  const int ix = (int)(cell % nx);
  v[t] = (loc == j && xl_color(ix, nx, wrapc) == color) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(kXlThreads) void xl_probe_get_kernel(const double* __restrict__ w, double* D, double* L,
                                                                 double* U, int64_t ndofs, int nx, int b, int wrapc,
                                                                 int color, int j) {
  const int64_t t = (int64_t)blockIdx.x * kXlThreads + threadIdx.x;
  if (t >= ndofs) return;
  const int64_t cell = t / b;
  const int row = (int)(t - cell * b);
  const int ix = (int)(cell % nx);
  if (xl_color(ix, nx, wrapc) != color) return;
  const int64_t bb = (int64_t)b * b;
  D[cell * bb + (int64_t)j * b + row] = w[t];
  if (ix + 1 < nx) L[(cell + 1) * bb + (int64_t)j * b + row] = w[t + b];   // A(ix+1, ix) e_j
  if (ix > 0) U[(cell - 1) * bb + (int64_t)j * b + row] = w[t - b];        // A(ix-1, ix) e_j
}

// In-place inverse of the b x b matrix S (column-major, in LDS) by
// Gauss-Jordan elimination with partial pivoting; every thread of the
// workgroup takes part.  Returns false (to every thread) if a pivot is 0.
__device__ bool xl_invert(double* S, int b, int* perm, int* sh_piv, double* sh_val) {
  const int tid = threadIdx.x;
  bool ok = true;
  for (int k = 0; k < b; ++k) {
    if (tid < 64) {
      // the first row r >= k of largest |S[r][k]|: an arg-max over the
      // first wavefront (b <= 64 rows), ties to the smaller row
      const int r = k + tid;
      double a = r < b ? fabs(S[k * b + r]) : -1.0;
      int idx = r;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double a2 = __shfl_xor(a, off, 64);
        const int i2 = __shfl_xor(idx, off, 64);
        if (a2 > a || (a2 == a && i2 < idx)) {
          a = a2;
          idx = i2;
        }
      }
      if (tid == 0) {
        perm[k] = idx;
        *sh_piv = idx;
      }
    }
    __syncthreads();
    const int p = *sh_piv;
    if (p != k)
      for (int c = tid; c < b; c += blockDim.x) {
        const double a = S[c * b + k];
        S[c * b + k] = S[c * b + p];
        S[c * b + p] = a;
      }
    __syncthreads();
    if (tid == 0) *sh_val = S[k * b + k];
    __syncthreads();
    const double pv = *sh_val;
    if (pv == 0.0) ok = false;
    const double ipv = 1.0 / pv;
    // row k scaled: S[k][k] = 1/pv, S[k][c] /= pv
    for (int c = tid; c < b; c += blockDim.x) S[c * b + k] = (c == k) ? ipv : S[c * b + k] * ipv;
    __syncthreads();
    // the other rows: S[r][c] -= S[r][k] S[k][c] (c != k), then S[r][k] = -S[r][k] / pv
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int c = e / b, r = e - c * b;
      if (r != k && c != k) S[e] = fma(-S[k * b + r], S[c * b + k], S[e]);
    }
    __syncthreads();
    for (int r = tid; r < b; r += blockDim.x)
      if (r != k) S[k * b + r] = -S[k * b + r] * ipv;
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = b - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int r = tid; r < b; r += blockDim.x) {
        const double a = S[k * b + r];
        S[k * b + r] = S[p * b + r];
        S[p * b + r] = a;
      }
    __syncthreads();
  }
  return ok;
}

// One workgroup per line: S_i = D_i - L_i G_{i-1}, D_i <- S_i^{-1},
// U_i <- G_i = S_i^{-1} U_i, L_i <- M_i = S_i^{-1} L_i (i > 0).
// fail[line] = 1 if a block was singular.  The next cell's three blocks are
// loaded into registers while the current cell is worked on, and staged in
// LDS, so that the block products read no global memory.
constexpr int kXlPer = (kXlMaxBlock * kXlMaxBlock + kXlThreads - 1) / kXlThreads;   // block entries per thread

__global__ __launch_bounds__(kXlThreads) void xl_factor_kernel(double* D, double* L, double* U, int nx, int b,
                                                              int* fail) {
  __shared__ double S[kXlMaxBlock * kXlMaxBlock];
  __shared__ double G[kXlMaxBlock * kXlMaxBlock];
  __shared__ double Lb[kXlMaxBlock * kXlMaxBlock];
  __shared__ double Ub[kXlMaxBlock * kXlMaxBlock];
  __shared__ int perm[kXlMaxBlock];
  __shared__ int sh_piv;
  __shared__ double sh_val;
  const int tid = threadIdx.x;
  const int line = blockIdx.x;
  const int64_t bb = (int64_t)b * b;
  bool ok = true;
  double nD[kXlPer], nL[kXlPer], nU[kXlPer];
  auto load_blocks = [&](int i) {
    const int64_t base = ((int64_t)line * nx + i) * bb;
#pragma unroll
    for (int t = 0; t < kXlPer; ++t) {
      const int e = tid + t * kXlThreads;
      const bool in = i < nx && e < bb;
      nD[t] = in ? D[base + e] : 0.0;
      nL[t] = in ? L[base + e] : 0.0;
      nU[t] = in ? U[base + e] : 0.0;
    }
  };
  load_blocks(0);
  for (int i = 0; i < nx; ++i) {
    const int64_t cell = (int64_t)line * nx + i;
#pragma unroll
    for (int t = 0; t < kXlPer; ++t) {
      const int e = tid + t * kXlThreads;
      if (e < bb) {
        S[e] = nD[t];
        Lb[e] = nL[t];
        Ub[e] = nU[t];
      }
    }
    __syncthreads();
    load_blocks(i + 1);   // in flight during this cell
    if (i > 0) {
      // S -= L G_{i-1}: (L G)[r][c] = sum_k L[r][k] G[k][c]
      for (int e = tid; e < b * b; e += blockDim.x) {
        const int c = e / b, r = e - c * b;
        double acc = 0.0;
        for (int k = 0; k < b; ++k) acc = fma(Lb[k * b + r], G[c * b + k], acc);
        S[e] -= acc;
      }
      __syncthreads();
    }
    ok = xl_invert(S, b, perm, &sh_piv, &sh_val) && ok;
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int c = e / b, r = e - c * b;
      D[cell * bb + e] = S[e];
      if (i > 0) {   // M_i = S_i^{-1} L_i
        double acc = 0.0;
        for (int k = 0; k < b; ++k) acc = fma(S[k * b + r], Lb[c * b + k], acc);
        L[cell * bb + e] = acc;
      }
      if (i + 1 < nx) {   // G_i = S_i^{-1} U_i (G_{i-1} is no longer read)
        double acc = 0.0;
        for (int k = 0; k < b; ++k) acc = fma(S[k * b + r], Ub[c * b + k], acc);
        G[e] = acc;
        U[cell * bb + e] = acc;
      }
    }
    __syncthreads();
  }
  if (tid == 0) fail[line] = ok ? 0 : 1;
}

// x = P^{-1} r along each line (x may be r): forward y_i = S_i^{-1} r_i -
// M_i y_{i-1}, backward x_i = y_i - G_i x_{i+1}.  One 64-lane workgroup (one
// wavefront, so LDS ordering needs only a wavefront-level fence) per line,
// lane = row.  The recurrence is a chain of dependent block products, so the
// kernel is bound by latency: each lane keeps its rows of the next cell's
// blocks in registers (BM >= b entries per block), loaded while the current
// cell is worked on, and the products run as four interleaved partial sums.
__device__ __forceinline__ void xl_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int BM>
__device__ __forceinline__ double xl_rowdot(const double (&m)[BM], const double* v, int b) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < BM; ++k)
    if (k < b) a[k & 3] = fma(m[k], v[k], a[k & 3]);
  return (a[0] + a[1]) + (a[2] + a[3]);
}

template <int BM>
__device__ __forceinline__ void xl_load_row(double (&m)[BM], const double* blk, int row, int b, bool on) {
#pragma unroll
  for (int k = 0; k < BM; ++k) m[k] = (on && k < b) ? blk[k * b + row] : 0.0;
}

template <int BM>
__global__ __launch_bounds__(kXlApplyThreads) void xl_apply_kernel(const double* r, double* x,
                                                                  const double* __restrict__ D,
                                                                  const double* __restrict__ L,
                                                                  const double* __restrict__ U, int nx, int b) {
  __shared__ double v[kXlMaxBlock];
  const int row = threadIdx.x;
  const bool on = row < b;
  const int line = blockIdx.x;
  const int64_t bb = (int64_t)b * b;
  const int64_t c0 = (int64_t)line * nx;
  double mL[BM] = {}, mD[BM], nL[BM] = {}, nD[BM] = {};
  xl_load_row<BM>(mD, D + c0 * bb, row, b, on);
  double rc = on ? r[c0 * b + row] : 0.0;
  double prev = 0.0;     // y_{i-1} at this row
  for (int i = 0; i < nx; ++i) {
    const int64_t cell = c0 + i;
    // the next cell's rows and right-hand side, in flight during this cell
    double rn = 0.0;
    if (i + 1 < nx) {
      xl_load_row<BM>(nL, L + (cell + 1) * bb, row, b, on);
      xl_load_row<BM>(nD, D + (cell + 1) * bb, row, b, on);
      rn = on ? r[(cell + 1) * b + row] : 0.0;
    }
    xl_wave_sync();
    v[row] = rc;
    xl_wave_sync();
    double y = xl_rowdot<BM>(mD, v, b);
    if (i > 0) {
      xl_wave_sync();
      v[row] = prev;
      xl_wave_sync();
      y -= xl_rowdot<BM>(mL, v, b);
    }
    if (on) x[cell * b + row] = y;
    prev = y;
#pragma unroll
    for (int k = 0; k < BM; ++k) {
      mL[k] = nL[k];
      mD[k] = nD[k];
    }
    rc = rn;
  }
  // backward: prev holds x_{nx-1} = y_{nx-1}
  double mG[BM] = {}, nG[BM] = {};
  if (nx >= 2) xl_load_row<BM>(mG, U + (c0 + nx - 2) * bb, row, b, on);
  double yc = (nx >= 2 && on) ? x[(c0 + nx - 2) * b + row] : 0.0;
  for (int i = nx - 2; i >= 0; --i) {
    const int64_t cell = c0 + i;
    double yn = 0.0;
    if (i >= 1) {
      xl_load_row<BM>(nG, U + (cell - 1) * bb, row, b, on);
      yn = on ? x[(cell - 1) * b + row] : 0.0;
    }
    xl_wave_sync();
    v[row] = prev;
    xl_wave_sync();
    prev = yc - xl_rowdot<BM>(mG, v, b);
    if (on) x[cell * b + row] = prev;
#pragma unroll
    for (int k = 0; k < BM; ++k) mG[k] = nG[k];
    yc = yn;
  }
}

// The same recurrences for b <= 16 with every lane of the wavefront busy and
// the loads kept well ahead of the chain.  Four lanes share a row (lane =
// 4 row + q); lane q holds the entries k = q, q + 4, q + 8, q + 12 of its
// row of each block, so its product over them is the partial sum a[q] of
// xl_rowdot, and two butterfly exchanges inside the lane quad give every
// lane of the row (a0 + a1) + (a2 + a3): the same rounding as the kernel
// above, bit for bit.  The products S_i^{-1} r_i come first, for every cell
// at once (xl_diag16_kernel, into x); the sweep then keeps the rows of the
// next kXlRing cells in a ring of registers (a loop unrolled by kXlRing, so
// every slot index is a constant): the loads of cell i + kXlRing are issued
// as cell i is done, to hide their latency behind the next steps (the
// compiler's wait counts for loads in flight across the loop's back edge
// are conservative, so the lookahead it keeps is shorter; the steps
// themselves, an LDS exchange, four dependent FMAs and two DPP exchanges,
// bound the sweep).
#ifndef VFP_XL_RING
#define VFP_XL_RING 12
#endif
constexpr int kXlRing = VFP_XL_RING;
constexpr int kXlDiagWaves = 4;     // wavefronts per workgroup of xl_diag16_kernel
constexpr size_t kXlLineLds = 60 * 1024;   // dynamic LDS for a line's rows (under the 64 KB default)
constexpr int kXlDiagPerWave = 4;   // cells per wavefront

// v from lane (lane ^ 1) and (lane ^ 2) of the same quad (DPP quad_perm)
template <int CTRL>
__device__ __forceinline__ double xl_quad_swap(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double xl_quad_sum(double a) {
  a = a + xl_quad_swap<0xB1>(a);   // quad_perm [1, 0, 3, 2]: a0 + a1, a2 + a3
  return a + xl_quad_swap<0x4E>(a);  // quad_perm [2, 3, 0, 1]
}

// x_i = S_i^{-1} r_i for every cell (x may be r: a wavefront reads its
// cells' r before any of its lanes stores), kXlDiagPerWave cells per
// wavefront with every load issued before the first product
__global__ __launch_bounds__(64 * kXlDiagWaves) void xl_diag16_kernel(const double* r, double* x,
                                                                     const double* __restrict__ D, int64_t ncells,
                                                                     int b) {
  const int lane = threadIdx.x & 63;
  const int64_t first = ((int64_t)blockIdx.x * kXlDiagWaves + (threadIdx.x >> 6)) * kXlDiagPerWave;
  const int row = lane >> 2, q = lane & 3;
  const bool on = row < b;
  const int rr = on ? row : 0;
  const int64_t bb = (int64_t)b * b;
  double dm[kXlDiagPerWave][4], rv[kXlDiagPerWave][4];
#pragma unroll
  for (int c = 0; c < kXlDiagPerWave; ++c) {
    const int64_t cell = first + c < ncells ? first + c : ncells - 1;   // a cell that exists
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = (q + 4 * m < b) ? q + 4 * m : 0;
      dm[c][m] = D[cell * bb + (int64_t)k * b + rr];
      rv[c][m] = r[cell * b + k];
    }
  }
  double out[kXlDiagPerWave];
#pragma unroll
  for (int c = 0; c < kXlDiagPerWave; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (q + 4 * m < b) acc = fma(dm[c][m], rv[c][m], acc);
    out[c] = xl_quad_sum(acc);
  }
#pragma unroll
  for (int c = 0; c < kXlDiagPerWave; ++c)
    if (q == 0 && on && first + c < ncells) x[(first + c) * b + row] = out[c];
}

// the two sweeps; x holds S_i^{-1} r_i on entry and P^{-1} r on exit.
// LY: the line's y (then x) rows stay in LDS (nx b doubles of dynamic LDS)
// and go to x in one coalesced pass at the end, so the recurrences issue no
// global stores and the backward ring holds only the rows of G.
template <bool LY>
__global__ __launch_bounds__(kXlApplyThreads) void xl_apply16_kernel(double* x, const double* __restrict__ M,
                                                                    const double* __restrict__ U, int nx, int b) {
  __shared__ double v[16];
  extern __shared__ double ys[];
  const int lane = threadIdx.x;
  const int row = lane >> 2, q = lane & 3;
  const bool on = row < b;
  const int line = blockIdx.x;
  const int64_t bb = (int64_t)b * b;
  const int64_t c0 = (int64_t)line * nx;
  if (lane < 16) v[lane] = 0.0;
  double p1[kXlRing][4], pv[kXlRing];
  // cell i of the line into a ring slot: the row of block A and the row's
  // entry of vector w.  The loads are unconditional, so that no branch
  // stands between a load and its use and the in-order wait counts stay
  // exact; an index outside the line, the block or the rows is clamped to an
  // entry that exists, and what is read there is never used (entries k >= b
  // are skipped in prod, rows >= b and cells past the line's end are not
  // stored).
  const int rr = on ? row : 0;
  auto fetch_rows = [&](double (&a)[4], const double* A, int i) {
    const int64_t cell = c0 + ((i >= 0 && i < nx) ? i : 0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = (q + 4 * m < b) ? q + 4 * m : 0;
      a[m] = A[cell * bb + (int64_t)k * b + rr];
    }
  };
  auto fetch = [&](double (&a)[4], double& w, const double* A, const double* vec, int i) {
    fetch_rows(a, A, i);
    w = vec[(c0 + ((i >= 0 && i < nx) ? i : 0)) * b + rr];
  };
  auto prod = [&](const double (&a)[4]) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (q + 4 * m < b) acc = fma(a[m], v[q + 4 * m], acc);
    return xl_quad_sum(acc);
  };
  // forward: y_i = c_i - M_i y_{i-1}; p1 = M rows, pv = c (read from x, where
  // y_i may then go: each cell's c is read kXlRing cells before its y is
  // stored)
#pragma unroll
  for (int s = 0; s < kXlRing; ++s) fetch(p1[s], pv[s], M, x, s);
  double prev = 0.0;
  for (int i0 = 0; i0 < nx; i0 += kXlRing) {
#pragma unroll
    for (int s = 0; s < kXlRing; ++s) {
      const int i = i0 + s;
      if (i < nx) {
        double y = pv[s];
        if (i > 0) {
          xl_wave_sync();
          if (q == 0 && on) v[row] = prev;
          xl_wave_sync();
          y -= prod(p1[s]);
        }
        if (q == 0 && on) {
          if constexpr (LY)
            ys[i * b + row] = y;
          else
            x[(c0 + i) * b + row] = y;
        }
        prev = y;
      }
      fetch(p1[s], pv[s], M, x, i + kXlRing);
    }
  }
  // backward: x_i = y_i - G_i x_{i+1}, i = nx-2 .. 0; p1 = G rows (and pv =
  // y from x without LY).  The y rows were stored above by the quad's lane 0
  // and are read back by all four lanes: order those stores before these
  // loads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
  for (int s = 0; s < kXlRing; ++s) {
    if constexpr (LY)
      fetch_rows(p1[s], U, nx - 2 - s);
    else
      fetch(p1[s], pv[s], U, x, nx - 2 - s);
  }
  for (int j0 = 0; j0 < nx - 1; j0 += kXlRing) {
#pragma unroll
    for (int s = 0; s < kXlRing; ++s) {
      const int i = nx - 2 - (j0 + s);
      if (i >= 0) {
        xl_wave_sync();
        if (q == 0 && on) v[row] = prev;
        xl_wave_sync();
        if constexpr (LY) {
          prev = ys[i * b + rr] - prod(p1[s]);
          if (q == 0 && on) ys[i * b + row] = prev;
        } else {
          prev = pv[s] - prod(p1[s]);
          if (q == 0 && on) x[(c0 + i) * b + row] = prev;
        }
      }
      if constexpr (LY)
        fetch_rows(p1[s], U, i - kXlRing);
      else
        fetch(p1[s], pv[s], U, x, i - kXlRing);
    }
  }
  if constexpr (LY) {
    xl_wave_sync();
    for (int e = lane; e < nx * b; e += kXlApplyThreads) x[c0 * b + e] = ys[e];
  }
}

// The factorisation for b <= 16 by one wavefront per line: the same
// operations in the same order as xl_factor_kernel (so the same blocks, bit
// for bit), ordered by wavefront-level fences instead of workgroup barriers,
// each lane holding 4 of the 256 entries of a block, and the pivot found by
// a DPP arg-max within the first 16-lane row.
template <int CTRL>
__device__ __forceinline__ int xl_dpp_int(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

// arg-max of a over the lanes of each 16-lane row (ties to the smaller
// index), in every lane of the row
__device__ __forceinline__ void xl_row16_argmax(double& a, int& idx) {
#define XL_ARGMAX_STEP(CTRL)                                          \
  {                                                                   \
    const double a2 = xl_quad_swap<CTRL>(a);                          \
    const int i2 = xl_dpp_int<CTRL>(idx);                             \
    if (a2 > a || (a2 == a && i2 < idx)) {                            \
      a = a2;                                                         \
      idx = i2;                                                       \
    }                                                                 \
  }
  XL_ARGMAX_STEP(0x121)   // row_ror:1
  XL_ARGMAX_STEP(0x122)   // row_ror:2
  XL_ARGMAX_STEP(0x124)   // row_ror:4
  XL_ARGMAX_STEP(0x128)   // row_ror:8
#undef XL_ARGMAX_STEP
}

__global__ __launch_bounds__(64) void xl_factor16_kernel(double* D, double* L, double* U, int nx, int b,
                                                        int* fail) {
  __shared__ double S[256], G[256], Lb[256], Ub[256];
  __shared__ int perm[16];
  const int lane = threadIdx.x;
  const int line = blockIdx.x;
  const int bb = b * b;
  bool ok = true;
  double nD[4], nL[4], nU[4];
  auto load_blocks = [&](int i) {
    const int64_t base = ((int64_t)line * nx + i) * bb;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      const bool in = i < nx && e < bb;
      nD[t] = in ? D[base + e] : 0.0;
      nL[t] = in ? L[base + e] : 0.0;
      nU[t] = in ? U[base + e] : 0.0;
    }
  };
  load_blocks(0);
  for (int i = 0; i < nx; ++i) {
    const int64_t cell = (int64_t)line * nx + i;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      if (e < bb) {
        S[e] = nD[t];
        Lb[e] = nL[t];
        Ub[e] = nU[t];
      }
    }
    xl_wave_sync();
    load_blocks(i + 1);
    if (i > 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int e = lane + 64 * t;
        if (e < bb) {
          const int c = e / b, r = e - c * b;
          double acc = 0.0;
          for (int k = 0; k < b; ++k) acc = fma(Lb[k * b + r], G[c * b + k], acc);
          S[e] -= acc;
        }
      }
      xl_wave_sync();
    }
    // Gauss-Jordan with partial pivoting (as xl_invert)
    for (int k = 0; k < b; ++k) {
      double a = (lane >= k && lane < b) ? fabs(S[k * b + lane]) : -1.0;
      int idx = lane;
      xl_row16_argmax(a, idx);
      const int p = __builtin_amdgcn_readfirstlane(idx);
      if (lane == 0) perm[k] = p;
      if (p != k && lane < b) {
        const double t0 = S[lane * b + k];
        S[lane * b + k] = S[lane * b + p];
        S[lane * b + p] = t0;
      }
      xl_wave_sync();
      const double pv = S[k * b + k];
      if (pv == 0.0) ok = false;
      const double ipv = 1.0 / pv;
      xl_wave_sync();
      if (lane < b) S[lane * b + k] = (lane == k) ? ipv : S[lane * b + k] * ipv;
      xl_wave_sync();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int e = lane + 64 * t;
        if (e < bb) {
          const int c = e / b, r = e - c * b;
          if (r != k && c != k) S[e] = fma(-S[k * b + r], S[c * b + k], S[e]);
        }
      }
      xl_wave_sync();
      if (lane < b && lane != k) S[k * b + lane] = -S[k * b + lane] * ipv;
      xl_wave_sync();
    }
    for (int k = b - 1; k >= 0; --k) {
      const int p = perm[k];
      if (p != k && lane < b) {
        const double t0 = S[k * b + lane];
        S[k * b + lane] = S[p * b + lane];
        S[p * b + lane] = t0;
      }
      xl_wave_sync();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      if (e < bb) {
        const int c = e / b, r = e - c * b;
        D[cell * bb + e] = S[e];
        if (i > 0) {
          double acc = 0.0;
          for (int k = 0; k < b; ++k) acc = fma(S[k * b + r], Lb[c * b + k], acc);
          L[cell * bb + e] = acc;
        }
        if (i + 1 < nx) {
          double acc = 0.0;
          for (int k = 0; k < b; ++k) acc = fma(S[k * b + r], Ub[c * b + k], acc);
          G[e] = acc;
          U[cell * bb + e] = acc;
        }
      }
    }
    xl_wave_sync();
  }
  if (lane == 0) fail[line] = ok ? 0 : 1;
}

}  // namespace

void xl_probe_set(double* v, int64_t ndofs, int nx, int b, int wrapc, int color, int j, hipStream_t s) {
  const int64_t blocks = (ndofs + kXlThreads - 1) / kXlThreads;
  hipLaunchKernelGGL(xl_probe_set_kernel, dim3((unsigned)blocks), dim3(kXlThreads), 0, s, v, ndofs, nx, b, wrapc,
                     color, j);
}

void xl_probe_get(const double* w, double* D, double* L, double* U, int64_t ndofs, int nx, int b, int wrapc,
                  int color, int j, hipStream_t s) {
  const int64_t blocks = (ndofs + kXlThreads - 1) / kXlThreads;
  hipLaunchKernelGGL(xl_probe_get_kernel, dim3((unsigned)blocks), dim3(kXlThreads), 0, s, w, D, L, U, ndofs, nx, b,
                     wrapc, color, j);
}

void xl_factor(double* D, double* L, double* U, int nlines, int nx, int b, int* fail, hipStream_t s) {
  if (b <= 16)
    hipLaunchKernelGGL(xl_factor16_kernel, dim3(nlines), dim3(64), 0, s, D, L, U, nx, b, fail);
  else
    hipLaunchKernelGGL(xl_factor_kernel, dim3(nlines), dim3(kXlThreads), 0, s, D, L, U, nx, b, fail);
}

void xl_apply(const double* r, double* x, const double* D, const double* L, const double* U, int nlines, int nx,
              int b, bool rowwise, hipStream_t s) {
  if (b <= 16 && !rowwise) {
    const int64_t ncells = (int64_t)nlines * nx;
    constexpr int per_block = kXlDiagWaves * kXlDiagPerWave;
    hipLaunchKernelGGL(xl_diag16_kernel, dim3((unsigned)((ncells + per_block - 1) / per_block)),
                       dim3(64 * kXlDiagWaves), 0, s, r, x, D, ncells, b);
    // the line's rows in LDS where they fit the default dynamic LDS limit
    const size_t ly = (size_t)nx * b * sizeof(double);
    if (ly <= kXlLineLds)
      hipLaunchKernelGGL(xl_apply16_kernel<true>, dim3(nlines), dim3(kXlApplyThreads), ly, s, x, L, U, nx, b);
    else
      hipLaunchKernelGGL(xl_apply16_kernel<false>, dim3(nlines), dim3(kXlApplyThreads), 0, s, x, L, U, nx, b);
  }
  else if (b <= 16)
    hipLaunchKernelGGL(xl_apply_kernel<16>, dim3(nlines), dim3(kXlApplyThreads), 0, s, r, x, D, L, U, nx, b);
  else if (b <= 32)
    hipLaunchKernelGGL(xl_apply_kernel<32>, dim3(nlines), dim3(kXlApplyThreads), 0, s, r, x, D, L, U, nx, b);
  else
    hipLaunchKernelGGL(xl_apply_kernel<kXlMaxBlock>, dim3(nlines), dim3(kXlApplyThreads), 0, s, r, x, D, L, U, nx,
                       b);
}

}  // namespace vfp
