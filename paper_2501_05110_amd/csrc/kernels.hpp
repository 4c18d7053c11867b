// HIP kernels for the DG x spherical-harmonic operator (gfx950 / CDNA4).
//
// Mapping.  One lane owns one (cell, lms) pair and keeps the cell's (k+1)^D
// nodal values of that coefficient in registers, so every basis contraction
// (interpolation to the Gauss points, test-function contraction with the
// inverse mass folded in, face interpolation and lift) is a compile-time
// sequence of FMAs with no cross-lane traffic.  The lms mixing by the sparse
// spherical-harmonic matrices needs values of other coefficients of the same
// cell: those are exchanged through LDS.  A 256-lane workgroup holds
// 256 / n cells (n = (l_max+1)^2).
//
// Operator (per cell, after the inverse mass matrix, which factorises over
// axes and cancels the Jacobian):
//   L = -T (G f_q) + sum_a (2/h_a) T'_a (F^a_q) + face lifts + M^{-1} h
// with f_q the state at the Gauss points, F^a = beta^a f, G = (R - div beta) f,
// T the tensor product of the 1-D test matrices tst (and dtst along axis a).
#pragma once
#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace vfp {

// One copy per translation unit (no relocatable device code); the host fills
// every copy that launches kernels reading it (upload_basis).
static __constant__ Basis1D c_basis[kMaxK];

// A generic pointer known to address global memory, retyped into the global
// address space: loads and stores through it are global (not flat) memory
// instructions, also for pointers that were themselves loaded from memory.
template <class T>
using global_ptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ global_ptr<T> gp(T* p) {
  return (global_ptr<T>)p;
}

// Moves within a row of 16 lanes (DPP), on the two
// 32-bit halves of a double.  CTRL: 0xB1 / 0x4E quad permutes (lane ^ 1,
// lane ^ 2), 0x124 / 0x128 rotations of the row by 4 / 8 lanes.  Every lane
// of the row must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The sum of v over the 16 lanes of this lane's DPP row, in every lane of it
// (a fixed order: pairs, quads, quad pairs, then the two halves).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x124>(v);
  return v + dpp_move<0x128>(v);
}

template <int B, int E>
struct IPow { static constexpr int v = B * IPow<B, E - 1>::v; };
template <int B>
struct IPow<B, 0> { static constexpr int v = 1; };

// Apply a (K1 x K1) matrix M along axis AX of a D-dimensional tensor with K1
// points per axis: out[.., q, ..] = sum_j M[q][j] in[.., j, ..].
template <int D, int K1, int AX>
__device__ __forceinline__ void sweep(const double* in, double* out, const double (&M)[kMaxK1][kMaxK1]) {
  constexpr int NB = IPow<K1, D>::v;
  constexpr int st = IPow<K1, AX>::v;
#pragma unroll
  for (int idx = 0; idx < NB; ++idx) {
    const int q = (idx / st) % K1;
    const int base = idx - q * st;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < K1; ++j) acc = fma(M[q][j], in[base + j * st], acc);
    out[idx] = acc;
  }
}

// In-place form of sweep: each line of K1 values along AX is replaced by M
// times itself (one line of temporaries instead of a second tensor).
template <int D, int K1, int AX>
__device__ __forceinline__ void sweep_ip(double* v, const double (&M)[kMaxK1][kMaxK1]) {
  constexpr int NB = IPow<K1, D>::v;
  constexpr int st = IPow<K1, AX>::v;
#pragma unroll
  for (int base = 0; base < NB; ++base) {
    if ((base / st) % K1 != 0) continue;
    double t[K1];
#pragma unroll
    for (int j = 0; j < K1; ++j) t[j] = v[base + j * st];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < K1; ++j) acc = fma(M[q][j], t[j], acc);
      v[base + q * st] = acc;
    }
  }
}

// Contract a quadrature-point tensor with the test matrices: axis DER uses
// dtst, the others tst (DER < 0: tst everywhere).  out += scale * result.
template <int D, int K, int DER>
__device__ __forceinline__ void contract_add(const double* g, double* out, double scale) {
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  const Basis1D& bs = c_basis[K - 1];
  double t0[NB], t1[NB];
  sweep<D, K1, 0>(g, t0, DER == 0 ? bs.dtst : bs.tst);
  if constexpr (D == 1) {
#pragma unroll
    for (int i = 0; i < NB; ++i) out[i] = fma(scale, t0[i], out[i]);
  } else if constexpr (D == 2) {
    sweep<D, K1, 1>(t0, t1, DER == 1 ? bs.dtst : bs.tst);
#pragma unroll
    for (int i = 0; i < NB; ++i) out[i] = fma(scale, t1[i], out[i]);
  } else {
    sweep<D, K1, 1>(t0, t1, DER == 1 ? bs.dtst : bs.tst);
    sweep<D, K1, 2>(t1, t0, DER == 2 ? bs.dtst : bs.tst);
#pragma unroll
    for (int i = 0; i < NB; ++i) out[i] = fma(scale, t0[i], out[i]);
  }
}

// contract_add with tst on every axis, in place: g is overwritten.
template <int D, int K>
__device__ __forceinline__ void contract_add_ip(double* g, double* out, double scale) {
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  const Basis1D& bs = c_basis[K - 1];
  sweep_ip<D, K1, 0>(g, bs.tst);
  if constexpr (D > 1) sweep_ip<D, K1, (D > 1 ? 1 : 0)>(g, bs.tst);
  if constexpr (D > 2) sweep_ip<D, K1, (D > 2 ? 2 : 0)>(g, bs.tst);
#pragma unroll
  for (int i = 0; i < NB; ++i) out[i] = fma(scale, g[i], out[i]);
}

// Interpolate nodal values to the Gauss points in place (all axes).
template <int D, int K>
__device__ __forceinline__ void interp_ip(double* v) {
  constexpr int K1 = K + 1;
  const Basis1D& bs = c_basis[K - 1];
  sweep_ip<D, K1, 0>(v, bs.phi);
  if constexpr (D > 1) sweep_ip<D, K1, (D > 1 ? 1 : 0)>(v, bs.phi);
  if constexpr (D > 2) sweep_ip<D, K1, (D > 2 ? 2 : 0)>(v, bs.phi);
}

// Interpolate nodal values to the Gauss points (all axes).
template <int D, int K>
__device__ __forceinline__ void interp(const double* w, double* f) {
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  const Basis1D& bs = c_basis[K - 1];
  if constexpr (D == 1) {
    sweep<1, K1, 0>(w, f, bs.phi);
  } else if constexpr (D == 2) {
    double t[NB];
    sweep<2, K1, 0>(w, t, bs.phi);
    sweep<2, K1, 1>(t, f, bs.phi);
  } else {
    double t[NB];
    sweep<3, K1, 0>(w, f, bs.phi);
    sweep<3, K1, 1>(f, t, bs.phi);
    sweep<3, K1, 2>(t, f, bs.phi);
  }
}

// Interpolate nodal values to the Gauss points with the derivative l_j' along
// axis DER and l_j along the others (reference coordinates).
template <int D, int K, int DER>
__device__ __forceinline__ void interp_deriv(const double* w, double* f) {
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  const Basis1D& bs = c_basis[K - 1];
  if constexpr (D == 1) {
    sweep<1, K1, 0>(w, f, bs.dphi);
  } else if constexpr (D == 2) {
    double t[NB];
    sweep<2, K1, 0>(w, t, DER == 0 ? bs.dphi : bs.phi);
    sweep<2, K1, 1>(t, f, DER == 1 ? bs.dphi : bs.phi);
  } else {
    double t[NB];
    sweep<3, K1, 0>(w, f, DER == 0 ? bs.dphi : bs.phi);
    sweep<3, K1, 1>(f, t, DER == 1 ? bs.dphi : bs.phi);
    sweep<3, K1, 2>(t, f, DER == 2 ? bs.dphi : bs.phi);
  }
}

// v <- (M1 x ... x M1) v (INV: the inverse) on the reference cell, in place;
// the caller supplies the Jacobian factor.
template <int D, int K, bool INV>
__device__ __forceinline__ void ref_mass(double* v) {
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  const Basis1D& bs = c_basis[K - 1];
  const double(&Mm)[kMaxK1][kMaxK1] = INV ? bs.imass : bs.mass;
  double t[NB];
  sweep<D, K1, 0>(v, t, Mm);
  if constexpr (D == 1) {
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = t[i];
  } else if constexpr (D == 2) {
    sweep<D, K1, 1>(t, v, Mm);
  } else {
    sweep<D, K1, 1>(t, v, Mm);
    sweep<D, K1, 2>(v, t, Mm);
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = t[i];
  }
}

// Jacobian of the affine map of cell ic: prod_a h_a / 2.
template <int D>
__device__ __forceinline__ double cell_jacobian(const MeshArgs& M, const int* ic) {
  double j = 1.0;
#pragma unroll
  for (int a = 0; a < D; ++a) j /= M.s2h[a][ic[a]];
  return j;
}

// Face helpers: a face normal to axis AX has (K+1)^(D-1) points; face index
// fi enumerates the remaining axes in increasing order, lowest fastest.
template <int D, int K, int AX>
__device__ __forceinline__ int face_node_to_cell_node(int fi, int jn) {
  constexpr int K1 = K + 1;
  int idx = 0, st = 1, rem = fi;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int j;
    if (a == AX) {
      j = jn;
    } else {
      j = rem % K1;
      rem /= K1;
    }
    idx += j * st;
    st *= K1;
  }
  return idx;
}

template <int D, int K>
__device__ __forceinline__ void face_interp(const double* nod, double* pts) {
  constexpr int K1 = K + 1;
  const Basis1D& bs = c_basis[K - 1];
  if constexpr (D == 1) {
    pts[0] = nod[0];
  } else if constexpr (D == 2) {
    sweep<1, K1, 0>(nod, pts, bs.phi);
  } else {
    double t[K1 * K1];
    sweep<2, K1, 0>(nod, t, bs.phi);
    sweep<2, K1, 1>(t, pts, bs.phi);
  }
}

template <int D, int K>
__device__ __forceinline__ void face_test(const double* pts, double* nod) {
  constexpr int K1 = K + 1;
  const Basis1D& bs = c_basis[K - 1];
  if constexpr (D == 1) {
    nod[0] = pts[0];
  } else if constexpr (D == 2) {
    sweep<1, K1, 0>(pts, nod, bs.tst);
  } else {
    double t[K1 * K1];
    sweep<2, K1, 0>(pts, t, bs.tst);
    sweep<2, K1, 1>(t, nod, bs.tst);
  }
}

}  // namespace vfp
