// Fused operator / Runge-Kutta stage kernel:  w_out = alpha u + beta L(w_in)
// with L(w) = M^{-1}(h - D w) of eq. definition-mass-and-dg-matrix.
//
// The same template with ADJ = true applies the adjoint operator in the
// variable mu = M^{-1} lambda:  K mu = -M^{-1} D^T mu, so that the Euclidean
// transpose of the linear part of L is  L^T = M K M^{-1}.  Writing D^T out per
// cell (transpose of the volume and face blocks of eq.
// definition-mass-and-dg-matrix with the upwind flux of eq.
// definition-upwind-flux):
//   volume:  K mu = -T((R - div beta)^T mu_q) + sum_a (2/h_a) T(beta^a d_a mu_q)
//            (beta^a symmetric; d_a mu_q the derivative interpolation)
//   faces :  with B = n.beta on a face from T1 (below) to T2 (above) and
//            d = mu(own trace) - mu(other trace):
//            T1 lifts -(2/h) B_+ d,  T2 lifts +(2/h) B_- d,
//            zero inflow: other trace 0; "continuous": B mu(own trace).
// The face part is the forward flux routine fed (F1, F2) = (d, 0) on the hi
// side and (0, d) on the lo side, or (own, own) at a continuous boundary.
//
// This header holds the general kernel templates; each stage_gen_*.hip
// instantiates one family of them (so that the families compile in
// parallel), and stage.hip picks the family at run time.
#pragma once

#include "kernels.hpp"
#include "launch.hpp"


namespace vfp {

namespace gen {

constexpr int kThreads = 256;

template <int N>
struct Tile {
  static constexpr int cpb = (kThreads / N) > 0 ? kThreads / N : 1;
};

// Per-lane copy of the sparse rows this lane needs.
template <int LMAX>
struct LaneRows {
  int axc[2];
  double axv[2], g1v[2];
  int axxc[2];
  double axxv[3], g2v[3];
  double g1tv[2], g2tv[3];
  int omc[3][2];
  double omv[3][2];
  int ayzc[2][4];
  double ayzv[2][4];
  double cv;
  int mem[LMAX + 1];
  double wrow[LMAX + 1], wcol[LMAX + 1];
  double lam;
};

template <int LMAX>
__device__ __forceinline__ void load_rows(const RowTables& T, int r, LaneRows<LMAX>& R) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    R.axc[s] = T.ax_col[s * N + r];
    R.axv[s] = T.ax_val[s * N + r];
    R.g1v[s] = T.g1_val[s * N + r];
    R.g1tv[s] = T.g1t_val[s * N + r];
    R.axxc[s] = T.axx_col[s * N + r];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    R.axxv[s] = T.axx_val[s * N + r];
    R.g2v[s] = T.g2_val[s * N + r];
    R.g2tv[s] = T.g2t_val[s * N + r];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      R.omc[c][s] = T.om_col[(c * 2 + s) * N + r];
      R.omv[c][s] = T.om_val[(c * 2 + s) * N + r];
    }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      R.ayzc[c][s] = T.ayz_col[(c * 4 + s) * N + r];
      R.ayzv[c][s] = T.ayz_val[(c * 4 + s) * N + r];
    }
  R.cv = T.c_val[r];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    R.mem[i] = T.blk_mem[i * N + r];
    R.wrow[i] = T.w_row[i * N + r];
    R.wcol[i] = T.w_col[i * N + r];
  }
  R.lam = T.lam[r];
}

// A^c f at one point, from the point's coefficient row in LDS.
template <int LMAX>
__device__ __forceinline__ double dir_apply(const LaneRows<LMAX>& R, int c, const double* p) {
  if (c == 0) return R.axv[0] * p[R.axc[0]] + R.axv[1] * p[R.axc[1]];
  const int k = c - 1;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = fma(R.ayzv[k][s], p[R.ayzc[k][s]], acc);
  return acc;
}

template <int LMAX>
__device__ __forceinline__ double om_apply(const LaneRows<LMAX>& R, int c, const double* p) {
  return R.omv[c][0] * p[R.omc[c][0]] + R.omv[c][1] * p[R.omc[c][1]];
}

struct PointScalars {
  double V, iV, idiv, ig;   // momentum-dependent
  double ca, cu;            // beta^p = -(a ca A^x + U' cu (A^x A^x)_t) along the momentum axis
  double U, dU, a;          // planar flow (x)
  double Up[3], divU;       // flow at the point (every flow kind) and its divergence over the run's axes
};

// Flow kinds of the general kernels: uniform U, a planar profile U_x(x), or
// U and div U at every volume point with the normal component of U at every
// face point.
enum : int { FLOW_UNIFORM = 0, FLOW_XPROF = 1, FLOW_POINTS = 2 };

template <int D, int K, bool MOM, int FL>
__device__ __forceinline__ PointScalars point_scalars(const FieldArgs& F, const int* ic, int q, int cell) {
  constexpr int K1 = K + 1;
  constexpr bool XPROF = FL == FLOW_XPROF;
  PointScalars s;
  if constexpr (MOM) {
    constexpr int stp = IPow<K1, D - 1>::v;
    const int ip = ic[D - 1] * K1 + (q / stp) % K1;
    s.V = F.V_vol[ip];
    s.iV = F.iV_vol[ip];
    s.idiv = F.idiv_vol[ip];
    s.ig = F.ig_vol[ip];
    s.ca = F.ca_vol[ip];
    s.cu = F.cu_vol[ip];
  } else {
    s.V = F.V0;
    s.iV = F.iV0;
    s.idiv = 0.0;
    s.ig = F.ig0;
    s.ca = s.cu = 0.0;
  }
  if constexpr (XPROF) {
    const int ix = ic[0] * K1 + q % K1;
    s.U = F.u_vol[ix];
    s.dU = F.du_vol[ix];
    s.a = F.a_vol[ix];
  } else {
    s.U = F.U[0];
    s.dU = 0.0;
    s.a = 0.0;
  }
  if constexpr (FL == FLOW_POINTS) {
    constexpr int NB = IPow<K1, D>::v;
    const double* up = F.u_pts + ((size_t)cell * NB + q) * 4;
    s.Up[0] = up[0];
    s.Up[1] = up[1];
    s.Up[2] = up[2];
    s.divU = up[3];
  } else {
    s.Up[0] = s.U;
    s.Up[1] = F.U[1];
    s.Up[2] = F.U[2];
    s.divU = s.dU;
  }
  return s;
}

template <int D, int K, int LMAX, bool MOM, int FL, int AX, bool ADJ>
__device__ __forceinline__ void face_axis(const KernelArgs& A, const LaneRows<LMAX>& R,
                                          double* shc, const double* w, double* res,
                                          const int* ic, int cell, int r, bool act, bool in_grp) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  constexpr int NF = IPow<K1, D - 1>::v;
  constexpr bool IS_P = MOM && (AX == D - 1);
  constexpr bool IS_X = (FL == FLOW_XPROF) && (AX == 0);
  constexpr bool IS_PT = (FL == FLOW_POINTS) && !IS_P;
  const Basis1D& bs = c_basis[K - 1];
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;
  int stride = 1;
#pragma unroll
  for (int b = 0; b < AX; ++b) stride *= M.n[b];

#pragma unroll
  for (int side = 0; side < 2; ++side) {
    double own[NF], nbr[NF];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) own[fi] = w[face_node_to_cell_node<D, K, AX>(fi, side ? K : 0)];
    const int ia = ic[AX], na = M.n[AX];
    int ni = side ? ia + 1 : ia - 1;
    const int bc = side ? M.bc_hi[AX] : M.bc_lo[AX];
    const bool inside = (ni >= 0 && ni < na);
    if (inside || bc == 0) {
      ni = (ni + na) % na;
      const size_t nb0 = (size_t)(cell + (ni - ia) * stride) * NB * N + r;
#pragma unroll
      for (int fi = 0; fi < NF; ++fi)
        nbr[fi] = act ? A.st.w_in[nb0 + (size_t)face_node_to_cell_node<D, K, AX>(fi, side ? 0 : K) * N]
                      : 0.0;
    } else if (bc == 1) {
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) nbr[fi] = 0.0;
    } else {
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) nbr[fi] = own[fi];
    }
    if constexpr (ADJ) {
      if (inside || bc != 2) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          own[fi] -= nbr[fi];
          nbr[fi] = 0.0;
        }
      }
    }
    // Constant face matrices (a uniform flow at fixed p): the flux is the
    // same linear map of the traces at every point of the face, so it is
    // formed at the Gauss-Lobatto face nodes and lifted with the 1-D
    // lift alone -- the Gauss rule integrates the face mass matrix exactly,
    // so M_F^{-1} int_F phi J equals the nodal J (no interpolation to the face
    // points and no test contraction)
    constexpr bool NODAL = !IS_X && !IS_P && !IS_PT;
    double F1[NF], F2[NF], J[NF];
    if constexpr (NODAL) {
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        F1[fi] = side ? own[fi] : nbr[fi];
        F2[fi] = side ? nbr[fi] : own[fi];
      }
    } else {
      face_interp<D, K>(side ? own : nbr, F1);
      face_interp<D, K>(side ? nbr : own, F2);
    }

    if constexpr (IS_X) {
      // characteristic variables of A^x (constant eigenvectors), speeds
      // U(x_F) + lambda V at each face point
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          shc[fi * N + r] = F1[fi];
          shc[(NF + fi) * N + r] = F2[fi];
        }
      }
      __syncthreads();
      const double UF = F.u_face[ia + side];
      double Jc[NF];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        double c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int j = 0; j <= LMAX; ++j) {
          c1 = fma(R.wcol[j], shc[fi * N + R.mem[j]], c1);
          c2 = fma(R.wcol[j], shc[(NF + fi) * N + R.mem[j]], c2);
        }
        double V;
        if constexpr (MOM) {
          constexpr int stp = IPow<K1, D - 2>::v;    // p is the last face axis
          V = F.V_vol[ic[D - 1] * K1 + (fi / stp) % K1];
        } else {
          V = F.V0;
        }
        const double mu = A.fld.t_adv * (UF + R.lam * V);
        Jc[fi] = fmax(mu, 0.0) * c1 + fmin(mu, 0.0) * c2;
      }
      __syncthreads();
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) shc[fi * N + r] = Jc[fi];
      }
      __syncthreads();
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i <= LMAX; ++i) acc = fma(R.wrow[i], shc[fi * N + R.mem[i]], acc);
        J[fi] = acc;
      }
      __syncthreads();
    } else if constexpr (IS_PT) {
      // flow at the face points: characteristic variables of A^AX (constant
      // dense eigenvectors W, eigenvalues lambda), speeds U^AX(x_F) + lambda V
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          shc[fi * N + r] = F1[fi];
          shc[(NF + fi) * N + r] = F2[fi];
        }
      }
      __syncthreads();
      const double* Wd = A.tab.wd[AX];
      const double lamr = A.tab.lamd[AX][r];
      // flat index of this face among the (N_AX + 1) x prod_{b != AX} N_b faces
      int fidx = 0;
#pragma unroll
      for (int b = D - 1; b >= 0; --b) fidx = fidx * (M.n[b] + (b == AX ? 1 : 0)) + (b == AX ? ia + side : ic[b]);
      const double* uf = F.uf_pts[AX] + (size_t)fidx * NF;
      double Jc[NF];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        double c1 = 0.0, c2 = 0.0;
        for (int j = 0; j < N; ++j) {
          const double wv = Wd[j * N + r];
          c1 = fma(wv, shc[fi * N + j], c1);
          c2 = fma(wv, shc[(NF + fi) * N + j], c2);
        }
        const double mu = A.fld.t_adv * fma(lamr, F.V0, uf[fi]);
        Jc[fi] = fmax(mu, 0.0) * c1 + fmin(mu, 0.0) * c2;
      }
      __syncthreads();
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) shc[fi * N + r] = Jc[fi];
      }
      __syncthreads();
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        double acc = 0.0;
        for (int kk = 0; kk < N; ++kk) acc = fma(Wd[r * N + kk], shc[fi * N + kk], acc);
        J[fi] = acc;
      }
      __syncthreads();
    } else if constexpr (IS_P) {
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          shc[fi * N + r] = F1[fi];
          shc[(NF + fi) * N + r] = F2[fi];
        }
      }
      __syncthreads();
      const int npf = M.n[D - 1] + 1;
      const int pf = ia + side;
      const double iVf = F.iV_face[pf];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        const int ix = ic[0] * K1 + fi % K1;
        const double a1 = -F.t_mom * F.a_vol[ix] * iVf;
        const double a2 = -F.t_mom * F.du_vol[ix] * F.cu_face[pf];
        const int code = F.pf_code[(size_t)pf * (M.n[0] * K1) + ix];
        const double* P1 = shc + fi * N;
        const double* P2 = shc + (NF + fi) * N;
        const double* Pu = (code == -1) ? P1 : P2;
        double jv = a1 * (R.axv[0] * Pu[R.axc[0]] + R.axv[1] * Pu[R.axc[1]]) +
                    a2 * (R.axxv[0] * Pu[R.axxc[0]] + R.axxv[1] * Pu[r] + R.axxv[2] * Pu[R.axxc[1]]);
        if (code >= 0) {
          const double* tb = F.pf_tab + ((size_t)code * N + r) * (LMAX + 1);
#pragma unroll
          for (int i = 0; i <= LMAX; ++i) jv = fma(tb[i], P1[R.mem[i]] - P2[R.mem[i]], jv);
        }
        J[fi] = jv;
      }
      __syncthreads();
    } else {
      // uniform spatial axis: J = (beta (F1+F2) + |beta| (F1-F2)) / 2
      if (in_grp) {
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          shc[fi * N + r] = F1[fi] + F2[fi];
          shc[(NF + fi) * N + r] = F1[fi] - F2[fi];
        }
      }
      __syncthreads();
      const int nfb = A.tab.nfb[AX], nfa = A.tab.nfa[AX];
      const int* fbc = A.tab.fb_col[AX];
      const double* fbv = A.tab.fb_val[AX];
      const int* fac = A.tab.fa_col[AX];
      const double* fav = A.tab.fa_val[AX];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) J[fi] = 0.0;
      for (int s = 0; s < nfb; ++s) {
        const int c = fbc[s * N + r];
        const double v = 0.5 * fbv[s * N + r];
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) J[fi] = fma(v, shc[fi * N + c], J[fi]);
      }
      for (int s = 0; s < nfa; ++s) {
        const int c = fac[s * N + r];
        const double v = 0.5 * fav[s * N + r];
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) J[fi] = fma(v, shc[(NF + fi) * N + c], J[fi]);
      }
      __syncthreads();
    }
    // lift: this cell is T2 of its lo face (+) and T1 of its hi face (-)
    double jn[NF];
    if constexpr (NODAL) {
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) jn[fi] = J[fi];
    } else {
      face_test<D, K>(J, jn);
    }
    const double sc = (side ? -1.0 : 1.0) * M.s2h[AX][ia];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi)
#pragma unroll
      for (int j = 0; j < K1; ++j)
        res[face_node_to_cell_node<D, K, AX>(fi, j)] =
            fma(sc * bs.lift[side][j], jn[fi], res[face_node_to_cell_node<D, K, AX>(fi, j)]);
  }
}

// Adjoint volume flux along axis AX: res += (2/h_AX) T(beta^AX d_AX mu).
// Writes the derivative values to the cell's LDS rows (all lanes of the block
// take part in the barriers).
template <int D, int K, int LMAX, bool MOM, int FL, int AX>
__device__ __forceinline__ void adj_flux_axis(const KernelArgs& A, const LaneRows<LMAX>& R, double* shc,
                                              const double* w, double* res, const int* ic, int cell, int r,
                                              bool in_grp) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int NB = IPow<K + 1, D>::v;
  constexpr bool IS_P = MOM && (AX == D - 1);
  const FieldArgs& F = A.fld;
  double dq[NB], tmp[NB];
  interp_deriv<D, K, AX>(w, dq);
  __syncthreads();
  if (in_grp) {
#pragma unroll
    for (int q = 0; q < NB; ++q) shc[q * N + r] = dq[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double* P = shc + q * N;
    const PointScalars s = point_scalars<D, K, MOM, FL>(F, ic, q, cell);
    if constexpr (IS_P) {
      const double Axf = R.axv[0] * P[R.axc[0]] + R.axv[1] * P[R.axc[1]];
      const double A2f = R.axxv[0] * P[R.axxc[0]] + R.axxv[1] * dq[q] + R.axxv[2] * P[R.axxc[1]];
      tmp[q] = -F.t_mom * (s.a * s.ca * Axf + s.dU * s.cu * A2f);
    } else {
      tmp[q] = F.t_adv * (s.Up[AX] * dq[q] + s.V * dir_apply<LMAX>(R, AX, P));
    }
  }
  contract_add<D, K, -1>(tmp, res, A.mesh.s2h[AX][ic[AX]]);
}

// Waves per SIMD the register allocation aims for: two.  The 3-D, k = 2
// instantiations (27 nodes per lane) need about 400 registers; at two waves
// the excess goes to scratch memory (several GB of HBM traffic per launch at
// 48^3 cells), at one wave to the accumulation registers, which measured
// slower (less latency hiding).  VFP_GENERAL_WAVES_3D selects it for them.
#ifndef VFP_GENERAL_WAVES
#define VFP_GENERAL_WAVES 2
#endif
#ifndef VFP_GENERAL_WAVES_3D
#define VFP_GENERAL_WAVES_3D 2
#endif
template <int D, int K>
constexpr int general_waves() { return (D == 3 && K == 2) ? VFP_GENERAL_WAVES_3D : VFP_GENERAL_WAVES; }

template <int D, int K, int LMAX, bool MOM, int FL, bool ADJ>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(general_waves<D, K>())))
void stage_kernel(KernelArgs A) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = IPow<K1, D>::v;
  constexpr int CPB = Tile<N>::cpb;
  constexpr int DS = MOM ? D - 1 : D;
  __shared__ double sh[CPB * NB * N];

  const int tid = threadIdx.x;
  const int cl = tid / N;
  const int r = tid - cl * N;
  const bool in_grp = cl < CPB;
  const int cell0 = blockIdx.x * CPB + cl;
  const bool act = in_grp && cell0 < A.mesh.ncells;
  const int cell = act ? cell0 : 0;
  // lanes past the last group use a private dummy slot of group 0's rows:
  // they never write (guarded below) but must join every barrier
  double* shc = sh + (in_grp ? cl : 0) * NB * N;
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;

  int ic[3];
  {
    int c = cell;
    ic[0] = c % M.n[0];
    c /= M.n[0];
    ic[1] = c % M.n[1];
    ic[2] = c / M.n[1];
  }
  LaneRows<LMAX> R;
  load_rows<LMAX>(A.tab, r, R);

  double w[NB];
  const size_t cbase = (size_t)cell * NB * N + r;
#pragma unroll
  for (int b = 0; b < NB; ++b) w[b] = act ? A.st.w_in[cbase + (size_t)b * N] : 0.0;

  double res[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) res[b] = 0.0;

  // A uniform flow at fixed p, forward: beta^a = U_a + V A^a is constant on
  // the cell, so the advection volume term is (2/h_a) (dvol along a) (beta^a w)
  // on the nodes (the test and interpolation matrices of the other axes
  // cancel, tst phi = I, because the Gauss rule integrates the mass matrix
  // exactly); only the reaction needs the Gauss points.  The faces run first
  // (they read w's traces), then w itself turns into its Gauss-point values.
  constexpr bool NODADV = !ADJ && !MOM && FL == FLOW_UNIFORM;
  if constexpr (NODADV) {
    face_axis<D, K, LMAX, MOM, FL, 0, ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
    if constexpr (D > 1) face_axis<D, K, LMAX, MOM, FL, (D > 1 ? 1 : 0), ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
    if constexpr (D > 2) face_axis<D, K, LMAX, MOM, FL, (D > 2 ? 2 : 0), ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
    const Basis1D& bs = c_basis[K - 1];
    if (in_grp) {
#pragma unroll
      for (int b = 0; b < NB; ++b) shc[b * N + r] = w[b];
    }
    __syncthreads();
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const int st = ax == 0 ? 1 : (ax == 1 ? K1 : K1 * K1);
      const double sc = F.t_adv * M.s2h[ax][ic[ax]];
      const double Ua = F.U[ax];
#pragma unroll
      for (int base = 0; base < NB; ++base) {
        if ((base / st) % K1 != 0) continue;
        double t[K1];
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          const int b = base + j * st;
          t[j] = fma(Ua, w[b], F.V0 * dir_apply<LMAX>(R, ax, shc + b * N));
        }
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < K1; ++j) acc = fma(bs.dvol[i][j], t[j], acc);
          res[base + i * st] = fma(sc, acc, res[base + i * st]);
        }
      }
    }
    __syncthreads();
    // G = (R - div beta) f at the Gauss points, in place of w
    interp_ip<D, K>(w);
    if (in_grp) {
#pragma unroll
      for (int q = 0; q < NB; ++q) shc[q * N + r] = w[q];
    }
    __syncthreads();
    const double nu = F.nu_cell ? F.nu_cell[cell] : F.nu0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double* P = shc + q * N;
      const double nuq = F.nu_pts ? F.nu_pts[(size_t)cell * NB + q] : nu;
      double g = F.t_col * nuq * R.cv * w[q];
      if (F.t_rot != 0.0) {
        double om[3];
        if (F.B_pts) {
          const double* bp = F.B_pts + ((size_t)cell * NB + q) * 3;
          om[0] = bp[0]; om[1] = bp[1]; om[2] = bp[2];
        } else {
          om[0] = F.B[0]; om[1] = F.B[1]; om[2] = F.B[2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (om[c] != 0.0) g -= F.ig0 * om[c] * om_apply<LMAX>(R, c, P);
      }
      w[q] = g;
    }
    contract_add_ip<D, K>(w, res, -1.0);
  } else {
  // ---- volume terms -----------------------------------------------------
  {
    double fq[NB];
    interp<D, K>(w, fq);
    if (in_grp) {
#pragma unroll
      for (int q = 0; q < NB; ++q) shc[q * N + r] = fq[q];
    }
    __syncthreads();

    const double nu = F.nu_cell ? F.nu_cell[cell] : F.nu0;
    double tmp[NB];
    // G = (R - div beta) f
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double* P = shc + q * N;
      const PointScalars s = point_scalars<D, K, MOM, FL>(F, ic, q, cell);
      const double f = fq[q];
      const double nuq = F.nu_pts ? F.nu_pts[(size_t)cell * NB + q] : nu;
      double g = F.t_col * nuq * R.cv * f;
      if constexpr (MOM) {
        const double fxp = P[R.axc[0]], fxm = P[R.axc[1]];
        const double fpp = P[R.axxc[0]], fmm = P[R.axxc[1]];
        const double Axf = R.axv[0] * fxp + R.axv[1] * fxm;
        const double G1f = R.g1v[0] * fxp + R.g1v[1] * fxm;
        const double G2f = R.g2v[0] * fpp + R.g2v[1] * f + R.g2v[2] * fmm;
        if constexpr (ADJ) {
          const double G1t = R.g1tv[0] * fxp + R.g1tv[1] * fxm;
          const double G2t = R.g2tv[0] * fpp + R.g2tv[1] * f + R.g2tv[2] * fmm;
          g += F.t_mom * (s.a * s.iV * G1t + s.dU * G2t - s.a * s.idiv * Axf);
          // (A^x A^x)_t is symmetric: the linear-p term is its own transpose
          if (F.t_divu != 0.0)
            g += F.t_mom * F.t_divu * s.dU * (R.axxv[0] * fpp + R.axxv[1] * f + R.axxv[2] * fmm);
        } else {
          g += F.t_mom * (s.a * s.iV * G1f + s.dU * G2f - s.a * s.idiv * Axf);
          // linear p: -div beta also holds + U' (A^x A^x)_t
          if (F.t_divu != 0.0)
            g += F.t_mom * F.t_divu * s.dU * (R.axxv[0] * fpp + R.axxv[1] * f + R.axxv[2] * fmm);
        }
      }
      if constexpr (FL != FLOW_UNIFORM) g -= F.t_adv * s.divU * f;
      if (F.t_rot != 0.0) {
        double om[3];
        if (F.B_pts) {
          const double* bp = F.B_pts + ((size_t)cell * NB + q) * 3;
          om[0] = bp[0]; om[1] = bp[1]; om[2] = bp[2];
        } else {
          om[0] = F.B[0]; om[1] = F.B[1]; om[2] = F.B[2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (om[c] != 0.0) g += (ADJ ? 1.0 : -1.0) * s.ig * om[c] * om_apply<LMAX>(R, c, P);
      }
      tmp[q] = g;
    }
    contract_add<D, K, -1>(tmp, res, -1.0);

    if constexpr (!ADJ) {
      // F^a = beta^a f for the spatial axes (axis a is the spatial component a)
#pragma unroll
      for (int ax = 0; ax < DS; ++ax) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double* P = shc + q * N;
          const PointScalars s = point_scalars<D, K, MOM, FL>(F, ic, q, cell);
          tmp[q] = F.t_adv * (s.Up[ax] * fq[q] + s.V * dir_apply<LMAX>(R, ax, P));
        }
        const double sc = M.s2h[ax][ic[ax]];
        if (ax == 0) contract_add<D, K, 0>(tmp, res, sc);
        if constexpr (D > 1)
          if (ax == 1) contract_add<D, K, (D > 1 ? 1 : 0)>(tmp, res, sc);
        if constexpr (D > 2)
          if (ax == 2) contract_add<D, K, (D > 2 ? 2 : 0)>(tmp, res, sc);
      }
      // F^{ln p} = beta^{ln p} f
      if constexpr (MOM) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double* P = shc + q * N;
          const PointScalars s = point_scalars<D, K, MOM, FL>(F, ic, q, cell);
          const double Axf = R.axv[0] * P[R.axc[0]] + R.axv[1] * P[R.axc[1]];
          const double A2f = R.axxv[0] * P[R.axxc[0]] + R.axxv[1] * fq[q] + R.axxv[2] * P[R.axxc[1]];
          tmp[q] = -F.t_mom * (s.a * s.ca * Axf + s.dU * s.cu * A2f);
        }
        contract_add<D, K, D - 1>(tmp, res, M.s2h[D - 1][ic[D - 1]]);
      }
    } else {
      // beta^a (d_a mu) at the Gauss points, tested with phi (all axes)
      adj_flux_axis<D, K, LMAX, MOM, FL, 0>(A, R, shc, w, res, ic, cell, r, in_grp);
      if constexpr (D > 1) adj_flux_axis<D, K, LMAX, MOM, FL, (D > 1 ? 1 : 0)>(A, R, shc, w, res, ic, cell, r, in_grp);
      if constexpr (D > 2) adj_flux_axis<D, K, LMAX, MOM, FL, (D > 2 ? 2 : 0)>(A, R, shc, w, res, ic, cell, r, in_grp);
    }
    __syncthreads();
  }

  // ---- faces ------------------------------------------------------------
  face_axis<D, K, LMAX, MOM, FL, 0, ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
  if constexpr (D > 1) face_axis<D, K, LMAX, MOM, FL, (D > 1 ? 1 : 0), ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
  if constexpr (D > 2) face_axis<D, K, LMAX, MOM, FL, (D > 2 ? 2 : 0), ADJ>(A, R, shc, w, res, ic, cell, r, act, in_grp);
  }

  // ---- source and output -------------------------------------------------
  if constexpr (ADJ) {
    if (A.adj.mass_out) {
      ref_mass<D, K, false>(res);
      const double jac = cell_jacobian<D>(M, ic);
#pragma unroll
      for (int b = 0; b < NB; ++b) res[b] *= jac;
    }
    if (A.adj.fwd && A.adj.grad_nu) {
      // d/dnu_c of <lambda, beta L(fwd)> = -beta t_col sum_lms C (M mu) . fwd
      double mw[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) mw[b] = w[b];
      ref_mass<D, K, false>(mw);
      double part = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) part = fma(mw[b], act ? A.adj.fwd[cbase + (size_t)b * N] : 0.0, part);
      part *= R.cv * cell_jacobian<D>(M, ic);
      if (in_grp) shc[r] = part;
      __syncthreads();
      if (act && r == 0) {
        double sum = 0.0;
        for (int j = 0; j < N; ++j) sum += shc[j];
        // one add per cell and launch (reproducible in stream order)
        atomicAdd(&A.adj.grad_nu[cell], -A.st.beta * F.t_col * sum);
      }
    }
    if (act && A.adj.t_out) {
#pragma unroll
      for (int b = 0; b < NB; ++b) A.adj.t_out[cbase + (size_t)b * N] = A.st.beta * res[b];
    }
  } else if (A.st.with_source && F.src && r == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) res[b] += F.src[(size_t)cell * NB + b];
  }
  if (act) {
    if (A.st.alpha != 0.0) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        A.st.w_out[cbase + (size_t)b * N] = fma(A.st.beta, res[b], A.st.alpha * A.st.u[cbase + (size_t)b * N]);
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) A.st.w_out[cbase + (size_t)b * N] = A.st.beta * res[b];
    }
  }
}

template <int D, int K, int LMAX, bool MOM, int FL, bool ADJ>
void launch_stage_t(const KernelArgs& a, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int CPB = Tile<N>::cpb;
  const int blocks = (a.mesh.ncells + CPB - 1) / CPB;
  hipLaunchKernelGGL((stage_kernel<D, K, LMAX, MOM, FL, ADJ>), dim3(blocks), dim3(kThreads), 0, s, a);
}

template <int D, int K, bool MOM, int FL, bool ADJ>
StageLauncher pick_lmax(int lmax) {
  switch (lmax) {
    case 1: return &launch_stage_t<D, K, 1, MOM, FL, ADJ>;
    case 2: return &launch_stage_t<D, K, 2, MOM, FL, ADJ>;
    case 3: return &launch_stage_t<D, K, 3, MOM, FL, ADJ>;
    case 4: return &launch_stage_t<D, K, 4, MOM, FL, ADJ>;
    case 5: return &launch_stage_t<D, K, 5, MOM, FL, ADJ>;
    case 6: return &launch_stage_t<D, K, 6, MOM, FL, ADJ>;
    case 7: return &launch_stage_t<D, K, 7, MOM, FL, ADJ>;
    default: break;
  }
  // l_max 8..11: runs along x at fixed p with a uniform flow (forward)
  if constexpr (D == 1 && !MOM && !ADJ && FL == FLOW_UNIFORM && K <= 2) {
    switch (lmax) {
      case 8: return &launch_stage_t<D, K, 8, MOM, FL, ADJ>;
      case 9: return &launch_stage_t<D, K, 9, MOM, FL, ADJ>;
      case 10: return &launch_stage_t<D, K, 10, MOM, FL, ADJ>;
      case 11: return &launch_stage_t<D, K, 11, MOM, FL, ADJ>;
      default: break;
    }
  }
  return nullptr;
}

// Degrees above 2 are built for the forward operator only: up to k = 5 on
// one axis and k = 3 on two (the lane's (k+1)^D nodal values stay in
// registers).
template <int D, bool MOM, int FL, bool ADJ>
StageLauncher pick_k(int k, int lmax) {
  if (k == 1) return pick_lmax<D, 1, MOM, FL, ADJ>(lmax);
  if (k == 2) return pick_lmax<D, 2, MOM, FL, ADJ>(lmax);
  if constexpr (!ADJ && D <= 2 && FL != FLOW_POINTS) {
    if (k == 3) return pick_lmax<D, 3, MOM, FL, ADJ>(lmax);
  }
  if constexpr (!ADJ && D == 1 && FL != FLOW_POINTS) {
    if (k == 4) return pick_lmax<D, 4, MOM, FL, ADJ>(lmax);
    if (k == 5) return pick_lmax<D, 5, MOM, FL, ADJ>(lmax);
  }
  return nullptr;
}
}  // namespace gen
}  // namespace vfp
