// Fused operator / Runge-Kutta stage for the (x, ln p) configuration with a
// planar flow U_x(x), a uniform magnetic field and a per-cell or uniform
// scattering rate -- the parallel-shock runs of Sec. 4.4.
//
//   w_out = alpha u + beta L(w_in),   L(w) = M^{-1}(h - D w)
//
// Lane = (cell, lms); the cell's (k+1)^2 nodal values of that coefficient stay
// in registers.  Per Gauss point the lane needs the coefficients
// (l+-1, m, s), (l+-2, m, s) and the rotation row of its own cell from LDS:
//   F^x = U f + V A^x f                                 (advection, x)
//   F^p = -(dU/dt / V) A^x f - U' (A^x A^x)_t f         (beta^{ln p} f)
//   G   = (dU/dt / V) G1 f + U' (G2 f - f) - dU/dt m/(gamma p) A^x f
//         - (q/(gamma m)) (B.Omega) f + nu C f         ((R - div beta) f)
// with G1 = (A^y Om^z - A^z Om^y)_t, G2 = (A^x G1)_t.  The weak form
//   L = -T(G) + (2/h_x) T'_x(F^x) + (2/h_p) T'_p(F^p) + face lifts + M^{-1} h
// is contracted row by row of Gauss points (sum factorisation).
//
// Latency: every global load (own state, the four neighbour traces and the
// per-cell field scalars) is issued at the start.  The per-cell scalars are
// staged once in LDS and read by broadcast.  Faces are processed before the
// volume so that the nodal state is dead once it has been interpolated.
#include "basis.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kThreads = 256;
#ifndef VFP_SHOCK_WAVES
#define VFP_SHOCK_WAVES 3
#endif

// per-cell scalar record in LDS (doubles): the packed x record of the cell's
// x column, the packed p record of its p row, the p-face codes and nu
enum : int {
  X_U = 0,       // t_adv (2/h_x) U_x at the x Gauss points            [3]
  X_DU = 3,      // dU_x/dx                                             [3]
  X_A = 6,       // t_mom dU_x/dt                                       [3]
  X_UF = 9,      // t_adv U_x at the lo / hi x face                     [2]
  X_S2H = 11,    // 2/h_x
  P_V = 16,      // V at the p Gauss points                             [3]
  P_IV = 19,     // 1/V                                                 [3]
  P_ID = 22,     // m/(gamma p)                                         [3]
  P_IG = 25,     // t_rot q/(gamma m)                                   [3]
  P_IVF = 28,    // t_mom / V at the lo / hi p face                     [2]
  P_S2H = 30,    // 2/h_p
  C_CODE = 32,   // p-face upwind codes [side][x point]                 [2*K1]
  C_NU = 38,     // t_col nu
  S_STRIDE = 40
};
static_assert(kRec == 16, "record layout");

template <int K, int LMAX, int NROT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(VFP_SHOCK_WAVES)))
void shock_kernel(KernelArgs A) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = K1 * K1;
  constexpr int CPB = (kThreads / N) > 0 ? kThreads / N : 1;
  constexpr int FV = NB;              // volume exchange rows per cell
  constexpr int FF = 4 * K1;          // face exchange rows per cell
  using CB = CBasis<K>;
  static_assert(K1 <= 3, "basis tables");
  __shared__ double shv[CPB * FV * N];
  __shared__ double shf[CPB * FF * N];
  __shared__ double shs[CPB * S_STRIDE];

  const int tid = threadIdx.x;
  const int cl = tid / N;
  const int r = tid - cl * N;
  const bool in_grp = cl < CPB;
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;
  const RowTables& T = A.tab;
  const int cell0 = blockIdx.x * CPB + cl;
  const bool act = in_grp && cell0 < M.ncells;
  const int cell = act ? cell0 : 0;
  const int nx = M.n[0], np = M.n[1];
  const int ix = cell % nx, ip = cell / nx;
  const int clc = in_grp ? cl : 0;
  double* vol = shv + clc * FV * N;
  double* fac = shf + clc * FF * N;
  double* sc = shs + clc * S_STRIDE;

  // ---- issue every global load --------------------------------------------
  const size_t cbase = (size_t)cell * NB * N + r;
  const double* win = A.st.w_in + cbase;
  double w[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) w[b] = act ? win[(size_t)b * N] : 0.0;

  // neighbour traces: tnx[side][j] (x faces, nodes along p) and tnp[side][j]
  // (p faces, nodes along x)
  double tnx[2][K1], tnp[2][K1];
  bool use_nx[2], use_np[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    int ni = side ? ix + 1 : ix - 1;
    const int bc = side ? M.bc_hi[0] : M.bc_lo[0];
    use_nx[side] = (ni >= 0 && ni < nx) || bc == 0;
    ni = (ni + nx) % nx;
    const double* nb0 = A.st.w_in + (size_t)(cell + (ni - ix)) * NB * N + r;
    const int jn = side ? 0 : K;
#pragma unroll
    for (int j = 0; j < K1; ++j) tnx[side][j] = (act && use_nx[side]) ? nb0[(size_t)(jn + K1 * j) * N] : 0.0;
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    int ni = side ? ip + 1 : ip - 1;
    const int bc = side ? M.bc_hi[1] : M.bc_lo[1];
    use_np[side] = (ni >= 0 && ni < np) || bc == 0;
    ni = (ni + np) % np;
    const double* nb0 = A.st.w_in + (size_t)(cell + (ni - ip) * nx) * NB * N + r;
    const int jn = side ? 0 : K;
#pragma unroll
    for (int j = 0; j < K1; ++j) tnp[side][j] = (act && use_np[side]) ? nb0[(size_t)(j + K1 * jn) * N] : 0.0;
  }

  // per-cell scalars: lanes of a cell share the record
  if (in_grp) {
    for (int e = r; e < kRec; e += N) {
      sc[e] = F.xrec[(size_t)ix * kRec + e];
      sc[kRec + e] = F.prec[(size_t)ip * kRec + e];
    }
    for (int e = r; e < 2 * K1; e += N)
      sc[C_CODE + e] = (double)F.pf_code[(size_t)(ip + e / K1) * (nx * K1) + ix * K1 + e % K1];
    if (r == 0) sc[C_NU] = F.t_col * (F.nu_cell ? F.nu_cell[cell] : F.nu0);
  }

  // lms rows used by the x faces
  int mem[LMAX + 1];
  double wcol[LMAX + 1];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    mem[i] = T.blk_mem[i * N + r];
    wcol[i] = T.w_col[i * N + r];
  }
  const double lam = T.lam[r];

  // ---- interpolation: volume points and face points -----------------------
  {
    double t[NB];
#pragma unroll
    for (int j1 = 0; j1 < K1; ++j1)
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        double acc = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) acc = fma(CB::phi[q0][j0], w[j0 + K1 * j1], acc);
        t[q0 + K1 * j1] = acc;
      }
    if (in_grp) {
#pragma unroll
      for (int q1 = 0; q1 < K1; ++q1)
#pragma unroll
        for (int q0 = 0; q0 < K1; ++q0) {
          double acc = 0.0;
#pragma unroll
          for (int j1 = 0; j1 < K1; ++j1) acc = fma(CB::phi[q1][j1], t[q0 + K1 * j1], acc);
          vol[(q0 + K1 * q1) * N + r] = acc;
        }
    }
  }
  // x faces: LDS rows (side*2 + which)*K1 + q, which 0 = lower cell, 1 = upper
  {
    const int bclo = M.bc_lo[0], bchi = M.bc_hi[0];
    double tr[2][2][K1];
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      tr[0][1][j] = w[0 + K1 * j];
      tr[1][0][j] = w[K + K1 * j];
      tr[0][0][j] = use_nx[0] ? tnx[0][j] : (bclo == 1 ? 0.0 : tr[0][1][j]);
      tr[1][1][j] = use_nx[1] ? tnx[1][j] : (bchi == 1 ? 0.0 : tr[1][0][j]);
    }
    if (in_grp) {
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int which = 0; which < 2; ++which)
#pragma unroll
          for (int q = 0; q < K1; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < K1; ++j) acc = fma(CB::phi[q][j], tr[side][which][j], acc);
            fac[((side * 2 + which) * K1 + q) * N + r] = acc;
          }
    }
  }
  // p-face traces are interpolated now, while w is live, and kept in registers
  double Fp[2][2][K1];
  {
    const int bclo = M.bc_lo[1], bchi = M.bc_hi[1];
    double tr[2][2][K1];
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      tr[0][1][j] = w[j];
      tr[1][0][j] = w[j + K1 * K];
      tr[0][0][j] = use_np[0] ? tnp[0][j] : (bclo == 1 ? 0.0 : tr[0][1][j]);
      tr[1][1][j] = use_np[1] ? tnp[1][j] : (bchi == 1 ? 0.0 : tr[1][0][j]);
    }
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int which = 0; which < 2; ++which)
#pragma unroll
        for (int q = 0; q < K1; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < K1; ++j) acc = fma(CB::phi[q][j], tr[side][which][j], acc);
          Fp[side][which][q] = acc;
        }
  }
  __syncthreads();

  double res[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) res[b] = 0.0;

  // ---- x faces: characteristic variables of A^x ------------------------------
  {
    double Jc[2][K1];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double UF = sc[X_UF + side];
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        const double* P1 = fac + ((side * 2 + 0) * K1 + q) * N;
        const double* P2 = fac + ((side * 2 + 1) * K1 + q) * N;
        double c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int j = 0; j <= LMAX; ++j) {
          c1 = fma(wcol[j], P1[mem[j]], c1);
          c2 = fma(wcol[j], P2[mem[j]], c2);
        }
        const double mu = fma(F.t_adv * lam, sc[P_V + q], UF);
        Jc[side][q] = fmax(mu, 0.0) * c1 + fmin(mu, 0.0) * c2;
      }
    }
    __syncthreads();
    if (in_grp) {
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int q = 0; q < K1; ++q) fac[(side * K1 + q) * N + r] = Jc[side][q];
    }
    __syncthreads();
    double wrow[LMAX + 1];
#pragma unroll
    for (int i = 0; i <= LMAX; ++i) wrow[i] = T.w_row[i * N + r];
    const double s2hx = sc[X_S2H];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      double J[K1];
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        const double* P = fac + (side * K1 + q) * N;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i <= LMAX; ++i) acc = fma(wrow[i], P[mem[i]], acc);
        J[q] = acc;
      }
      const double scl = side ? -s2hx : s2hx;
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1) {
        double jn = 0.0;
#pragma unroll
        for (int q = 0; q < K1; ++q)
          if (CB::tst[i1][q] != 0.0) jn = fma(CB::tst[i1][q], J[q], jn);
        jn *= scl;
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) res[i0 + K1 * i1] = fma(CB::lift[side][i0], jn, res[i0 + K1 * i1]);
      }
    }
  }
  __syncthreads();

  // ---- ln p faces: beta^{ln p} = a1 A^x + a2 (A^x A^x)_t per point ---------
  const int axc0 = T.ax_col[r], axc1 = T.ax_col[N + r];
  const double axv0 = T.ax_val[r], axv1 = T.ax_val[N + r];
  const int axxc0 = T.axx_col[r], axxc1 = T.axx_col[N + r];
  const double axxv0 = T.axx_val[r], axxv1 = T.axx_val[N + r], axxv2 = T.axx_val[2 * N + r];
  {
    if (in_grp) {
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int which = 0; which < 2; ++which)
#pragma unroll
          for (int q = 0; q < K1; ++q) fac[((side * 2 + which) * K1 + q) * N + r] = Fp[side][which][q];
    }
    __syncthreads();
    const double s2hp = sc[P_S2H];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double iVf = sc[P_IVF + side];
      double J[K1];
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        const double a1 = -sc[X_A + q] * iVf;
        const double a2 = -F.t_mom * sc[X_DU + q];
        const int code = (int)sc[C_CODE + side * K1 + q];
        const double* P1 = fac + ((side * 2 + 0) * K1 + q) * N;
        const double* P2 = fac + ((side * 2 + 1) * K1 + q) * N;
        const double* Pu = (code == -1) ? P1 : P2;
        double jv = a1 * fma(axv0, Pu[axc0], axv1 * Pu[axc1]) +
                    a2 * fma(axxv0, Pu[axxc0], fma(axxv1, Pu[r], axxv2 * Pu[axxc1]));
        if (code >= 0) {
          const double* tb = F.pf_tab + ((size_t)code * N + r) * (LMAX + 1);
#pragma unroll
          for (int i = 0; i <= LMAX; ++i) jv = fma(tb[i], P1[mem[i]] - P2[mem[i]], jv);
        }
        J[q] = jv;
      }
      const double scl = side ? -s2hp : s2hp;
#pragma unroll
      for (int i0 = 0; i0 < K1; ++i0) {
        double jn = 0.0;
#pragma unroll
        for (int q = 0; q < K1; ++q)
          if (CB::tst[i0][q] != 0.0) jn = fma(CB::tst[i0][q], J[q], jn);
        jn *= scl;
#pragma unroll
        for (int i1 = 0; i1 < K1; ++i1) res[i0 + K1 * i1] = fma(CB::lift[side][i1], jn, res[i0 + K1 * i1]);
      }
    }
  }

  // u (the stage base) is loaded now so that its latency hides behind the
  // volume work; each lane reads its own entries before writing them, which
  // keeps the in-place form w_out == u correct
  double uu[NB];
  const bool use_u = A.st.alpha != 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) uu[b] = (act && use_u) ? A.st.u[cbase + (size_t)b * N] : 0.0;

  // ---- volume -------------------------------------------------------------
  {
    const double g1v0 = T.g1_val[r], g1v1 = T.g1_val[N + r];
    const double g2v0 = T.g2_val[r], g2v1 = T.g2_val[N + r], g2v2 = T.g2_val[2 * N + r];
    int rc[NROT];
    double rv[NROT];
#pragma unroll
    for (int s = 0; s < NROT; ++s) {
      rc[s] = T.rot_col[s * N + r];
      rv[s] = T.rot_val[s * N + r];
    }
    const double nuc = T.c_val[r] * sc[C_NU];
    const double mom_s2hp = -F.t_mom * sc[P_S2H];
    const double t_adv = F.t_adv, t_mom = F.t_mom;
    const double tas2hx = t_adv * sc[X_S2H];
#pragma unroll
    for (int q1 = 0; q1 < K1; ++q1) {
      const double pV = tas2hx * sc[P_V + q1];
      const double piV = sc[P_IV + q1];
      const double pid = sc[P_ID + q1];
      const double pig = sc[P_IG + q1];
      double ac[K1], bc[K1];
#pragma unroll
      for (int i = 0; i < K1; ++i) ac[i] = bc[i] = 0.0;
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        const double U = sc[X_U + q0];
        const double dU = sc[X_DU + q0];
        const double a = sc[X_A + q0];
        const double* P = vol + (q0 + K1 * q1) * N;
        const double f = P[r];
        const double fxp = P[axc0], fxm = P[axc1];
        const double fpp = P[axxc0], fmm = P[axxc1];
        double Rf = 0.0;
#pragma unroll
        for (int s = 0; s < NROT; ++s) Rf = fma(rv[s], P[rc[s]], Rf);
        const double Axf = fma(axv0, fxp, axv1 * fxm);
        const double G1f = fma(g1v0, fxp, g1v1 * fxm);
        const double A2f = fma(axxv0, fpp, fma(axxv1, f, axxv2 * fmm));
        const double G2f = fma(g2v0, fpp, fma(g2v1, f, g2v2 * fmm));
        const double aiV = a * piV;
        const double X = fma(U, f, pV * Axf);
        const double Pp = mom_s2hp * fma(aiV, Axf, dU * A2f);
        double G = fma(aiV, G1f, dU * fma(t_mom, G2f, -t_adv * f));
        G = fma(-a * pid, Axf, G);
        G = fma(-pig, Rf, G);
        G = fma(nuc, f, G);
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          if (CB::tst[i][q0] != 0.0) ac[i] = fma(-CB::tst[i][q0], G, ac[i]);
          if (CB::dtst[i][q0] != 0.0) ac[i] = fma(CB::dtst[i][q0], X, ac[i]);
          if (CB::tst[i][q0] != 0.0) bc[i] = fma(CB::tst[i][q0], Pp, bc[i]);
        }
      }
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) {
          double v = res[i0 + K1 * i1];
          if (CB::tst[i1][q1] != 0.0) v = fma(CB::tst[i1][q1], ac[i0], v);
          if (CB::dtst[i1][q1] != 0.0) v = fma(CB::dtst[i1][q1], bc[i0], v);
          res[i0 + K1 * i1] = v;
        }
    }
  }

  // ---- source and output ---------------------------------------------------
  if (A.st.with_source && F.src && r == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) res[b] += F.src[(size_t)cell * NB + b];
  }
  if (act) {
    const double al = A.st.alpha, be = A.st.beta;
#pragma unroll
    for (int b = 0; b < NB; ++b) A.st.w_out[cbase + (size_t)b * N] = fma(be, res[b], al * uu[b]);
  }
}

template <int K, int LMAX, int NROT>
void launch_shock_t(const KernelArgs& a, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int CPB = (kThreads / N) > 0 ? kThreads / N : 1;
  const int blocks = (a.mesh.ncells + CPB - 1) / CPB;
  hipLaunchKernelGGL((shock_kernel<K, LMAX, NROT>), dim3(blocks), dim3(kThreads), 0, s, a);
}

template <int K, int NROT>
StageLauncher pick(int lmax) {
  switch (lmax) {
    case 1: return &launch_shock_t<K, 1, NROT>;
    case 2: return &launch_shock_t<K, 2, NROT>;
    case 3: return &launch_shock_t<K, 3, NROT>;
    case 4: return &launch_shock_t<K, 4, NROT>;
    case 5: return &launch_shock_t<K, 5, NROT>;
    case 6: return &launch_shock_t<K, 6, NROT>;
    case 7: return &launch_shock_t<K, 7, NROT>;
    default: return nullptr;
  }
}

}  // namespace

StageLauncher find_shock_launcher(int k, int lmax, int nrot) {
  if (nrot != 1 && nrot != 5) return nullptr;
  if (k == 1) return nrot == 1 ? pick<1, 1>(lmax) : pick<1, 5>(lmax);
  if (k == 2) return nrot == 1 ? pick<2, 1>(lmax) : pick<2, 5>(lmax);
  return nullptr;
}

}  // namespace vfp
