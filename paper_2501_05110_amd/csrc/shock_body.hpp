// Device body of the (x, ln p) stage kernels, shared by the single-run
// kernels (stage_shock.hip) and the batched kernels (stage_batch.hip).
// Fused operator / Runge-Kutta stage for the (x, ln p) configuration with a
// planar flow U_x(x), a uniform magnetic field and a per-cell or uniform
// scattering rate -- the parallel-shock runs of Sec. 4.4.
//
//   w_out = alpha u + beta L(w_in),   L(w) = M^{-1}(h - D w)
//
// Lane = (cell, lms); the cell's (k+1)^2 nodal values of that coefficient stay
// in registers.  Per Gauss point the lane needs the coefficients
// (l+-1, m, s), (l+-2, m, s) and the rotation row of its own cell, which are
// exchanged through LDS:
//   F^x = U f + V A^x f                                 (advection, x)
//   F^p = -(dU/dt / V) A^x f - U' (A^x A^x)_t f         (beta^{ln p} f)
//   G   = (dU/dt / V) G1 f + U' (G2 f - f) - dU/dt m/(gamma p) A^x f
//         - (q/(gamma m)) (B.Omega) f + nu C f         ((R - div beta) f)
// with G1 = (A^y Om^z - A^z Om^y)_t, G2 = (A^x G1)_t.  The weak form
//   L = -T(G) + (2/h_x) T'_x(F^x) + (2/h_p) T'_p(F^p) + face lifts + M^{-1} h
// is contracted row by row of Gauss points (sum factorisation).
//
// With ADJ = true the same kernel applies the adjoint operator
// K = -M^{-1} D^T in mu = M^{-1} lambda variables:
//   K mu = T(beta^x d_x mu + beta^p d_p mu - (R - div beta)^T mu) + face lifts
// (all tested with phi, derivative interpolation of mu; G1, G2 and B.Omega
// transposed), and the faces take the forward flux routine with the traces
// (d, 0) / (0, d), d = mu(own) - mu(other), or (own, own) at a continuous
// boundary.  Each row of Gauss points then exchanges three fields (mu and its
// two derivatives) through LDS.
//
// Scheduling.  All global loads (own state, the four neighbour traces, the
// per-cell field scalars) are issued at the start; the scalars go to LDS.
// Each face side, and each row of Gauss points, then passes through one small
// LDS exchange area of 2(k+1) rows per cell, so that few values are live at
// once.  When a cell's n lanes never straddle a wavefront (n divides 64) the
// workgroup is one wavefront and the exchanges need no workgroup barrier.
#pragma once
#include <type_traits>

#include "basis.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace vfp {
namespace shock {

#ifndef VFP_SHOCK_WAVES
#define VFP_SHOCK_WAVES 1
#endif
#ifndef VFP_NT_STORE
#define VFP_NT_STORE 1
#endif
#ifndef VFP_NT_LOAD_U
#define VFP_NT_LOAD_U 0
#endif
#ifndef VFP_LATE_U
#define VFP_LATE_U 0
#endif
// ln p neighbour traces loaded after the x faces, and only for cells whose
// x column has a flow gradient (measured faster: 96.7 against 100.8 us per
// launch at 1024 x 128)
#ifndef VFP_LATE_PT
#define VFP_LATE_PT 1
#endif

// per-cell scalar record in LDS (doubles): the packed x record of the cell's
// x column, the packed p record of its p row, the p-face codes and nu
enum : int {
  X_U = 0,       // t_adv (2/h_x) U_x at the x Gauss points            [3]
  X_DU = 3,      // dU_x/dx                                             [3]
  X_A = 6,       // t_mom dU_x/dt                                       [3]
  X_UF = 9,      // t_adv U_x at the lo / hi x face                     [2]
  X_S2H = 11,    // 2/h_x
  X_GRAD = 12,   // 1 if dU_x/dx or dU_x/dt is non-zero at a Gauss point of the cell
  P_V = 16,      // V at the p Gauss points                             [3]
  P_IV = 19,     // 1/V                                                 [3]
  P_ID = 22,     // m/(gamma p)                                         [3]
  P_IG = 25,     // t_rot q/(gamma m)                                   [3]
  P_IVF = 28,    // t_mom / V at the lo / hi p face                     [2]
  P_S2H = 30,    // 2/h_p
  C_CODE = 32,   // p-face upwind codes [side][x point]                 [2*K1]
  C_NU = 38,     // t_col nu
  S_STRIDE = 40,
  // linear p axis only: coefficients of dU/dt and U' in beta^p
  P2_CA = 40,    // gamma m at the p Gauss points                      [3]
  P2_CU = 43,    // p at the p Gauss points                            [3]
  P2_CUF = 46,   // p at the lo / hi p face                            [2]
  S_STRIDE_LINP = 48
};
constexpr int kRec2 = 8;         // doubles per extra p record (linear p axis)
static_assert(kRec == 16, "record layout");

// Workgroup shape: TPB lanes (0: the default, one wavefront where n divides
// 64, else 256 lanes) holding floor(TPB / n) cells (at least one).  kWave:
// the lanes of every cell lie in one wavefront, so the per-cell LDS
// exchanges need only wavefront-level ordering.
template <int N, int TPB = 0>
struct Launch {
  static constexpr int kThreads = TPB ? TPB : ((64 % N) == 0 ? 64 : 256);
  static constexpr bool kWave = (64 % N) == 0 || kThreads == 64;
  static constexpr int kCells = (kThreads / N) > 0 ? kThreads / N : 1;
  // cells whose lanes share one wavefront (the uniformity scope of a branch
  // taken before wavefront-level ordering points)
  static constexpr int kCellsPerWave = (64 % N) == 0 ? 64 / N : kCells;
};

// Orders the LDS exchange between the lanes of one cell.  LDS operations of
// one wavefront complete in order, so within a wavefront a compiler-level
// fence suffices; otherwise the workgroup synchronises.
template <int N, int TPB = 0>
__device__ __forceinline__ void cell_sync() {
  if constexpr (Launch<N, TPB>::kWave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One tile (kCells cells) of one run: the whole operator / stage for those
// cells.  blk is the tile index within the run.
// LINP: the momentum axis is p itself (beta^p = -(dU/dt gamma m A^x
// + U' p (A^x A^x)_t), -div beta = dU/dt V A^x + U' (A^x A^x)_t - div U);
// the p record then carries V, 1/V, -V (in the m/(gamma p) slot), q/(gamma m),
// t_mom gamma m at the faces, and the extra record gamma m, p, p at the faces.
template <int K, int LMAX, int NROT, bool ADJ, bool LINP = false, int TPB = 0>
__device__ __forceinline__ void shock_body(const KernelArgs& A, int blk) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = K1 * K1;
  using LS = Launch<N, TPB>;
  constexpr int CPB = LS::kCells;
  constexpr int XR = (ADJ ? 3 : 2) * K1;   // exchange rows per cell
  using CB = CBasis<K>;
  static_assert(K1 <= 3, "basis tables");
  constexpr int XS = XR * N;           // per-cell exchange area
  __shared__ double shx[CPB * XS];
  constexpr int SST = LINP ? S_STRIDE_LINP : S_STRIDE;
  __shared__ double shs[CPB * SST];

  const int tid = threadIdx.x;
  const int cl = tid / N;
  const int r = tid - cl * N;
  const bool in_grp = cl < CPB;
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;
  const RowTables& T = A.tab;
  const int cell0 = blk * CPB + cl;
  const bool act = in_grp && cell0 < M.ncells;
  const int cell = act ? cell0 : 0;
  const int nx = M.n[0], np = M.n[1];
  const int ix = cell % nx, ip = cell / nx;
  const int clc = in_grp ? cl : 0;
  double* X = shx + clc * XS;
  double* sc = shs + clc * SST;

  // ---- issue every global load, in order of first use ------------------------
  constexpr int NREC = (kRec + N - 1) / N;
  constexpr int NCODE = (2 * K1 + N - 1) / N;
  double rx[NREC], rp[NREC], rcode[NCODE], rnu = 0.0;
#pragma unroll
  for (int it = 0; it < NREC; ++it) {
    const int e = r + it * N;
    rx[it] = (in_grp && e < kRec) ? gp(F.xrec)[(size_t)ix * kRec + e] : 0.0;
    rp[it] = (in_grp && e < kRec) ? gp(F.prec)[(size_t)ip * kRec + e] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < NCODE; ++it) {
    const int e = r + it * N;
    rcode[it] = (in_grp && e < 2 * K1) ? gp(F.pf_coded)[(size_t)(ip + e / K1) * (nx * K1) + ix * K1 + e % K1]
                                       : 0.0;
  }
  if (in_grp && r == 0) rnu = F.t_col * (gp(F.nu_cell) ? gp(F.nu_cell)[cell] : F.nu0);
  constexpr int NREC2 = LINP ? (kRec2 + N - 1) / N : 1;
  double rp2[NREC2];
  if constexpr (LINP) {
#pragma unroll
    for (int it = 0; it < NREC2; ++it) {
      const int e = r + it * N;
      rp2[it] = (in_grp && e < kRec2) ? gp(F.prec2)[(size_t)ip * kRec2 + e] : 0.0;
    }
  }

  const size_t cbase = (size_t)cell * NB * N + r;
  const auto win = gp(A.st.w_in) + cbase;
  double w[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) w[b] = win[(size_t)b * N];   // lanes past the end read cell 0

  // neighbour traces: tn[axis][side][j]; x faces carry nodes along p, p faces
  // nodes along x.  Boundary sides are resolved to 0 (zero inflow) or the own
  // trace (continuous) below.
  double tn[2][2][K1];
  bool use_n[2][2];
  // the ln p neighbours' traces matter only where the cell's x column has a
  // flow gradient (elsewhere beta^{ln p} = 0 and the ln p flux vanishes);
  // with VFP_LATE_PT they are loaded after the x faces, and only there
  const bool cgrad = !VFP_LATE_PT || gp(F.xrec)[(size_t)ix * kRec + X_GRAD] != 0.0;
  auto load_traces = [&](int ax) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int ia = ax ? ip : ix, na = ax ? np : nx, st = ax ? nx : 1;
      int ni = side ? ia + 1 : ia - 1;
      const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
      use_n[ax][side] = (ni >= 0 && ni < na) || bc == 0;
      ni = (ni + na) % na;
      const auto nb0 = gp(A.st.w_in) + (size_t)(cell + (ni - ia) * st) * NB * N + r;
      const int jn = side ? 0 : K;
      const bool need = ax == 0 || cgrad;
#pragma unroll
      for (int j = 0; j < K1; ++j) {
        const int node = ax ? (j + K1 * jn) : (jn + K1 * j);
        tn[ax][side][j] = need ? nb0[(size_t)node * N] : 0.0;   // a valid cell; unused where !use_n
      }
    }
  };
  load_traces(0);
  if constexpr (!VFP_LATE_PT) load_traces(1);

  // rows for the x faces
  int mem[LMAX + 1];
  double wcol[LMAX + 1], wrow[LMAX + 1];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    mem[i] = gp(T.blk_mem)[i * N + r];
    wcol[i] = gp(T.w_col)[i * N + r];
    wrow[i] = gp(T.w_row)[i * N + r];
  }
  const double lam = gp(T.lam)[r];

  if (in_grp) {
#pragma unroll
    for (int it = 0; it < NREC; ++it) {
      const int e = r + it * N;
      if (e < kRec) {
        sc[e] = rx[it];
        sc[kRec + e] = rp[it];
      }
    }
#pragma unroll
    for (int it = 0; it < NCODE; ++it) {
      const int e = r + it * N;
      if (e < 2 * K1) sc[C_CODE + e] = rcode[it];
    }
    if (r == 0) sc[C_NU] = rnu;
    if constexpr (LINP) {
#pragma unroll
      for (int it = 0; it < NREC2; ++it) {
        const int e = r + it * N;
        if (e < kRec2) sc[P2_CA + e] = rp2[it];
      }
    }
  }

  double res[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) res[b] = 0.0;

  // ---- x faces: characteristic variables of A^x ------------------------------
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    double own[K1], oth[K1];
    const int bc = side ? M.bc_hi[0] : M.bc_lo[0];
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      own[j] = w[(side ? K : 0) + K1 * j];
      oth[j] = use_n[0][side] ? tn[0][side][j] : (bc == 1 ? 0.0 : own[j]);
    }
    if constexpr (ADJ) {
      if (use_n[0][side] || bc != 2) {
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          own[j] -= oth[j];
          oth[j] = 0.0;
        }
      }
    }
    // lower cell's trace to rows [0, K1), upper cell's to rows [K1, 2 K1)
    if (in_grp) {
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          a = fma(CB::phi[q][j], side ? own[j] : oth[j], a);
          b = fma(CB::phi[q][j], side ? oth[j] : own[j], b);
        }
        X[q * N + r] = a;
        X[(K1 + q) * N + r] = b;
      }
    }
    cell_sync<N, TPB>();
    double Jc[K1];
    const double UF = sc[X_UF + side];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double c1 = 0.0, c2 = 0.0;
#pragma unroll
      for (int j = 0; j <= LMAX; ++j) {
        c1 = fma(wcol[j], X[q * N + mem[j]], c1);
        c2 = fma(wcol[j], X[(K1 + q) * N + mem[j]], c2);
      }
      const double mu = fma(F.t_adv * lam, sc[P_V + q], UF);
      Jc[q] = fmax(mu, 0.0) * c1 + fmin(mu, 0.0) * c2;
    }
    cell_sync<N, TPB>();
    if (in_grp) {
#pragma unroll
      for (int q = 0; q < K1; ++q) X[q * N + r] = Jc[q];
    }
    cell_sync<N, TPB>();
    double J[K1];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i <= LMAX; ++i) acc = fma(wrow[i], X[q * N + mem[i]], acc);
      J[q] = acc;
    }
    const double scl = side ? -sc[X_S2H] : sc[X_S2H];
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
    cell_sync<N, TPB>();
  }

  // Where the flow has no gradient (dU/dx = dU/dt = 0 at every Gauss point of
  // the x cell) beta^{ln p} vanishes and so do all momentum terms: the p-face
  // flux is zero and the volume drops those terms (exactly: they are products
  // with zero).  The test is uniform over the scope of the ordering points
  // below -- the wavefront with wavefront-level ordering, else the workgroup
  // -- whose cells' records are all in LDS after the x faces, so every
  // ordering point is taken by all of its lanes alike.
  bool grad = false;
  {
    constexpr int CPW = LS::kCellsPerWave;
    const int c0 = LS::kWave ? (tid / 64) * CPW : 0;
#pragma unroll
    for (int c2 = 0; c2 < CPW; ++c2)
      if (c0 + c2 < CPB) grad |= shs[(c0 + c2) * SST + X_GRAD] != 0.0;
  }

  if constexpr (VFP_LATE_PT) load_traces(1);

  // ---- ln p faces: beta^{ln p} = a1 A^x + a2 (A^x A^x)_t per point ---------
  const int axc0 = gp(T.ax_col)[r], axc1 = gp(T.ax_col)[N + r];
  const double axv0 = gp(T.ax_val)[r], axv1 = gp(T.ax_val)[N + r];
  const int axxc0 = gp(T.axx_col)[r], axxc1 = gp(T.axx_col)[N + r];
  const double axxv0 = gp(T.axx_val)[r], axxv1 = gp(T.axx_val)[N + r], axxv2 = gp(T.axx_val)[2 * N + r];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (!grad) break;
    double own[K1], oth[K1];
    const int bc = side ? M.bc_hi[1] : M.bc_lo[1];
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      own[j] = w[j + K1 * (side ? K : 0)];
      oth[j] = use_n[1][side] ? tn[1][side][j] : (bc == 1 ? 0.0 : own[j]);
    }
    if constexpr (ADJ) {
      if (use_n[1][side] || bc != 2) {
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          own[j] -= oth[j];
          oth[j] = 0.0;
        }
      }
    }
    if (in_grp) {
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          a = fma(CB::phi[q][j], side ? own[j] : oth[j], a);
          b = fma(CB::phi[q][j], side ? oth[j] : own[j], b);
        }
        X[q * N + r] = a;
        X[(K1 + q) * N + r] = b;
      }
    }
    cell_sync<N, TPB>();
    const double iVf = sc[P_IVF + side];
    double J[K1];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      const double a1 = -sc[X_A + q] * iVf;
      double a2 = -F.t_mom * sc[X_DU + q];
      if constexpr (LINP) a2 *= sc[P2_CUF + side];
      const int code = (int)sc[C_CODE + side * K1 + q];
      const double* P1 = X + q * N;
      const double* P2 = X + (K1 + q) * N;
      const double* Pu = (code == -1) ? P1 : P2;
      double jv = a1 * fma(axv0, Pu[axc0], axv1 * Pu[axc1]) +
                  a2 * fma(axxv0, Pu[axxc0], fma(axxv1, Pu[r], axxv2 * Pu[axxc1]));
      if (code >= 0) {
        const auto tb = gp(F.pf_tab) + ((size_t)code * N + r) * (LMAX + 1);
#pragma unroll
        for (int i = 0; i <= LMAX; ++i) jv = fma(tb[i], P1[mem[i]] - P2[mem[i]], jv);
      }
      J[q] = jv;
    }
    const double scl = side ? -sc[P_S2H] : sc[P_S2H];
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
    cell_sync<N, TPB>();
  }

  // u (the stage base) is loaded now so that its latency hides behind the
  // volume work; each lane reads its own entries before writing them, which
  // keeps the in-place form w_out == u correct
  double uu[NB];
  const bool use_u = A.st.alpha != 0.0;
  if constexpr (!(VFP_LATE_U || ADJ)) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#if VFP_NT_LOAD_U
    uu[b] = use_u ? __builtin_nontemporal_load(&gp(A.st.u)[cbase + (size_t)b * N]) : 0.0;
#else
    uu[b] = use_u ? gp(A.st.u)[cbase + (size_t)b * N] : 0.0;
#endif
  }
  }
  double ff[ADJ ? NB : 1];
  const bool use_g = ADJ && gp(A.adj.fwd) && gp(A.adj.grad_nu);
  auto load_ff = [&]() {
    if constexpr (ADJ) {
#pragma unroll
      for (int b = 0; b < NB; ++b) ff[b] = use_g ? gp(A.adj.fwd)[cbase + (size_t)b * N] : 0.0;
    }
  };
  if constexpr (!(VFP_LATE_U || ADJ)) load_ff();

  // ---- volume, one row of Gauss points (fixed q1) at a time -----------------
  if constexpr (!ADJ) {
    const double g1v0 = gp(T.g1_val)[r], g1v1 = gp(T.g1_val)[N + r];
    const double g2v0 = gp(T.g2_val)[r], g2v1 = gp(T.g2_val)[N + r], g2v2 = gp(T.g2_val)[2 * N + r];
    int rc[NROT];
    double rv[NROT];
#pragma unroll
    for (int s = 0; s < NROT; ++s) {
      rc[s] = gp(T.rot_col)[s * N + r];
      rv[s] = gp(T.rot_val)[s * N + r];
    }
    const double nuc = gp(T.c_val)[r] * sc[C_NU];
    const double mom_s2hp = -F.t_mom * sc[P_S2H];
    const double t_adv = F.t_adv, t_mom = F.t_mom;
    const double tas2hx = t_adv * sc[X_S2H];
    // interpolate along x once: t[q0 + K1 j1]
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
    // GR = false: no flow gradient in the workgroup (the momentum terms and
    // the divergence term are zero)
    auto rows = [&](auto gtag) {
      constexpr bool GR = decltype(gtag)::value;
#pragma unroll
      for (int q1 = 0; q1 < K1; ++q1) {
        if (in_grp) {
#pragma unroll
          for (int q0 = 0; q0 < K1; ++q0) {
            double acc = 0.0;
#pragma unroll
            for (int j1 = 0; j1 < K1; ++j1)
              if (CB::phi[q1][j1] != 0.0) acc = fma(CB::phi[q1][j1], t[q0 + K1 * j1], acc);
            X[q0 * N + r] = acc;
          }
        }
        cell_sync<N, TPB>();
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
          const double* P = X + q0 * N;
          const double f = P[r];
          const double fxp = P[axc0], fxm = P[axc1];
          double Rf = 0.0;
#pragma unroll
          for (int s = 0; s < NROT; ++s) Rf = fma(rv[s], P[rc[s]], Rf);
          const double Axf = fma(axv0, fxp, axv1 * fxm);
          const double Xf = fma(U, f, pV * Axf);
          double G = 0.0, Pp = 0.0;
          if constexpr (GR) {
            const double dU = sc[X_DU + q0];
            const double a = sc[X_A + q0];
            const double fpp = P[axxc0], fmm = P[axxc1];
            const double G1f = fma(g1v0, fxp, g1v1 * fxm);
            const double A2f = fma(axxv0, fpp, fma(axxv1, f, axxv2 * fmm));
            const double G2f = fma(g2v0, fpp, fma(g2v1, f, g2v2 * fmm));
            const double aiV = a * piV;
            if constexpr (LINP) {
              Pp = mom_s2hp * fma(a * sc[P2_CA + q1], Axf, dU * sc[P2_CU + q1] * A2f);
            } else {
              Pp = mom_s2hp * fma(aiV, Axf, dU * A2f);
            }
            G = fma(aiV, G1f, dU * fma(t_mom, G2f, -t_adv * f));
            G = fma(-a * pid, Axf, G);
            if constexpr (LINP) G = fma(t_mom * dU, A2f, G);
          }
          G = fma(-pig, Rf, G);
          G = fma(nuc, f, G);
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            if (CB::tst[i][q0] != 0.0) ac[i] = fma(-CB::tst[i][q0], G, ac[i]);
            if (CB::dtst[i][q0] != 0.0) ac[i] = fma(CB::dtst[i][q0], Xf, ac[i]);
            if constexpr (GR)
              if (CB::tst[i][q0] != 0.0) bc[i] = fma(CB::tst[i][q0], Pp, bc[i]);
          }
        }
#pragma unroll
        for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
          for (int i0 = 0; i0 < K1; ++i0) {
            double v = res[i0 + K1 * i1];
            if (CB::tst[i1][q1] != 0.0) v = fma(CB::tst[i1][q1], ac[i0], v);
            if constexpr (GR)
              if (CB::dtst[i1][q1] != 0.0) v = fma(CB::dtst[i1][q1], bc[i0], v);
            res[i0 + K1 * i1] = v;
          }
        cell_sync<N, TPB>();
      }
    };
    if (grad) rows(std::true_type{});
    else rows(std::false_type{});
  } else {
    const double g1t0 = gp(T.g1t_val)[r], g1t1 = gp(T.g1t_val)[N + r];
    const double g2t0 = gp(T.g2t_val)[r], g2t1 = gp(T.g2t_val)[N + r], g2t2 = gp(T.g2t_val)[2 * N + r];
    int rc[NROT];
    double rv[NROT];
#pragma unroll
    for (int s = 0; s < NROT; ++s) {
      rc[s] = gp(T.rot_col)[s * N + r];
      rv[s] = gp(T.rot_val)[s * N + r];
    }
    const double nuc = gp(T.c_val)[r] * sc[C_NU];
    const double mom_s2hp = -F.t_mom * sc[P_S2H];
    const double t_adv = F.t_adv, t_mom = F.t_mom;
    const double tas2hx = t_adv * sc[X_S2H];
    auto rows = [&](auto gtag) {
      constexpr bool GR = decltype(gtag)::value;
#pragma unroll
      for (int q1 = 0; q1 < K1; ++q1) {
        if (in_grp) {
          // along ln p first for this row (values and, with a gradient,
          // ln p derivatives per x node), then along x: few values live
          double wy[K1], wdy[K1];
#pragma unroll
          for (int j0 = 0; j0 < K1; ++j0) {
            double a = 0.0, d = 0.0;
#pragma unroll
            for (int j1 = 0; j1 < K1; ++j1) {
              if (CB::phi[q1][j1] != 0.0) a = fma(CB::phi[q1][j1], w[j0 + K1 * j1], a);
              if constexpr (GR)
                if (CB::dphi[q1][j1] != 0.0) d = fma(CB::dphi[q1][j1], w[j0 + K1 * j1], d);
            }
            wy[j0] = a;
            wdy[j0] = d;
          }
#pragma unroll
          for (int q0 = 0; q0 < K1; ++q0) {
            double f = 0.0, dx = 0.0, dp = 0.0;
#pragma unroll
            for (int j0 = 0; j0 < K1; ++j0) {
              f = fma(CB::phi[q0][j0], wy[j0], f);
              if (CB::dphi[q0][j0] != 0.0) dx = fma(CB::dphi[q0][j0], wy[j0], dx);
              if constexpr (GR) dp = fma(CB::phi[q0][j0], wdy[j0], dp);
            }
            X[q0 * N + r] = f;
            X[(K1 + q0) * N + r] = dx;
            if constexpr (GR) X[(2 * K1 + q0) * N + r] = dp;
          }
        }
        cell_sync<N, TPB>();
        const double pV = tas2hx * sc[P_V + q1];
        const double piV = sc[P_IV + q1];
        const double pid = sc[P_ID + q1];
        const double pig = sc[P_IG + q1];
        double ac[K1];
#pragma unroll
        for (int i = 0; i < K1; ++i) ac[i] = 0.0;
#pragma unroll
        for (int q0 = 0; q0 < K1; ++q0) {
          const double U = sc[X_U + q0];
          const double* P = X + q0 * N;
          const double* Qx = X + (K1 + q0) * N;
          const double f = P[r];
          double Rf = 0.0;
#pragma unroll
          for (int s = 0; s < NROT; ++s) Rf = fma(rv[s], P[rc[s]], Rf);
          double G = 0.0, Pa = 0.0;
          if constexpr (GR) {
            const double dU = sc[X_DU + q0];
            const double a = sc[X_A + q0];
            const double* Qp = X + (2 * K1 + q0) * N;
            const double fxp = P[axc0], fxm = P[axc1];
            const double fpp = P[axxc0], fmm = P[axxc1];
            const double Axf = fma(axv0, fxp, axv1 * fxm);
            const double G1t = fma(g1t0, fxp, g1t1 * fxm);
            const double G2t = fma(g2t0, fpp, fma(g2t1, f, g2t2 * fmm));
            const double aiV = a * piV;
            G = fma(aiV, G1t, dU * fma(t_mom, G2t, -t_adv * f));
            G = fma(-a * pid, Axf, G);
            const double Axp = fma(axv0, Qp[axc0], axv1 * Qp[axc1]);
            const double A2p = fma(axxv0, Qp[axxc0], fma(axxv1, Qp[r], axxv2 * Qp[axxc1]));
            if constexpr (LINP) {
              // (A^x A^x)_t is symmetric: the divergence term is its own transpose
              G = fma(t_mom * dU, fma(axxv0, fpp, fma(axxv1, f, axxv2 * fmm)), G);
              Pa = mom_s2hp * fma(a * sc[P2_CA + q1], Axp, dU * sc[P2_CU + q1] * A2p);
            } else {
              Pa = mom_s2hp * fma(aiV, Axp, dU * A2p);
            }
          }
          G = fma(pig, Rf, G);                // (B.Omega)^T = -B.Omega
          G = fma(nuc, f, G);
          const double Axd = fma(axv0, Qx[axc0], axv1 * Qx[axc1]);
          const double Xa = fma(U, Qx[r], pV * Axd);
          const double h = GR ? Xa + Pa - G : Xa - G;
#pragma unroll
          for (int i = 0; i < K1; ++i)
            if (CB::tst[i][q0] != 0.0) ac[i] = fma(CB::tst[i][q0], h, ac[i]);
        }
#pragma unroll
        for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
          for (int i0 = 0; i0 < K1; ++i0)
            if (CB::tst[i1][q1] != 0.0) res[i0 + K1 * i1] = fma(CB::tst[i1][q1], ac[i0], res[i0 + K1 * i1]);
        cell_sync<N, TPB>();
      }
    };
    if (grad) rows(std::true_type{});
    else rows(std::false_type{});
  }

  // ---- source and output ---------------------------------------------------
  if constexpr (ADJ) {
    // (M1 x M1) v on the reference cell
    auto ref_mass2 = [&](double* v) {
      double tm[NB];
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) {
          double acc = 0.0;
#pragma unroll
          for (int j0 = 0; j0 < K1; ++j0) acc = fma(CB::mass[i0][j0], v[j0 + K1 * i1], acc);
          tm[i0 + K1 * i1] = acc;
        }
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) {
          double acc = 0.0;
#pragma unroll
          for (int j1 = 0; j1 < K1; ++j1) acc = fma(CB::mass[i1][j1], tm[i0 + K1 * j1], acc);
          v[i0 + K1 * i1] = acc;
        }
    };
    if constexpr (VFP_LATE_U || ADJ) load_ff();
    const double jac = 1.0 / (sc[X_S2H] * sc[P_S2H]);
    if (A.adj.mass_out) {
      ref_mass2(res);
#pragma unroll
      for (int b = 0; b < NB; ++b) res[b] *= jac;
    }
    if (use_g) {
      // d/dnu_c of <M mu, beta L(fwd)> = -beta t_col sum C (M mu) . fwd
      ref_mass2(w);
      double part = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) part = fma(w[b], ff[b], part);
      part *= gp(T.c_val)[r] * jac;
      // one add per cell and launch, so stream order keeps the sum
      // reproducible; nothing waits for the old value
      if constexpr (N == 16 && LS::kThreads == 64) {
        // the cell's 16 lanes are one DPP row: a register reduction
        const double sum = row16_sum(part);
        if (act && r == 0) atomicAdd(&A.adj.grad_nu[cell], -A.st.beta * F.t_col * sum);
      } else {
        if (in_grp) X[r] = part;
        cell_sync<N, TPB>();
        if (act && r == 0) {
          double sum = 0.0;
          for (int j = 0; j < N; ++j) sum += X[j];
          atomicAdd(&A.adj.grad_nu[cell], -A.st.beta * F.t_col * sum);
        }
      }
    }
    if (act && gp(A.adj.t_out)) {
#pragma unroll
      for (int b = 0; b < NB; ++b) gp(A.adj.t_out)[cbase + (size_t)b * N] = A.st.beta * res[b];
    }
  } else if (A.st.with_source && gp(F.src) && r == 0 && act) {
    double src[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) src[b] = gp(F.src)[(size_t)cell * NB + b];
#pragma unroll
    for (int b = 0; b < NB; ++b) res[b] += src[b];
  }
  // the adjoint loads its stage base and forward state last (fewer live
  // registers through the volume; measured faster)
  if constexpr (VFP_LATE_U || ADJ) {
#pragma unroll
    for (int b = 0; b < NB; ++b) uu[b] = use_u ? gp(A.st.u)[cbase + (size_t)b * N] : 0.0;
  }
  // the adjoint may add one more state to its output (the reverse sweep's
  // running sum, carried one stage late)
  double ad[ADJ ? NB : 1];
  bool use_ad = false;
  if constexpr (ADJ) {
    use_ad = gp(A.adj.add_in) != nullptr;
#pragma unroll
    for (int b = 0; b < NB; ++b) ad[b] = use_ad ? gp(A.adj.add_in)[cbase + (size_t)b * N] : 0.0;
  }
  if (act && (!ADJ || gp(A.st.w_out))) {
    const double al = A.st.alpha, be = A.st.beta;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = fma(be, res[b], al * uu[b]);
      if constexpr (ADJ) {
        if (use_ad) v += ad[b];
      }
#if VFP_NT_STORE
      // the stage output is not read again in this launch: streaming stores
      // keep it from displacing the neighbour traces in L2
      __builtin_nontemporal_store(v, &gp(A.st.w_out)[cbase + (size_t)b * N]);
#else
      gp(A.st.w_out)[cbase + (size_t)b * N] = v;
#endif
    }
  }
}

// Launch order -> tile so that each XCD owns one contiguous range of tiles
// (workgroups are dealt to the 8 XCDs round robin in launch order): a tile's
// x-neighbours are then processed by the same XCD, through the same L2.
__device__ __forceinline__ int xcd_tile(int item, int total) {
  constexpr int kXcd = 8;
  const int x = item % kXcd, i = item / kXcd;
  const int per = total / kXcd, rem = total % kXcd;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

}  // namespace shock
}  // namespace vfp
