// Kernel argument blocks shared by the host library and the HIP kernels.
#pragma once
#include <cstdint>

namespace vfp {

constexpr int kMaxLmax = 11;     // above 7: runs along x with B along x only (general kernels)
constexpr int kMaxN = (kMaxLmax + 1) * (kMaxLmax + 1);
constexpr int kMaxK = 5;           // general kernels: k <= 5 on one axis, 3 on two, 2 on three
constexpr int kMaxK1 = kMaxK + 1;
constexpr int kMaxUniSlots = 24;   // max non-zeros per row of a uniform-axis face matrix
constexpr int kRec = 16;           // doubles per packed x / p scalar record

// One-dimensional basis data for degree K on the reference interval [-1,1]:
// Gauss-Lobatto Lagrange basis l_j, (K+1)-point Gauss rule (g_q, w_q), and
// the 1-D mass matrix M1_ij = sum_q w_q l_i(g_q) l_j(g_q) (exact).  Entries
// beyond K+1 are zero.
struct Basis1D {
  double phi[kMaxK1][kMaxK1];    // phi[q][j]  = l_j(g_q)
  double tst[kMaxK1][kMaxK1];    // tst[i][q]  = sum_j (M1^{-1})_ij l_j(g_q) w_q
  double dtst[kMaxK1][kMaxK1];   // dtst[i][q] = sum_j (M1^{-1})_ij l_j'(g_q) w_q
  double lift[2][kMaxK1];        // lift[side][i] = (M1^{-1})_{i, 0 or K}
  double dphi[kMaxK1][kMaxK1];   // dphi[q][j] = l_j'(g_q)
  double dvol[kMaxK1][kMaxK1];   // dvol[i][j] = sum_q dtst[i][q] phi[q][j]: the 1-D volume derivative
                                 // term of a coefficient constant on the cell, in node space
  double mass[kMaxK1][kMaxK1];   // M1
  double imass[kMaxK1][kMaxK1];  // M1^{-1}
};

// Per-row (lms) sparse rows of the spherical-harmonic matrices, stored
// structure-of-arrays: field[slot * n + row].  Missing entries point at the
// row itself with value 0.
struct RowTables {
  const int* ax_col;    // 2 slots: (l+1,m,s), (l-1,m,s)            A^x
  const double* ax_val;
  const double* g1_val; // same columns: (A^y Om^z - A^z Om^y)_t
  const int* axx_col;   // 2 slots: (l+2,m,s), (l-2,m,s)            (A^x A^x)_t
  const double* axx_val;// 3 slots: l+2, self, l-2
  const double* g2_val; // same columns: (A^x (A^y Om^z - A^z Om^y))_t
  const double* g1t_val;// transposes of G1 and G2 on the same (symmetric) patterns
  const double* g2t_val;
  const int* om_col;    // 3 matrices x 2 slots: Omega^x, Omega^y, Omega^z
  const double* om_val;
  const int* ayz_col;   // 2 matrices x 4 slots: A^y, A^z
  const double* ayz_val;
  const double* c_val;  // l(l+1)/2
  // eigen data of A^x restricted to the (m,s) block of each row
  const int* blk_mem;   // (lmax+1) slots: lms indices of the block members
  const double* w_row;  // (lmax+1) slots: W[row][i]
  const double* w_col;  // (lmax+1) slots: W[member j][pos(row)]
  const double* lam;    // eigenvalue of characteristic pos(row)
  // rotation row (B . Omega) for a uniform B, padded to nrot slots
  const int* rot_col;
  const double* rot_val;
  int nrot;
  // dense eigen-decomposition of A^a per spatial axis (point flows):
  // wd[a][j n + k] = W[j][k] (orthonormal columns), lamd[a][k] = lambda_k
  const double* wd[3];
  const double* lamd[3];
  // uniform-axis face matrices beta^a and |beta^a| (per spatial axis)
  const int* fb_col[3];
  const double* fb_val[3];
  const int* fa_col[3];
  const double* fa_val[3];
  int nfb[3];
  int nfa[3];
};

struct FieldArgs {
  // planar flow along x (profile) -- used by the kernels built for a planar profile
  const double* u_vol;   // [N0 (k+1)]
  const double* du_vol;
  const double* a_vol;
  const double* u_face;  // [N0 + 1]
  double U[3];           // uniform flow components (y, z always; x without a profile)
  // flow at the points (kernels built for point flows): [cell][q][4] holding
  // U^x, U^y, U^z and div U (summed over the run's spatial axes); and per
  // axis a the normal component U^a at the face points [face][qf], faces
  // numbered over (N_a + 1) positions on axis a and N_b on the others (axis 0
  // fastest), points over the other axes in increasing order (first fastest)
  const double* u_pts;
  const double* uf_pts[3];
  // momentum axis profiles (ln p): at volume points [Np (k+1)] and faces [Np+1]
  const double* V_vol;
  const double* iV_vol;   // 1/V
  const double* idiv_vol; // -div beta holds -dU/dt idiv A^x: m/(gamma p) (ln p) or -V (linear p)
  const double* ig_vol;   // q/(gamma m)
  const double* iV_face;  // coefficient of dU/dt in beta^p at p faces: 1/V (ln p) or gamma m (p)
  // along the momentum axis beta^p = -t_mom (dU/dt ca A^x + U' cu (A^x A^x)_t):
  // ln p: ca = 1/V, cu = 1; linear p: ca = gamma m, cu = p
  const double* ca_vol;   // [Np (k+1)]
  const double* cu_vol;
  const double* cu_face;  // [Np + 1]
  double t_divu;          // 1 on a linear p axis: -div beta holds + U' (A^x A^x)_t
  double V0, iV0, ig0;    // fixed-momentum values
  // p-face upwind data: code per (p face, x point) stored [pf][x point]:
  // -1 beta>=0, -2 beta<=0, >= 0 index into pf_tab ([code][n][lmax+1] rows of
  // beta_+ in the block)
  const int* pf_code;
  const double* pf_coded;   // the same codes as doubles (staged into LDS as is)
  const double* pf_tab;
  const double* pf_dtab;    // [code][2][n][lmax+1] rows of dB_+ in the directions A^x, (A^xA^x)_t
  // packed per-cell-row scalars for the (x, ln p) kernel (kRec doubles each):
  // xrec[ix]: t_adv (2/h_x) U(x_q) [3], U'(x_q) [3], t_mom dU/dt(x_q) [3],
  //           t_adv U at the lo / hi face [2], 2/h_x, gradient flag
  //           (1 if dU/dx or dU/dt is non-zero at one of its Gauss points)
  // prec[ip]: V(p_q) [3], 1/V [3], m/(gamma p) [3], t_rot q/(gamma m) [3],
  //           t_mom / V at the lo / hi face [2], 2/h_p
  const double* xrec;
  const double* prec;
  const double* prec2;    // linear p axis: [ip][8] gamma m (3), p (3) at the Gauss points, p at the faces (2)
  // magnetic field
  double B[3];            // uniform B
  const double* B_pts;    // [cell][q][3] or null
  // scattering and source
  double nu0;
  const double* nu_cell;  // [cell] or null
  const double* nu_pts;   // [cell][q] at the volume points, or null (takes precedence)
  const double* src;      // [cell][nb] = M^{-1} h (000 component) or null
  // term multipliers (0 or 1)
  double t_adv, t_mom, t_rot, t_col;
};

struct MeshArgs {
  int n[3];               // cells per axis (1 for unused axes)
  int ncells;
  int bc_lo[3], bc_hi[3];
  const double* s2h[3];   // 2 / h per cell along each axis
};

struct StageArgs {
  const double* w_in;
  const double* u;        // may be null when alpha == 0
  double* w_out;
  double alpha;           // w_out = alpha u + beta L(w_in)
  double beta;
  int with_source;
};

// Extra outputs of the adjoint kernels (operator K = -M^{-1} D^T, acting on
// mu = M^{-1} lambda).  With st.alpha = 1 the kernel forms t = beta K(w_in),
// writes t_out (if not null) and w_out = u + t.
struct AdjArgs {
  double* t_out;          // may be null
  const double* fwd;      // forward stage input paired with w_in for d/dnu, or null
  double* grad_nu;        // [cell] accumulated: -beta t_col sum C (M fwd) . w_in
  int mass_out;           // 1: multiply the result by the cell mass matrix
  // (x, ln p) kernels only: a state added to w_out (null: none), and w_out
  // may then be null to skip that output
  const double* add_in;
};

struct KernelArgs {
  MeshArgs mesh;
  FieldArgs fld;
  RowTables tab;
  StageArgs st;
  AdjArgs adj;
  int tile_map;           // 1: launch order -> tile by XCD ranges (shock kernels)
};

// Batched (x, ln p) stage: one launch covers the tiles of many runs.  Run r
// owns tiles [start[r], start[r+1]); descs[r] holds its arguments.
struct BatchArgs {
  const KernelArgs* descs;
  const int* start;       // nruns + 1 prefix sums of tiles
  const int* tile_run;    // [total] run of each tile
  int nruns;
  int total;              // start[nruns]
  int tile_map;
};

}  // namespace vfp
