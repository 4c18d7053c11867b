// Sensitivities of one Runge-Kutta stage to the planar flow profile, for the
// gradients of a loss with respect to the shock-profile parameters.
//
// For a stage w_i = u + c dt L(w_{i-1}) with adjoint lambda_i = M mu_i,
//     dJ/dfield += c dt <mu_i, d(h - D w_{i-1}) / dfield>
// (L = M^{-1}(h - D w), eq. matrix-formulation-system-odes; h does not depend
// on the flow).  D depends on the planar flow U(x) through
//   volume  (eq. definition-mass-and-dg-matrix):
//     -phi (R - div beta) f + (grad phi) . beta f at each Gauss point, with
//     beta^x = t_adv (U + V A^x), beta^{ln p} = -t_mom (a/V A^x + U' (A^xA^x)_t),
//     R - div beta containing  t_mom (a/V G1 + U' G2 - a m/(gamma p) A^x)
//     - t_adv U' (a = dU/dt, U' = dU/dx, G1, G2 the truncated products of the
//     shock terms);
//   x faces (eq. definition-upwind-flux): J = W(max(m,0) W^T f1 + min(m,0)
//     W^T f2), m = t_adv (U_F + lambda V) the speeds along the constant
//     eigenvectors W of A^x, so dJ/dU_F = t_adv W (H(m) W^T f1 + (1 - H(m))
//     W^T f2), H the Heaviside step (1/2 at 0);
//   ln p faces: J = B_+ f1 + B_- f2 = B_+ (f1 - f2) + B f2 with B = a1 A^x +
//     a2 (A^xA^x)_t, a1 = -t_mom a / V_F, a2 = -t_mom U'; B_+ is differentiated
//     on its spectral decomposition B = Q diag(l) Q^T (Daleckii-Krein):
//       dB_+ = Q (Gamma o (Q^T dB Q)) Q^T,  Gamma_kl = (l_k^+ - l_l^+)/(l_k - l_l)
//     (H(l_k) where l_k = l_l), tabulated on the host for the two directions
//     dB = A^x, (A^xA^x)_t at every mixed-sign point; where B is definite,
//     dB_+ = dB or 0.
// On a face from T1 (below) to T2 (above) the pairing is  int_F (mu_2 - mu_1).J
// (the trace of a cell outside the mesh counts as zero).
//
// Each cell accumulates into its own slots: its x Gauss points
// (summed over its p points), its lower x and ln p faces, and its upper faces
// where they are the (non-periodic) end of the mesh.  The lanes of a cell
// exchange forward values through a few LDS rows for the l-coupling and sum
// their shares of the slots through the same rows, and one lane adds each
// slot's sum with an atomic add that nothing waits for (a slot receives one
// add per launch, so launches in stream order give a reproducible sum).
// fgrad_reduce sums the slots per x point.  Given a grad_nu array, the U part
// also adds the stage's dJ/dnu term per cell (the collision pairing of the
// same mu and forward state), so that a reverse sweep with both gradients
// need not read the forward state in its adjoint stages.
#include <type_traits>

#include "basis.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kFgThreads = 64;

// The workgroup is one wavefront: LDS operations of a wavefront complete in
// order, so ordering the exchanges needs only a wavefront-scope fence (no
// wait for outstanding global loads, as a workgroup barrier would imply).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K>
struct GSlots {
  static constexpr int K1 = K + 1;
  static constexpr int VOL = 0;            // [K1 x points][3]: U, U', a (summed over the p points)
  static constexpr int XF = 3 * K1;        // [2]: lower, upper x face
  static constexpr int PF = XF + 2;        // [2 sides][K1 x points][2]: a, U'
  static constexpr int SIZE = PF + 4 * K1;
};

// Heaviside with H(0) = 1/2
__device__ __forceinline__ double heav(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5); }

// The sensitivities split in two parts over the same cells (workgroups of
// one launch):
//   PART 0: dJ/dU at the x Gauss points (volume) and dJ/dU_F (x faces), for
//           every cell;
//   PART 1: dJ/dU' and dJ/d(dU/dt) (volume and ln p faces), for the cells of
//           the support only: a workgroup without a support cell returns at
//           once (the decision is uniform over the workgroup).
// They write disjoint slots of a cell.
template <int K, int PART>
struct FgRows {
  static constexpr int K1 = K + 1;
  // partial-sum rows reduced per cell at the end, and LDS rows per cell
  static constexpr int NRED = PART == 0 ? K1 + 2 : 6 * K1;
  static constexpr int NEX = PART == 0 ? 3 * K1 : 2 * K1;   // exchange rows of a face
  static constexpr int XRW = NRED > NEX ? NRED : NEX;
  // slot of reduction row j
  __device__ static constexpr int slot(int j) {
    using S = GSlots<K>;
    if (PART == 0) return j < K1 ? S::VOL + 3 * j : S::XF + (j - K1);
    return j < 2 * K1 ? S::VOL + 3 * (j >> 1) + 1 + (j & 1) : S::PF + (j - 2 * K1);
  }
};

// waves per SIMD the register allocation aims for
#ifndef VFP_FG_WAVES
#define VFP_FG_WAVES 2
#endif

template <int K, int LMAX, int PART>
__device__ __forceinline__ void fgrad_body(const KernelArgs& A, const double* __restrict__ mu,
                                           const double* __restrict__ fwd, double cdt,
                                           double* __restrict__ slots, const unsigned char* __restrict__ support,
                                           double* __restrict__ grad_nu, double* lds, int blk) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = K1 * K1;
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  using CB = CBasis<K>;
  using S = GSlots<K>;
  using FR = FgRows<K, PART>;
  constexpr int NS = S::SIZE;
  constexpr int XRW = FR::XRW;
  constexpr int ax = PART == 0 ? 0 : 1;     // the face axis of this part

  const int tid = threadIdx.x;
  const int cl = tid / N;
  const int r = tid - cl * N;
  const bool in_grp = cl < CPB;
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;
  const RowTables& T = A.tab;
  const int nx = M.n[0], np = M.n[1];
  if constexpr (PART == 1) {
    if (support) {
      bool any = false;
      for (int c2 = 0; c2 < CPB; ++c2) {
        const int cc = blk * CPB + c2;
        if (cc < M.ncells) any |= support[cc % nx] != 0;
      }
      if (!any) return;
    }
  }
  const int cell0 = blk * CPB + cl;
  const bool act = in_grp && cell0 < M.ncells;
  const int cell = act ? cell0 : 0;
  const int ix = cell % nx, ip = cell / nx;
  double* X = lds + (in_grp ? cl : 0) * XRW * N;

  // ---- the cell's values and the neighbour traces along this part's axis
  const size_t cbase = (size_t)cell * NB * N + r;
  double w[NB], m[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    w[b] = fwd[cbase + (size_t)b * N];
    m[b] = mu[cbase + (size_t)b * N];
  }
  const int ia = ax ? ip : ix, na = ax ? np : nx;
  double nf[2][K1], nm[2][K1];
  bool usen[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int st = ax ? nx : 1;
    int ni = side ? ia + 1 : ia - 1;
    const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
    usen[side] = (ni >= 0 && ni < na) || bc == 0;
    ni = (ni + na) % na;
    const size_t nb0 = (size_t)(cell + (ni - ia) * st) * NB * N + r;
    const int jn = side ? 0 : K;
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      const int node = ax ? (j + K1 * jn) : (jn + K1 * j);
      nf[side][j] = fwd[nb0 + (size_t)node * N];
      nm[side][j] = mu[nb0 + (size_t)node * N];
    }
  }
  // the ln p face codes are loaded with the state, so that the derivative
  // table rows they select cost one round trip later, not two
  int pcode[2][K1];
  if constexpr (PART == 1) {
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < K1; ++q) pcode[side][q] = F.pf_code[(size_t)(ip + side) * (nx * K1) + ix * K1 + q];
  }
  const double* xr = F.xrec + (size_t)ix * kRec;
  const double* pr = F.prec + (size_t)ip * kRec;
  const double s2hx = xr[11], s2hp = pr[14];
  const double jac = 1.0 / (s2hx * s2hp);
  const double t_adv = F.t_adv, t_mom = F.t_mom;
  const double gw[3] = {K == 1 ? 1.0 : 5.0 / 9.0, K == 1 ? 1.0 : 8.0 / 9.0, 5.0 / 9.0};
  // the l-block of this lane's row (members, eigenvector column, eigenvalue
  // of A^x) and, for the x faces, U at the faces and V at the p points
  int mem[LMAX + 1];
  double wcol[LMAX + 1];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    mem[i] = T.blk_mem[i * N + r];
    if constexpr (PART == 0) wcol[i] = T.w_col[i * N + r];
  }
  double lam = 0.0, uxf[2] = {0.0, 0.0}, vq[K1];
  if constexpr (PART == 0) {
    lam = T.lam[r];
    uxf[0] = xr[9];
    uxf[1] = xr[10];
#pragma unroll
    for (int q = 0; q < K1; ++q) vq[q] = pr[q];
  }

  // this lane's share of the reduction rows (FgRows::slot)
  double red[FR::NRED];
#pragma unroll
  for (int i = 0; i < FR::NRED; ++i) red[i] = 0.0;

  // ---- volume, one row of Gauss points (fixed q1) at a time: interpolate
  // along ln p first (K1 values per row), then along x (a loop, not
  // unrolled, so that the rows do not all stay live at once)
#pragma unroll 1
  for (int q1 = 0; q1 < K1; ++q1) {
    const double gw1 = (K == 1) ? 1.0 : (q1 == 1 ? 8.0 / 9.0 : 5.0 / 9.0);
    double wy[K1], my[K1], mdy[K1];
#pragma unroll
    for (int j0 = 0; j0 < K1; ++j0) {
      double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
      for (int j1 = 0; j1 < K1; ++j1) {
        a = fma(CB::phi[q1][j1], w[j0 + K1 * j1], a);
        b = fma(CB::phi[q1][j1], m[j0 + K1 * j1], b);
        if constexpr (PART == 1) c = fma(CB::dphi[q1][j1], m[j0 + K1 * j1], c);
      }
      wy[j0] = a;
      my[j0] = b;
      mdy[j0] = c;
    }
    if constexpr (PART == 0) {
      // dJ/dU: t_adv (2/h_x) (d_x mu) f, no exchange
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        double f = 0.0, mx = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) {
          f = fma(CB::phi[q0][j0], wy[j0], f);
          mx = fma(CB::dphi[q0][j0], my[j0], mx);
        }
        red[q0] += gw[q0] * gw1 * jac * (s2hx * t_adv * mx * f);
      }
    } else {
      // dJ/dU' and dJ/d(dU/dt): the momentum and divergence terms, with the
      // l-coupling of f through LDS
      const int axc0 = T.ax_col[r], axc1 = T.ax_col[N + r];
      const double axv0 = T.ax_val[r], axv1 = T.ax_val[N + r];
      const int axxc0 = T.axx_col[r], axxc1 = T.axx_col[N + r];
      const double axxv0 = T.axx_val[r], axxv1 = T.axx_val[N + r], axxv2 = T.axx_val[2 * N + r];
      const double g1v0 = T.g1_val[r], g1v1 = T.g1_val[N + r];
      const double g2v0 = T.g2_val[r], g2v1 = T.g2_val[N + r], g2v2 = T.g2_val[2 * N + r];
      double fq[K1];
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        double f = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) f = fma(CB::phi[q0][j0], wy[j0], f);
        fq[q0] = f;
        if (in_grp) X[q0 * N + r] = f;
      }
      wave_sync();
      const double iV = pr[3 + q1], pid = pr[6 + q1];
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        double mq = 0.0, mp = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) {
          mq = fma(CB::phi[q0][j0], my[j0], mq);
          mp = fma(CB::phi[q0][j0], mdy[j0], mp);
        }
        const double* P = X + q0 * N;
        const double f = fq[q0];
        const double Axf = fma(axv0, P[axc0], axv1 * P[axc1]);
        const double A2f = fma(axxv0, P[axxc0], fma(axxv1, f, axxv2 * P[axxc1]));
        const double G1f = fma(g1v0, P[axc0], g1v1 * P[axc1]);
        const double G2f = fma(g2v0, P[axxc0], fma(g2v1, f, g2v2 * P[axxc1]));
        const double wq = gw[q0] * gw1 * jac;
        red[2 * q0 + 0] += wq * (-mq * (t_mom * G2f - t_adv * f) - s2hp * t_mom * mp * A2f);
        red[2 * q0 + 1] += wq * (-mq * t_mom * (iV * G1f - pid * Axf) - s2hp * t_mom * t_mom * mp * iV * Axf);
      }
      wave_sync();
    }
  }

  // ---- faces along this part's axis: the cell's lower face, and its upper
  // face where it is the (non-periodic) end of the mesh; on a face from T1
  // (below) to T2 (above) the pairing is int_F (mu_2 - mu_1) . dJ, with the
  // trace of a cell outside the mesh counted as zero.  One side at a time:
  // the side's f1, f2 rows go to rows [0, 2 K1) of X.
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
    const bool valid = act && (side == 0 || (ia == na - 1 && bc != 0));
    double dmu[K1];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double fo = 0.0, fn = 0.0, mo = 0.0, mn = 0.0;
#pragma unroll
      for (int j = 0; j < K1; ++j) {
        const double ph = CB::phi[q][j];
        const int node = ax ? (j + K1 * (side ? K : 0)) : ((side ? K : 0) + K1 * j);
        fo = fma(ph, w[node], fo);
        fn = fma(ph, nf[side][j], fn);
        mo = fma(ph, m[node], mo);
        mn = fma(ph, nm[side][j], mn);
      }
      if (!usen[side]) {
        fn = (bc == 1) ? 0.0 : fo;   // exterior of zero inflow / continuous
        mn = 0.0;
      }
      dmu[q] = valid ? (side ? mn - mo : mo - mn) : 0.0;   // mu_2 - mu_1
      if (in_grp) {
        X[q * N + r] = side ? fo : fn;          // f1 (lower cell)
        X[(K1 + q) * N + r] = side ? fn : fo;   // f2 (upper cell)
        if constexpr (PART == 0) X[(2 * K1 + q) * N + r] = gw[q] * dmu[q];
      }
    }
    wave_sync();
    const double* R1 = X;
    const double* R2 = X + K1 * N;
    if constexpr (PART == 0) {
      // x face: dJ/dU_F = t_adv W (H(m) c1 + (1 - H(m)) c2), c = W^T f, paired
      // with mu_2 - mu_1 over the lanes: sum_r dmu_r (W d)_r = sum_k d_k
      // (W^T dmu)_k, so lane k forms d_k (W^T dmu)_k and the cell's
      // reduction sums them (rows [2 K1, 3 K1) hold gw dmu)
      const double* Rm = X + 2 * K1 * N;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double c1 = 0.0, c2 = 0.0, cm = 0.0;
#pragma unroll
        for (int j = 0; j <= LMAX; ++j) {
          c1 = fma(wcol[j], R1[q * N + mem[j]], c1);
          c2 = fma(wcol[j], R2[q * N + mem[j]], c2);
          cm = fma(wcol[j], Rm[q * N + mem[j]], cm);
        }
        const double h = heav(uxf[side] + t_adv * lam * vq[q]);
        acc = fma(t_adv * (h * c1 + (1.0 - h) * c2), cm, acc);
      }
      red[K1 + side] = acc / s2hp;
    } else {
      // ln p face: dJ = dB_+ (f1 - f2) + dB f2 (dB f1 where B >= 0)
      const int axc0 = T.ax_col[r], axc1 = T.ax_col[N + r];
      const double axv0 = T.ax_val[r], axv1 = T.ax_val[N + r];
      const int axxc0 = T.axx_col[r], axxc1 = T.axx_col[N + r];
      const double axxv0 = T.axx_val[r], axxv1 = T.axx_val[N + r], axxv2 = T.axx_val[2 * N + r];
      const double tmv = pr[12 + side];     // t_mom / V at this face
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        const int code = pcode[side][q];
        const double* Pu = (code == -1) ? R1 + q * N : R2 + q * N;
        double ja = -t_mom * tmv * fma(axv0, Pu[axc0], axv1 * Pu[axc1]);
        double ju = -t_mom * fma(axxv0, Pu[axxc0], fma(axxv1, Pu[r], axxv2 * Pu[axxc1]));
        if (code >= 0) {
          // dB_+ (f1 - f2) from the rows of the derivative tables of B_+
          const double* ta = F.pf_dtab + ((size_t)code * 2 * N + r) * (LMAX + 1);
          const double* tx = ta + (size_t)N * (LMAX + 1);
          double dkA = 0.0, dkX = 0.0;
#pragma unroll
          for (int i = 0; i <= LMAX; ++i) {
            const double dfi = R1[q * N + mem[i]] - R2[q * N + mem[i]];
            dkA = fma(ta[i], dfi, dkA);
            dkX = fma(tx[i], dfi, dkX);
          }
          ja = fma(-t_mom * tmv, dkA, ja);
          ju = fma(-t_mom, dkX, ju);
        }
        red[2 * K1 + side * 2 * K1 + 2 * q + 0] = gw[q] * dmu[q] * ja / s2hx;
        red[2 * K1 + side * 2 * K1 + 2 * q + 1] = gw[q] * dmu[q] * ju / s2hx;
      }
    }
    wave_sync();
  }

  // ---- one reduction over the cell's lanes for this part's slots; each
  // slot gets one add per launch, in stream order across launches (so the
  // sum is reproducible), with no returned value, so nothing waits for it
  if constexpr (N == 16) {
    // the cell's 16 lanes are one DPP row: register reductions, lane r
    // adding slot r (and r + 16)
    double mine = 0.0, mine2 = 0.0;
#pragma unroll
    for (int i = 0; i < FR::NRED; ++i) {
      const double sum = row16_sum(red[i]);
      if (i == r) mine = sum;
      if (i == r + 16) mine2 = sum;
    }
    if (act && r < FR::NRED) atomicAdd(&slots[(size_t)cell * NS + FR::slot(r)], cdt * mine);
    if (act && r + 16 < FR::NRED) atomicAdd(&slots[(size_t)cell * NS + FR::slot(r + 16)], cdt * mine2);
  } else {
    if (in_grp)
#pragma unroll
      for (int i = 0; i < FR::NRED; ++i) X[i * N + r] = red[i];
    wave_sync();
    if (act)
      for (int j = r; j < FR::NRED; j += N) {
        double sum = 0.0;
        for (int l = 0; l < N; ++l) sum += X[j * N + l];
        atomicAdd(&slots[(size_t)cell * NS + FR::slot(j)], cdt * sum);
      }
  }

  // ---- dJ/dnu of the cell from the same pair (the U part runs on every
  // cell): the collision term's pairing -cdt t_col sum_r c_r (M mu)_r . f_r,
  // with (M mu) the reference mass (M1 x M1) applied to the lane's row and
  // scaled by the cell's Jacobian; the products and their order are those
  // of the adjoint stage's own accumulation, so either place gives the same
  // per-cell term
  if constexpr (PART == 0) {
    if (grad_nu) {
      double tm[NB], mm[NB];
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) {
          double a = 0.0;
#pragma unroll
          for (int j0 = 0; j0 < K1; ++j0) a = fma(CB::mass[i0][j0], m[j0 + K1 * i1], a);
          tm[i0 + K1 * i1] = a;
        }
#pragma unroll
      for (int i1 = 0; i1 < K1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < K1; ++i0) {
          double a = 0.0;
#pragma unroll
          for (int j1 = 0; j1 < K1; ++j1) a = fma(CB::mass[i1][j1], tm[i0 + K1 * j1], a);
          mm[i0 + K1 * i1] = a;
        }
      double part = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) part = fma(mm[b], w[b], part);
      part *= T.c_val[r] * jac;
      if constexpr (N == 16) {
        const double sum = row16_sum(part);
        if (act && r == 0) atomicAdd(&grad_nu[cell], -cdt * F.t_col * sum);
      } else {
        wave_sync();
        if (in_grp) X[r] = part;
        wave_sync();
        if (act && r == 0) {
          double sum = 0.0;
          for (int j = 0; j < N; ++j) sum += X[j];
          atomicAdd(&grad_nu[cell], -cdt * F.t_col * sum);
        }
      }
    }
  }
}

// Both parts in one launch, spread evenly over the grid so that the two
// interleave on the machine (each is bound by memory latency, not
// bandwidth): of the nblk + np1 workgroups, workgroup i takes part 1 where
// floor((i + 1) np1 / total) steps past floor(i np1 / total), and part 0
// otherwise.  p1_blocks lists the tiles that hold a support cell (np1 of
// them), so that no workgroup is spent on a tile without one; null means
// every tile (np1 = nblk: even workgroups part 0, odd ones part 1), and
// then part 1 checks the support itself.
template <int K, int LMAX>
__global__ __launch_bounds__(kFgThreads) __attribute__((amdgpu_waves_per_eu(VFP_FG_WAVES)))
void fgrad_kernel(KernelArgs A, const double* __restrict__ mu, const double* __restrict__ fwd, double cdt,
                  double* __restrict__ slots, const unsigned char* __restrict__ support,
                  const int* __restrict__ p1_blocks, int nblk, int np1, double* __restrict__ grad_nu) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  constexpr int X0 = FgRows<K, 0>::XRW, X1 = FgRows<K, 1>::XRW;
  __shared__ double lds[CPB * (X0 > X1 ? X0 : X1) * N];
  const long long total = (long long)nblk + np1, i = blockIdx.x;
  const int c0 = (int)(i * np1 / total), c1 = (int)((i + 1) * np1 / total);
  if (c1 > c0)
    fgrad_body<K, LMAX, 1>(A, mu, fwd, cdt, slots, p1_blocks ? nullptr : support, nullptr, lds,
                           p1_blocks ? p1_blocks[c0] : c0);
  else
    fgrad_body<K, LMAX, 0>(A, mu, fwd, cdt, slots, support, grad_nu, lds, (int)i - c0);
}

// g_u, g_dudx, g_dudt at the nx (k+1) x Gauss points and g_uface at the nx+1
// x faces, summed over the slots of every cell.
template <int K>
__global__ void fgrad_reduce_kernel(MeshArgs M, const double* __restrict__ slots, double* g_u, double* g_du,
                                    double* g_a, double* g_uf) {
  using S = GSlots<K>;
  constexpr int K1 = K + 1;
  const int nx = M.n[0], np = M.n[1];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nx * K1) {
    const int ix = t / K1, q0 = t - ix * K1;
    double su = 0.0, sd = 0.0, sa = 0.0;
    for (int ip = 0; ip < np; ++ip) {
      const double* o = slots + (size_t)(ip * nx + ix) * S::SIZE;
      su += o[S::VOL + 3 * q0 + 0];
      sd += o[S::VOL + 3 * q0 + 1];
      sa += o[S::VOL + 3 * q0 + 2];
      sa += o[S::PF + 2 * q0 + 0] + o[S::PF + 2 * K1 + 2 * q0 + 0];
      sd += o[S::PF + 2 * q0 + 1] + o[S::PF + 2 * K1 + 2 * q0 + 1];
    }
    g_u[t] = su;
    g_du[t] = sd;
    g_a[t] = sa;
  } else if (t < nx * K1 + nx + 1) {
    const int f = t - nx * K1;
    double s = 0.0;
    for (int ip = 0; ip < np; ++ip) {
      if (f < nx) s += slots[(size_t)(ip * nx + f) * S::SIZE + S::XF + 0];
      if (f >= 1) s += slots[(size_t)(ip * nx + f - 1) * S::SIZE + S::XF + 1];
    }
    g_uf[f] = s;
  }
}

template <int K, int LMAX>
void launch_fg_t(const KernelArgs& a, const double* mu, const double* fwd, double cdt, double* slots,
                 const unsigned char* support, const int* p1_blocks, int np1, double* grad_nu, hipStream_t s) {
  const int blocks = field_grad_tiles(a.mesh.ncells, LMAX);
  if (!p1_blocks) np1 = blocks;
  if (blocks + np1 == 0) return;
  hipLaunchKernelGGL((fgrad_kernel<K, LMAX>), dim3(blocks + np1), dim3(kFgThreads), 0, s, a, mu, fwd, cdt, slots,
                     support, p1_blocks, blocks, np1, grad_nu);
}

template <int K>
FieldGradLauncher pick_fg(int lmax) {
  switch (lmax) {
    case 1: return &launch_fg_t<K, 1>;
    case 2: return &launch_fg_t<K, 2>;
    case 3: return &launch_fg_t<K, 3>;
    case 4: return &launch_fg_t<K, 4>;
    case 5: return &launch_fg_t<K, 5>;
    case 6: return &launch_fg_t<K, 6>;
    case 7: return &launch_fg_t<K, 7>;
    default: return nullptr;
  }
}

template <int K>
void launch_fgr_t(const MeshArgs& m, const double* slots, double* g_u, double* g_du, double* g_a, double* g_uf,
                  hipStream_t s) {
  const int n = m.n[0] * (K + 1) + m.n[0] + 1;
  hipLaunchKernelGGL((fgrad_reduce_kernel<K>), dim3((n + 127) / 128), dim3(128), 0, s, m, slots, g_u, g_du, g_a,
                     g_uf);
}

}  // namespace

FieldGradLauncher find_field_grad_launcher(int k, int lmax) {
  if (k == 1) return pick_fg<1>(lmax);
  if (k == 2) return pick_fg<2>(lmax);
  return nullptr;
}

FieldGradReduce find_field_grad_reduce(int k) {
  if (k == 1) return &launch_fgr_t<1>;
  if (k == 2) return &launch_fgr_t<2>;
  return nullptr;
}

int field_grad_slots_per_cell(int k) { return k == 1 ? GSlots<1>::SIZE : GSlots<2>::SIZE; }

int field_grad_tile_cells(int lmax) {
  const int n = (lmax + 1) * (lmax + 1);
  return kFgThreads / n > 0 ? kFgThreads / n : 1;
}

int field_grad_tiles(int ncells, int lmax) {
  const int c = field_grad_tile_cells(lmax);
  return (ncells + c - 1) / c;
}

}  // namespace vfp
