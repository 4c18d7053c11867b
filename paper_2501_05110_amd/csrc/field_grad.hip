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
//     (H(l_k) where l_k = l_l); where B is definite, dB_+ = dB or 0.
// On a face from T1 (below) to T2 (above) the pairing is  int_F (mu_2 - mu_1).J
// (the trace of a cell outside the mesh counts as zero).
//
// Each cell accumulates into its own slots (no atomics): its volume points,
// its lower x and ln p faces, and its upper faces where they are the
// (non-periodic) end of the mesh.  fgrad_reduce sums the slots per x point.
#include "basis.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kFgThreads = 64;

template <int K>
struct GSlots {
  static constexpr int K1 = K + 1;
  static constexpr int NB = K1 * K1;
  static constexpr int VOL = 0;            // [NB][3]: U, U', a at each volume point
  static constexpr int XF = 3 * NB;        // [2]: lower, upper x face
  static constexpr int PF = XF + 2;        // [2 sides][K1 x points][2]: a, U'
  static constexpr int SIZE = PF + 4 * K1;
};

// Heaviside with H(0) = 1/2
__device__ __forceinline__ double heav(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5); }

template <int K, int LMAX>
__global__ __launch_bounds__(kFgThreads) void fgrad_kernel(KernelArgs A, const double* __restrict__ mu,
                                                           const double* __restrict__ fwd, double cdt,
                                                           double* __restrict__ slots) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = K1 * K1;
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  constexpr int NR = 3 * NB;                // reduction rows per cell
  using CB = CBasis<K>;
  using S = GSlots<K>;
  // per cell: f, mu, d_x mu, d_p mu at the Gauss points, then partial sums
  __shared__ double lds[CPB * (4 * NB + NR) * N];

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
  double* L = lds + (in_grp ? cl : 0) * (4 * NB + NR) * N;
  double* Fq = L;
  double* Mq = L + NB * N;
  double* Mx = L + 2 * NB * N;
  double* Mp = L + 3 * NB * N;
  double* Rd = L + 4 * NB * N;

  const double* xr = F.xrec + (size_t)ix * kRec;
  const double* pr = F.prec + (size_t)ip * kRec;
  const double s2hx = xr[11], s2hp = pr[14];
  const double jac = 1.0 / (s2hx * s2hp);
  const double t_adv = F.t_adv, t_mom = F.t_mom;
  const double gw[3] = {K == 1 ? 1.0 : 5.0 / 9.0, K == 1 ? 1.0 : 8.0 / 9.0, 5.0 / 9.0};

  const size_t cbase = (size_t)cell * NB * N + r;
  double w[NB], m[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    w[b] = act ? fwd[cbase + (size_t)b * N] : 0.0;
    m[b] = act ? mu[cbase + (size_t)b * N] : 0.0;
  }
  const int axc0 = T.ax_col[r], axc1 = T.ax_col[N + r];
  const double axv0 = T.ax_val[r], axv1 = T.ax_val[N + r];
  const int axxc0 = T.axx_col[r], axxc1 = T.axx_col[N + r];
  const double axxv0 = T.axx_val[r], axxv1 = T.axx_val[N + r], axxv2 = T.axx_val[2 * N + r];
  const double g1v0 = T.g1_val[r], g1v1 = T.g1_val[N + r];
  const double g2v0 = T.g2_val[r], g2v1 = T.g2_val[N + r], g2v2 = T.g2_val[2 * N + r];
  double* out = slots + (size_t)cell * S::SIZE;

  // reduce Rd[o][0..N) over the cell's lanes into out[base + o] (scaled)
  auto reduce_rows = [&](int nrows, int base, const double* scale) {
    __syncthreads();
    if (act)
      for (int o = r; o < nrows; o += N) {
        double sum = 0.0;
        for (int j = 0; j < N; ++j) sum += Rd[o * N + j];
        out[base + o] += cdt * scale[o] * sum;
      }
    __syncthreads();
  };

  // ---- volume ------------------------------------------------------------
#pragma unroll
  for (int q1 = 0; q1 < K1; ++q1)
#pragma unroll
    for (int q0 = 0; q0 < K1; ++q0) {
      double f = 0.0, a = 0.0, dx = 0.0, dp = 0.0;
#pragma unroll
      for (int j1 = 0; j1 < K1; ++j1)
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) {
          const int b = j0 + K1 * j1;
          f = fma(CB::phi[q0][j0] * CB::phi[q1][j1], w[b], f);
          a = fma(CB::phi[q0][j0] * CB::phi[q1][j1], m[b], a);
          dx = fma(CB::dphi[q0][j0] * CB::phi[q1][j1], m[b], dx);
          dp = fma(CB::phi[q0][j0] * CB::dphi[q1][j1], m[b], dp);
        }
      const int q = q0 + K1 * q1;
      if (in_grp) {
        Fq[q * N + r] = f;
        Mq[q * N + r] = a;
        Mx[q * N + r] = dx;
        Mp[q * N + r] = dp;
      }
    }
  __syncthreads();
  double vscale[NR];
#pragma unroll
  for (int q1 = 0; q1 < K1; ++q1)
#pragma unroll
    for (int q0 = 0; q0 < K1; ++q0) {
      const int q = q0 + K1 * q1;
      const double* P = Fq + q * N;
      const double f = P[r];
      const double Axf = fma(axv0, P[axc0], axv1 * P[axc1]);
      const double A2f = fma(axxv0, P[axxc0], fma(axxv1, f, axxv2 * P[axxc1]));
      const double G1f = fma(g1v0, P[axc0], g1v1 * P[axc1]);
      const double G2f = fma(g2v0, P[axxc0], fma(g2v1, f, g2v2 * P[axxc1]));
      const double iV = pr[3 + q1], pid = pr[6 + q1];
      const double mq = Mq[q * N + r], mx = Mx[q * N + r], mp = Mp[q * N + r];
      const double pu = s2hx * t_adv * mx * f;
      const double pdu = -mq * (t_mom * G2f - t_adv * f) - s2hp * t_mom * mp * A2f;
      const double pa = -mq * t_mom * (iV * G1f - pid * Axf) - s2hp * t_mom * t_mom * mp * iV * Axf;
      if (in_grp) {
        Rd[(3 * q + 0) * N + r] = pu;
        Rd[(3 * q + 1) * N + r] = pdu;
        Rd[(3 * q + 2) * N + r] = pa;
      }
      const double wq = gw[q0] * gw[q1] * jac;
      vscale[3 * q] = vscale[3 * q + 1] = vscale[3 * q + 2] = wq;
    }
  reduce_rows(NR, S::VOL, vscale);

  // ---- x faces -------------------------------------------------------------
  int mem[LMAX + 1];
  double wcol[LMAX + 1], wrow[LMAX + 1];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    mem[i] = T.blk_mem[i * N + r];
    wcol[i] = T.w_col[i * N + r];
    wrow[i] = T.w_row[i * N + r];
  }
  const double lam = T.lam[r];
  for (int side = 0; side < 2; ++side) {
    const int bc = side ? M.bc_hi[0] : M.bc_lo[0];
    const bool valid = act && (side == 0 || (ix == nx - 1 && bc != 0));
    int ni = side ? ix + 1 : ix - 1;
    const bool inside = ni >= 0 && ni < nx;
    const bool use_n = inside || bc == 0;
    ni = (ni + nx) % nx;
    const size_t nb0 = (size_t)(cell + (ni - ix)) * NB * N + r;
    const int jo = side ? K : 0, jn = side ? 0 : K;   // own / neighbour node column
    double pr_acc = 0.0;
    for (int q1 = 0; q1 < K1; ++q1) {
      double fo = 0.0, fn = 0.0, mo = 0.0, mn = 0.0;
#pragma unroll
      for (int j1 = 0; j1 < K1; ++j1) {
        const double ph = CB::phi[q1][j1];
        fo = fma(ph, w[jo + K1 * j1], fo);
        mo = fma(ph, m[jo + K1 * j1], mo);
        const double vf = (act && use_n) ? fwd[nb0 + (size_t)(jn + K1 * j1) * N] : 0.0;
        const double vm = (act && use_n) ? mu[nb0 + (size_t)(jn + K1 * j1) * N] : 0.0;
        fn = fma(ph, vf, fn);
        mn = fma(ph, vm, mn);
      }
      if (!use_n) fn = (bc == 1) ? 0.0 : fo;   // exterior state of zero inflow / continuous
      const double f1 = side ? fo : fn, f2 = side ? fn : fo;
      const double m1 = side ? mo : mn, m2 = side ? mn : mo;
      if (in_grp) {
        Fq[r] = f1;
        Fq[N + r] = f2;
      }
      __syncthreads();
      double c1 = 0.0, c2 = 0.0;
#pragma unroll
      for (int j = 0; j <= LMAX; ++j) {
        c1 = fma(wcol[j], Fq[mem[j]], c1);
        c2 = fma(wcol[j], Fq[N + mem[j]], c2);
      }
      const double V = pr[0 + q1];
      const double sp = xr[9 + side] + t_adv * lam * V;
      const double h = heav(sp);
      const double d = t_adv * (h * c1 + (1.0 - h) * c2);
      __syncthreads();
      if (in_grp) Fq[r] = d;
      __syncthreads();
      double dj = 0.0;
#pragma unroll
      for (int i = 0; i <= LMAX; ++i) dj = fma(wrow[i], Fq[mem[i]], dj);
      __syncthreads();
      pr_acc += gw[q1] * (m2 - m1) * dj;
    }
    if (in_grp) Rd[r] = valid ? pr_acc : 0.0;
    const double one[1] = {1.0 / s2hp};
    __syncthreads();
    if (valid && r == 0) {
      double sum = 0.0;
      for (int j = 0; j < N; ++j) sum += Rd[j];
      out[S::XF + side] += cdt * one[0] * sum;
    }
    __syncthreads();
  }

  // ---- ln p faces --------------------------------------------------------
  // block position of this row: l - m, and the block size
  int lrow = 0;
  while ((lrow + 1) * (lrow + 1) <= r) ++lrow;
  const int mrow = r - lrow * (lrow + 1) < 0 ? lrow * (lrow + 1) - r : r - lrow * (lrow + 1);
  const int pos = lrow - mrow, bsz = LMAX - mrow + 1;
  size_t eoff = 0;
  for (int mm = 0; mm < mrow; ++mm) eoff += (size_t)(LMAX - mm + 1) * (LMAX - mm + 2);
  const size_t eigsz = [] {
    size_t e = 0;
    for (int mm = 0; mm <= LMAX; ++mm) e += (size_t)(LMAX - mm + 1) * (LMAX - mm + 2);
    return e;
  }();
  for (int side = 0; side < 2; ++side) {
    const int bc = side ? M.bc_hi[1] : M.bc_lo[1];
    const bool valid = act && (side == 0 || (ip == np - 1 && bc != 0));
    int ni = side ? ip + 1 : ip - 1;
    const bool inside = ni >= 0 && ni < np;
    const bool use_n = inside || bc == 0;
    ni = (ni + np) % np;
    const size_t nb0 = (size_t)(cell + (ni - ip) * nx) * NB * N + r;
    const int jo = side ? K : 0, jn = side ? 0 : K;
    const int pf = ip + side;
    const double tmv = pr[12 + side];                   // t_mom / V at this face
    double acc_a[K1], acc_u[K1];
    for (int q0 = 0; q0 < K1; ++q0) {
      double fo = 0.0, fn = 0.0, mo = 0.0, mn = 0.0;
#pragma unroll
      for (int j0 = 0; j0 < K1; ++j0) {
        const double ph = CB::phi[q0][j0];
        fo = fma(ph, w[j0 + K1 * jo], fo);
        mo = fma(ph, m[j0 + K1 * jo], mo);
        const double vf = (act && use_n) ? fwd[nb0 + (size_t)(j0 + K1 * jn) * N] : 0.0;
        const double vm = (act && use_n) ? mu[nb0 + (size_t)(j0 + K1 * jn) * N] : 0.0;
        fn = fma(ph, vf, fn);
        mn = fma(ph, vm, mn);
      }
      if (!use_n) fn = (bc == 1) ? 0.0 : fo;
      const double f1 = side ? fo : fn, f2 = side ? fn : fo;
      const double m1 = side ? mo : mn, m2 = side ? mn : mo;
      if (in_grp) {
        Fq[r] = f1;
        Fq[N + r] = f2;
        Fq[2 * N + r] = f1 - f2;
      }
      __syncthreads();
      const int code = F.pf_code[(size_t)pf * (nx * K1) + ix * K1 + q0];
      const double* Pu = (code == -1) ? Fq : Fq + N;     // the state dB multiplies
      const double ax_u = fma(axv0, Pu[axc0], axv1 * Pu[axc1]);
      const double axx_u = fma(axxv0, Pu[axxc0], fma(axxv1, Pu[r], axxv2 * Pu[axxc1]));
      double ja = -t_mom * tmv * ax_u, ju = -t_mom * axx_u;
      if (code >= 0) {
        // Daleckii-Krein: row r of Q (Gamma o Q^T dB Q) Q^T (f1 - f2) for dB =
        // A^x and (A^xA^x)_t restricted to the (m, s) block of row r
        const double* eg = F.pf_eig + (size_t)code * eigsz + eoff;
        const double* lamb = eg;                         // [bsz]
        const double* Q = eg + bsz;                      // [bsz][bsz], column e = eigenvector e
        double y[LMAX + 1], zA[LMAX + 1], zX[LMAX + 1];
        for (int e = 0; e < bsz; ++e) {
          double acc = 0.0;
          for (int i = 0; i < bsz; ++i) acc = fma(Q[i * bsz + e], Fq[2 * N + mem[i]], acc);
          y[e] = acc;
        }
        for (int k = 0; k < bsz; ++k) zA[k] = zX[k] = 0.0;
        for (int l = 0; l < bsz; ++l) {
          // v = dB q_l for both dB, in block coordinates
          for (int i = 0; i < bsz; ++i) {
            const int ri = mem[i];
            const int c0 = T.ax_col[ri], c1 = T.ax_col[N + ri];
            const double a0 = T.ax_val[ri], a1v = T.ax_val[N + ri];
            const int x0 = T.axx_col[ri], x1 = T.axx_col[N + ri];
            const double b0 = T.axx_val[ri], b1 = T.axx_val[N + ri], b2 = T.axx_val[2 * N + ri];
            // block positions of the column entries (l +- 1, l +- 2 in the block)
            double vA = 0.0, vX = b1 * Q[i * bsz + l];
            if (c0 != ri && i + 1 < bsz) vA = fma(a0, Q[(i + 1) * bsz + l], vA);
            if (c1 != ri && i - 1 >= 0) vA = fma(a1v, Q[(i - 1) * bsz + l], vA);
            if (x0 != ri && i + 2 < bsz) vX = fma(b0, Q[(i + 2) * bsz + l], vX);
            if (x1 != ri && i - 2 >= 0) vX = fma(b2, Q[(i - 2) * bsz + l], vX);
            // D_kl = q_k . v for every k: accumulate Gamma_kl D_kl y_l into z_k
            for (int k = 0; k < bsz; ++k) {
              const double lk = lamb[k], ll = lamb[l];
              const double dl = lk - ll;
              const double gam = (fabs(dl) > 1e-14 * (fabs(lk) + fabs(ll)))
                                     ? (fmax(lk, 0.0) - fmax(ll, 0.0)) / dl
                                     : heav(lk);
              zA[k] = fma(gam * Q[i * bsz + k] * vA, y[l], zA[k]);
              zX[k] = fma(gam * Q[i * bsz + k] * vX, y[l], zX[k]);
            }
          }
        }
        double dkA = 0.0, dkX = 0.0;
        for (int k = 0; k < bsz; ++k) {
          dkA = fma(Q[pos * bsz + k], zA[k], dkA);
          dkX = fma(Q[pos * bsz + k], zX[k], dkX);
        }
        ja = fma(-t_mom * tmv, dkA, ja);
        ju = fma(-t_mom, dkX, ju);
      }
      acc_a[q0] = gw[q0] * (m2 - m1) * ja;
      acc_u[q0] = gw[q0] * (m2 - m1) * ju;
      __syncthreads();
    }
    if (in_grp)
      for (int q0 = 0; q0 < K1; ++q0) {
        Rd[(2 * q0 + 0) * N + r] = valid ? acc_a[q0] : 0.0;
        Rd[(2 * q0 + 1) * N + r] = valid ? acc_u[q0] : 0.0;
      }
    __syncthreads();
    if (valid)
      for (int o = r; o < 2 * K1; o += N) {
        double sum = 0.0;
        for (int j = 0; j < N; ++j) sum += Rd[o * N + j];
        out[S::PF + side * 2 * K1 + o] += cdt * sum / s2hx;
      }
    __syncthreads();
  }
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
      for (int q1 = 0; q1 < K1; ++q1) {
        const int q = q0 + K1 * q1;
        su += o[S::VOL + 3 * q + 0];
        sd += o[S::VOL + 3 * q + 1];
        sa += o[S::VOL + 3 * q + 2];
      }
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
                 hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  const int blocks = (a.mesh.ncells + CPB - 1) / CPB;
  hipLaunchKernelGGL((fgrad_kernel<K, LMAX>), dim3(blocks), dim3(kFgThreads), 0, s, a, mu, fwd, cdt, slots);
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

}  // namespace vfp
