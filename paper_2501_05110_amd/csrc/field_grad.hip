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
// Each cell accumulates into its own slots (no atomics): its x Gauss points
// (summed over its p points), its lower x and ln p faces, and its upper faces
// where they are the (non-periodic) end of the mesh.  All global loads are
// issued first; the lanes of a cell exchange forward values through LDS for
// the l-coupling and reduce once at the end.  fgrad_reduce sums the slots per
// x point.
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

template <int K, int LMAX>
__global__ __launch_bounds__(kFgThreads) void fgrad_kernel(KernelArgs A, const double* __restrict__ mu,
                                                           const double* __restrict__ fwd, double cdt,
                                                           double* __restrict__ slots,
                                                           const unsigned char* __restrict__ support) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  constexpr int NB = K1 * K1;
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  constexpr int XRW = 4 * K1;               // exchange rows per cell
  using CB = CBasis<K>;
  using S = GSlots<K>;
  constexpr int NS = S::SIZE;               // partial-sum rows per cell
  __shared__ double lds[CPB * (XRW + NS) * N];

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
  double* X = lds + (in_grp ? cl : 0) * (XRW + NS) * N;
  double* Rd = X + XRW * N;

  // ---- every global load first ---------------------------------------------
  const size_t cbase = (size_t)cell * NB * N + r;
  double w[NB], m[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    w[b] = fwd[cbase + (size_t)b * N];
    m[b] = mu[cbase + (size_t)b * N];
  }
  const double* xr = F.xrec + (size_t)ix * kRec;
  const double* pr = F.prec + (size_t)ip * kRec;
  const double s2hx = xr[11], s2hp = pr[14];
  const double jac = 1.0 / (s2hx * s2hp);
  const double t_adv = F.t_adv, t_mom = F.t_mom;
  const double gw[3] = {K == 1 ? 1.0 : 5.0 / 9.0, K == 1 ? 1.0 : 8.0 / 9.0, 5.0 / 9.0};
  const int axc0 = T.ax_col[r], axc1 = T.ax_col[N + r];
  const double axv0 = T.ax_val[r], axv1 = T.ax_val[N + r];
  const int axxc0 = T.axx_col[r], axxc1 = T.axx_col[N + r];
  const double axxv0 = T.axx_val[r], axxv1 = T.axx_val[N + r], axxv2 = T.axx_val[2 * N + r];
  const double g1v0 = T.g1_val[r], g1v1 = T.g1_val[N + r];
  const double g2v0 = T.g2_val[r], g2v1 = T.g2_val[N + r], g2v2 = T.g2_val[2 * N + r];
  int mem[LMAX + 1];
  double wcol[LMAX + 1], wrow[LMAX + 1];
#pragma unroll
  for (int i = 0; i <= LMAX; ++i) {
    mem[i] = T.blk_mem[i * N + r];
    wcol[i] = T.w_col[i * N + r];
    wrow[i] = T.w_row[i * N + r];
  }
  const double lam = T.lam[r];
  int pcode[2][K1];
#pragma unroll
  for (int side = 0; side < 2; ++side)
#pragma unroll
    for (int q0 = 0; q0 < K1; ++q0) pcode[side][q0] = F.pf_code[(size_t)(ip + side) * (nx * K1) + ix * K1 + q0];

  // this lane's share of every slot goes to row i of Rd; the volume rows are
  // accumulated in registers first
  double part[3 * K1];
#pragma unroll
  for (int i = 0; i < 3 * K1; ++i) part[i] = 0.0;

  // The U' and dU/dt sensitivities (volume and ln p faces) are formed for
  // the x cells the caller's support marks (all without one); the decision
  // is uniform over the wavefront (the workgroup), whose LDS exchanges all
  // lanes then take alike.  dJ/dU (volume and x faces) is formed everywhere.
  bool full = support == nullptr;
  if (!full) {
    for (int c2 = 0; c2 < CPB; ++c2) {
      const int cc = blockIdx.x * CPB + c2;
      if (cc < M.ncells) full |= support[cc % nx] != 0;
    }
  }
  if (!full) {
    // dJ/dU at the x Gauss points: t_adv (2/h_x) (d_x mu) f, no exchange
#pragma unroll
    for (int q1 = 0; q1 < K1; ++q1) {
      double wy[K1], my[K1];
#pragma unroll
      for (int j0 = 0; j0 < K1; ++j0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int j1 = 0; j1 < K1; ++j1) {
          a = fma(CB::phi[q1][j1], w[j0 + K1 * j1], a);
          b = fma(CB::phi[q1][j1], m[j0 + K1 * j1], b);
        }
        wy[j0] = a;
        my[j0] = b;
      }
#pragma unroll
      for (int q0 = 0; q0 < K1; ++q0) {
        double f = 0.0, mx = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < K1; ++j0) {
          f = fma(CB::phi[q0][j0], wy[j0], f);
          mx = fma(CB::dphi[q0][j0], my[j0], mx);
        }
        const double wq = gw[q0] * gw[q1] * jac;
        part[S::VOL + 3 * q0 + 0] += wq * (s2hx * t_adv * mx * f);
      }
    }
  } else {
  // ---- volume, one row of Gauss points (fixed q1) at a time: interpolate
  // along ln p first (K1 values per row), then along x
#pragma unroll
  for (int q1 = 0; q1 < K1; ++q1) {
    double wy[K1], my[K1], mdy[K1];
#pragma unroll
    for (int j0 = 0; j0 < K1; ++j0) {
      double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
      for (int j1 = 0; j1 < K1; ++j1) {
        a = fma(CB::phi[q1][j1], w[j0 + K1 * j1], a);
        b = fma(CB::phi[q1][j1], m[j0 + K1 * j1], b);
        c = fma(CB::dphi[q1][j1], m[j0 + K1 * j1], c);
      }
      wy[j0] = a;
      my[j0] = b;
      mdy[j0] = c;
    }
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
      double mq = 0.0, mx = 0.0, mp = 0.0;
#pragma unroll
      for (int j0 = 0; j0 < K1; ++j0) {
        mq = fma(CB::phi[q0][j0], my[j0], mq);
        mx = fma(CB::dphi[q0][j0], my[j0], mx);
        mp = fma(CB::phi[q0][j0], mdy[j0], mp);
      }
      const double* P = X + q0 * N;
      const double f = fq[q0];
      const double Axf = fma(axv0, P[axc0], axv1 * P[axc1]);
      const double A2f = fma(axxv0, P[axxc0], fma(axxv1, f, axxv2 * P[axxc1]));
      const double G1f = fma(g1v0, P[axc0], g1v1 * P[axc1]);
      const double G2f = fma(g2v0, P[axxc0], fma(g2v1, f, g2v2 * P[axxc1]));
      const double wq = gw[q0] * gw[q1] * jac;
      part[S::VOL + 3 * q0 + 0] += wq * (s2hx * t_adv * mx * f);
      part[S::VOL + 3 * q0 + 1] += wq * (-mq * (t_mom * G2f - t_adv * f) - s2hp * t_mom * mp * A2f);
      part[S::VOL + 3 * q0 + 2] +=
          wq * (-mq * t_mom * (iV * G1f - pid * Axf) - s2hp * t_mom * t_mom * mp * iV * Axf);
    }
    wave_sync();
  }

  }

  if (in_grp)
#pragma unroll
    for (int i = 0; i < 3 * K1; ++i) Rd[(S::VOL + i) * N + r] = part[i];

  // neighbour traces [axis][side][j]: forward and adjoint values
  // neighbour traces [axis][side][j]: forward and adjoint values
  double nf[2][2][K1], nm[2][2][K1];
  bool use_n[2][2];
#pragma unroll
  for (int ax = 0; ax < 2; ++ax)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int ia = ax ? ip : ix, na = ax ? np : nx, st = ax ? nx : 1;
      int ni = side ? ia + 1 : ia - 1;
      const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
      use_n[ax][side] = (ni >= 0 && ni < na) || bc == 0;
      ni = (ni + na) % na;
      const size_t nb0 = (size_t)(cell + (ni - ia) * st) * NB * N + r;
      const int jn = side ? 0 : K;
#pragma unroll
      for (int j = 0; j < K1; ++j) {
        const int node = ax ? (j + K1 * jn) : (jn + K1 * j);
        nf[ax][side][j] = fwd[nb0 + (size_t)node * N];
        nm[ax][side][j] = mu[nb0 + (size_t)node * N];
      }
    }

  // ---- faces: this cell's lower faces, and its upper faces at the
  // (non-periodic) end of the mesh; on a face from T1 (below) to T2 (above)
  // the pairing is int_F (mu_2 - mu_1) . dJ, with the trace of a cell outside
  // the mesh counted as zero
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    if (ax == 1 && !full) {
      // no U' and dU/dt sensitivities here: the ln p face slots stay zero
      if (in_grp)
#pragma unroll
        for (int i = 0; i < 4 * K1; ++i) Rd[(S::PF + i) * N + r] = 0.0;
      break;
    }
    const int ia = ax ? ip : ix, na = ax ? np : nx;
    // f1, f2 rows of both sides: [side][f1 / f2][q] in X
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double fo = 0.0, fn = 0.0;
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          const double ph = CB::phi[q][j];
          const int node = ax ? (j + K1 * (side ? K : 0)) : ((side ? K : 0) + K1 * j);
          fo = fma(ph, w[node], fo);
          fn = fma(ph, nf[ax][side][j], fn);
        }
        if (!use_n[ax][side]) fn = (bc == 1) ? 0.0 : fo;   // exterior of zero inflow / continuous
        if (in_grp) {
          X[((side * 2 + 0) * K1 + q) * N + r] = side ? fo : fn;   // f1 (lower cell)
          X[((side * 2 + 1) * K1 + q) * N + r] = side ? fn : fo;   // f2 (upper cell)
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int bc = side ? M.bc_hi[ax] : M.bc_lo[ax];
      const bool valid = act && (side == 0 || (ia == na - 1 && bc != 0));
      double dmu[K1];
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double mo = 0.0, mn = 0.0;
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          const double ph = CB::phi[q][j];
          const int node = ax ? (j + K1 * (side ? K : 0)) : ((side ? K : 0) + K1 * j);
          mo = fma(ph, m[node], mo);
          mn = fma(ph, nm[ax][side][j], mn);
        }
        if (!use_n[ax][side]) mn = 0.0;
        dmu[q] = valid ? (side ? mn - mo : mo - mn) : 0.0;   // mu_2 - mu_1
      }
      const double* R1 = X + (side * 2 + 0) * K1 * N;
      const double* R2 = X + (side * 2 + 1) * K1 * N;
      if (ax == 0) {
        // x face: dJ/dU_F = t_adv W (H(m) c1 + (1 - H(m)) c2), c = W^T f
        double d[K1];
#pragma unroll
        for (int q = 0; q < K1; ++q) {
          double c1 = 0.0, c2 = 0.0;
#pragma unroll
          for (int j = 0; j <= LMAX; ++j) {
            c1 = fma(wcol[j], R1[q * N + mem[j]], c1);
            c2 = fma(wcol[j], R2[q * N + mem[j]], c2);
          }
          const double h = heav(xr[9 + side] + t_adv * lam * pr[0 + q]);
          d[q] = t_adv * (h * c1 + (1.0 - h) * c2);
        }
        wave_sync();
        if (in_grp)
#pragma unroll
          for (int q = 0; q < K1; ++q) X[((side * 2 + 0) * K1 + q) * N + r] = d[q];
        wave_sync();
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < K1; ++q) {
          double dj = 0.0;
#pragma unroll
          for (int i = 0; i <= LMAX; ++i) dj = fma(wrow[i], R1[q * N + mem[i]], dj);
          acc = fma(gw[q] * dmu[q], dj, acc);
        }
        if (in_grp) Rd[(S::XF + side) * N + r] = acc / s2hp;
      } else {
        // ln p face: dJ = dB_+ (f1 - f2) + dB f2 (dB f1 where B >= 0)
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
          if (in_grp) {
            Rd[(S::PF + side * 2 * K1 + 2 * q + 0) * N + r] = gw[q] * dmu[q] * ja / s2hx;
            Rd[(S::PF + side * 2 * K1 + 2 * q + 1) * N + r] = gw[q] * dmu[q] * ju / s2hx;
          }
        }
      }
    }
    wave_sync();
  }

  // ---- one reduction over the cell's lanes for every slot --------------------
  wave_sync();
  if (act)
    for (int o = r; o < NS; o += N) {
      double sum = 0.0;
      for (int j = 0; j < N; ++j) sum += Rd[o * N + j];
      slots[(size_t)cell * NS + o] += cdt * sum;
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
                 const unsigned char* support, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int CPB = (kFgThreads / N) > 0 ? kFgThreads / N : 1;
  const int blocks = (a.mesh.ncells + CPB - 1) / CPB;
  hipLaunchKernelGGL((fgrad_kernel<K, LMAX>), dim3(blocks), dim3(kFgThreads), 0, s, a, mu, fwd, cdt, slots,
                     support);
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
