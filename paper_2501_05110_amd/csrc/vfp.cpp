// Host side of the C ABI in include/vfp.h: argument checking, set-up of the
// spherical-harmonic tables and field data, and kernel launches.
#include "vfp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "kargs.hpp"
#include "launch.hpp"
#include "shtab.hpp"

using namespace vfp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                            \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) return fail(VFP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Owned device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory (page-locked, so device-to-host copies into it go
// straight over the bus instead of through a staging buffer)
struct HostPin {
  double* p = nullptr;
  ~HostPin() {
    if (p) (void)hipHostFree(p);
  }
};

int upload(DevBuf& b, const void* host, size_t bytes) {
  b.release();
  if (bytes == 0) return VFP_OK;
  if (std::getenv("VFP_FAIL_ALLOC")) return fail(VFP_ENOMEM, "allocation of %zu bytes refused (VFP_FAIL_ALLOC)", bytes);
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(VFP_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  HIP_TRY(hipMemcpy(b.p, host, bytes, hipMemcpyHostToDevice));
  return VFP_OK;
}

template <class T>
int upload_vec(DevBuf& b, const std::vector<T>& v) { return upload(b, v.data(), v.size() * sizeof(T)); }

// Legendre polynomial P_n(x) and its derivative by the three-term recurrence
// (the derivative from P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), |x| < 1).
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int l = 2; l <= n; ++l) {
    const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// q-point Gauss-Legendre rule: the roots of P_q by Newton's method from the
// Chebyshev guesses, weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(q, t, p, dp);
      const double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p, dp;
    legendre(q, t, p, dp);
    x[i] = std::fabs(t) < 1e-15 ? 0.0 : t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// k+1 Gauss-Lobatto nodes: -1, 1 and the roots of P_k' by Newton's method
// (P_k'' = (2 x P_k' - k (k+1) P_k) / (1 - x^2)) from the Chebyshev-Lobatto
// points; for k <= 2 these are the equidistant nodes.
std::vector<double> lobatto_nodes(int k) {
  std::vector<double> x(k + 1);
  x[0] = -1.0;
  x[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double t = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, t, p, dp);
      const double d2 = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      const double dt = dp / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = std::fabs(t) < 1e-15 ? 0.0 : t;
  }
  return x;
}

// 1-D basis data for degree k (Gauss-Lobatto Lagrange basis, (k+1)-point
// Gauss rule) computed in double precision.
Basis1D make_basis(int k) {
  Basis1D B;
  std::memset(&B, 0, sizeof B);
  const int K1 = k + 1;
  const std::vector<double> nodes = lobatto_nodes(k);
  std::vector<double> g, w;
  gauss_rule(K1, g, w);
  auto lag = [&](int j, double x) {
    double v = 1.0;
    for (int m = 0; m < K1; ++m)
      if (m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    return v;
  };
  auto dlag = [&](int j, double x) {
    double d = 0.0;
    for (int m = 0; m < K1; ++m) {
      if (m == j) continue;
      double t = 1.0 / (nodes[j] - nodes[m]);
      for (int i = 0; i < K1; ++i)
        if (i != j && i != m) t *= (x - nodes[i]) / (nodes[j] - nodes[i]);
      d += t;
    }
    return d;
  };
  double M1[kMaxK1][kMaxK1] = {}, Mi[kMaxK1][kMaxK1] = {};
  for (int i = 0; i < K1; ++i)
    for (int j = 0; j < K1; ++j)
      for (int q = 0; q < K1; ++q) M1[i][j] += w[q] * lag(i, g[q]) * lag(j, g[q]);
  // invert the small SPD matrix by Gauss-Jordan
  double a[kMaxK1][2 * kMaxK1] = {};
  for (int i = 0; i < K1; ++i) {
    for (int j = 0; j < K1; ++j) a[i][j] = M1[i][j];
    a[i][K1 + i] = 1.0;
  }
  for (int c = 0; c < K1; ++c) {
    double piv = a[c][c];
    for (int j = 0; j < 2 * K1; ++j) a[c][j] /= piv;
    for (int r = 0; r < K1; ++r)
      if (r != c) {
        double f = a[r][c];
        for (int j = 0; j < 2 * K1; ++j) a[r][j] -= f * a[c][j];
      }
  }
  for (int i = 0; i < K1; ++i)
    for (int j = 0; j < K1; ++j) Mi[i][j] = a[i][K1 + j];
  for (int q = 0; q < K1; ++q)
    for (int j = 0; j < K1; ++j) B.phi[q][j] = lag(j, g[q]);
  for (int i = 0; i < K1; ++i)
    for (int q = 0; q < K1; ++q) {
      double t = 0.0, dt = 0.0;
      for (int j = 0; j < K1; ++j) {
        t += Mi[i][j] * lag(j, g[q]);
        dt += Mi[i][j] * dlag(j, g[q]);
      }
      B.tst[i][q] = t * w[q];
      B.dtst[i][q] = dt * w[q];
    }
  for (int i = 0; i < K1; ++i) {
    B.lift[0][i] = Mi[i][0];
    B.lift[1][i] = Mi[i][k];
  }
  for (int q = 0; q < K1; ++q)
    for (int j = 0; j < K1; ++j) B.dphi[q][j] = dlag(j, g[q]);
  for (int i = 0; i < K1; ++i)
    for (int j = 0; j < K1; ++j) {
      double acc = 0.0;
      for (int q = 0; q < K1; ++q) acc += B.dtst[i][q] * B.phi[q][j];
      B.dvol[i][j] = acc;
    }
  for (int i = 0; i < K1; ++i)
    for (int j = 0; j < K1; ++j) {
      B.mass[i][j] = M1[i][j];
      B.imass[i][j] = Mi[i][j];
    }
  return B;
}

std::vector<double> gauss_points(int k) {
  std::vector<double> g, w;
  gauss_rule(k + 1, g, w);
  return g;
}

bool g_basis_ready[64] = {};

}  // namespace

struct vfp_ctx {
  int lmax = 0, k = 0, naxes = 0, n = 0, nb = 0, K1 = 0;
  int axes[3] = {0, 0, 0};
  unsigned terms = 0;
  double mass = 1.0, charge = 1.0;
  bool mom = false;
  bool linp = false;        // the momentum axis is p itself (else ln p)
  int nspace = 0;
  int device = -1;
  ShMatrices S;

  bool mesh_set = false;
  int ncell[3] = {1, 1, 1};
  int ncells = 0;
  std::vector<double> nodes[3];
  int bc_lo[3] = {0, 0, 0}, bc_hi[3] = {0, 0, 0};
  double p_fixed = std::numeric_limits<double>::quiet_NaN();

  bool planar = false;
  double U[3] = {0, 0, 0};
  std::vector<double> u_vol, du_vol, a_vol, u_face;
  double B[3] = {0, 0, 0};
  bool have_Bpts = false;
  double nu0 = 0.0;
  bool have_nu_cell = false;
  bool have_nu_pts = false;  // nu at the volume points (vfp_set_scattering_points)
  bool have_src = false;
  bool pflow = false;        // U at the points (vfp_set_flow_points)
  double pflow_umax[3] = {0, 0, 0};   // max |U^a| over the volume and face points

  // device data
  DevBuf d_s2h[3], d_u_vol, d_du_vol, d_a_vol, d_u_face;
  DevBuf d_V_vol, d_iV_vol, d_idiv_vol, d_ig_vol, d_iV_face, d_ca_vol, d_cu_vol, d_cu_face;
  DevBuf d_pf_code, d_pf_coded, d_pf_tab, d_pf_dtab, d_Bpts, d_nu, d_src;
  DevBuf d_itab, d_dtab, d_xrec, d_prec, d_prec2;
  DevBuf d_u_pts, d_uf_pts[3], d_nu_pts;
  DevBuf d_fg_support;      // x cells whose U' and dU/dt sensitivities are formed (vfp_field_grad_support)
  DevBuf d_fg_blocks;       // the field-gradient tiles holding a support cell
  int fg_nblocks = 0;
  DevBuf d_flag;            // one int: the finiteness check of vfp_advance (VFP_CHECK_FINITE)
  RowTables tab{};
  FieldArgs fld{};
  MeshArgs meshargs{};
  StageLauncher launcher = nullptr;
  StageLauncher adj_launcher = nullptr;
  bool adj_shock = false;   // adj_launcher is the (x, ln p) kernel (AdjArgs::add_in available)
  MassLauncher mass_launcher = nullptr;
  HostPin h_kry;            // 3 kKryMaxVectors doubles: the Theta-method's per-iteration read-backs
  double beta_pmax = 0.0;   // spectral-radius bound of beta^{ln p} over p faces
  double vmax = 0.0;
  double lam_max = 0.0;     // largest eigenvalue of A^x
  size_t o_rot[2] = {0, 0};
  bool force_general = false;
  bool shock = false;       // the (x, ln p) kernels are in use
  int tile_map = 0;         // XCD-range tile order for the (x, ln p) kernels (VFP_TILE_MAP=1)
  int shape = 0;            // workgroup shape slot of the forward (x, ln p) kernel (vfp_autotune)
  ResidentLauncher resident = nullptr;   // whole-run single-workgroup stepping (small runs on one axis)
  uint64_t gen = 0;         // bumped by every set-up call; a batch bound to older data refuses to run
  bool pf_dk = false;       // the p-face derivative tables (field gradients) are kept
};

namespace {

double momentum_V(const vfp_ctx* c, double p) {
  double g = std::sqrt(1.0 + (p / c->mass) * (p / c->mass));
  return p / (g * c->mass);
}

// -------------------------------------------------------- row tables --

int build_row_tables(vfp_ctx* c) {
  const int n = c->n, L = c->lmax;
  const ShMatrices& S = c->S;
  auto lms = [&](int r, int& l, int& m, int& s) {
    l = (int)std::floor(std::sqrt((double)r) + 1e-9);
    int d = r - l * (l + 1);
    m = std::abs(d);
    s = d > 0 ? 1 : 0;
  };
  std::vector<int> iv;
  std::vector<double> dv;
  // offsets into iv / dv
  auto ialloc = [&](size_t cnt) { size_t o = iv.size(); iv.resize(o + cnt, 0); return o; };
  auto dalloc = [&](size_t cnt) { size_t o = dv.size(); dv.resize(o + cnt, 0.0); return o; };
  size_t o_axc = ialloc(2 * n), o_axv = dalloc(2 * n), o_g1v = dalloc(2 * n);
  size_t o_axxc = ialloc(2 * n), o_axxv = dalloc(3 * n), o_g2v = dalloc(3 * n);
  size_t o_g1t = dalloc(2 * n), o_g2t = dalloc(3 * n);
  size_t o_omc = ialloc(6 * n), o_omv = dalloc(6 * n);
  size_t o_ayzc = ialloc(8 * n), o_ayzv = dalloc(8 * n);
  size_t o_cv = dalloc(n);
  size_t o_mem = ialloc((L + 1) * n), o_wrow = dalloc((L + 1) * n), o_wcol = dalloc((L + 1) * n);
  size_t o_lam = dalloc(n);

  auto check_covered = [&](const Mat& A, int r, std::initializer_list<int> cols, const char* name) -> int {
    for (int j = 0; j < n; ++j) {
      if (A(r, j) == 0.0) continue;
      bool ok = false;
      for (int cc : cols) ok |= (cc == j);
      if (!ok) return fail(VFP_EDEVICE, "internal: %s row %d has an entry outside its stencil", name, r);
    }
    return VFP_OK;
  };

  for (int r = 0; r < n; ++r) {
    int l, m, s;
    lms(r, l, m, s);
    int cp = (l + 1 <= L) ? lms_index(l + 1, m, s) : r;
    int cm = (l - 1 >= m) ? lms_index(l - 1, m, s) : r;
    iv[o_axc + r] = cp;
    iv[o_axc + n + r] = cm;
    dv[o_axv + r] = (cp != r) ? S.A[0](r, cp) : 0.0;
    dv[o_axv + n + r] = (cm != r) ? S.A[0](r, cm) : 0.0;
    dv[o_g1v + r] = (cp != r) ? S.G1(r, cp) : 0.0;
    dv[o_g1v + n + r] = (cm != r) ? S.G1(r, cm) : 0.0;
    if (int e = check_covered(S.A[0], r, {cp, cm}, "A^x")) return e;
    if (int e = check_covered(S.G1, r, {cp, cm}, "G1")) return e;
    int cpp = (l + 2 <= L) ? lms_index(l + 2, m, s) : r;
    int cmm = (l - 2 >= m) ? lms_index(l - 2, m, s) : r;
    iv[o_axxc + r] = cpp;
    iv[o_axxc + n + r] = cmm;
    dv[o_axxv + r] = (cpp != r) ? S.AXX(r, cpp) : 0.0;
    dv[o_axxv + n + r] = S.AXX(r, r);
    dv[o_axxv + 2 * n + r] = (cmm != r) ? S.AXX(r, cmm) : 0.0;
    dv[o_g2v + r] = (cpp != r) ? S.G2(r, cpp) : 0.0;
    dv[o_g2v + n + r] = S.G2(r, r);
    dv[o_g2v + 2 * n + r] = (cmm != r) ? S.G2(r, cmm) : 0.0;
    // transposed values on the same patterns (both are symmetric in l <-> l')
    dv[o_g1t + r] = (cp != r) ? S.G1(cp, r) : 0.0;
    dv[o_g1t + n + r] = (cm != r) ? S.G1(cm, r) : 0.0;
    dv[o_g2t + r] = (cpp != r) ? S.G2(cpp, r) : 0.0;
    dv[o_g2t + n + r] = S.G2(r, r);
    dv[o_g2t + 2 * n + r] = (cmm != r) ? S.G2(cmm, r) : 0.0;
    if (int e = check_covered(S.AXX, r, {cpp, r, cmm}, "(AxAx)_t")) return e;
    if (int e = check_covered(S.G2, r, {cpp, r, cmm}, "G2")) return e;
    for (int cc = 0; cc < 3; ++cc) {
      int slot = 0;
      for (int j = 0; j < n; ++j) {
        if (S.Om[cc](r, j) == 0.0) continue;
        if (slot >= 2) return fail(VFP_EDEVICE, "internal: Omega row %d has more than 2 entries", r);
        iv[o_omc + (cc * 2 + slot) * n + r] = j;
        dv[o_omv + (cc * 2 + slot) * n + r] = S.Om[cc](r, j);
        ++slot;
      }
      for (; slot < 2; ++slot) iv[o_omc + (cc * 2 + slot) * n + r] = r;
    }
    for (int cc = 0; cc < 2; ++cc) {
      int slot = 0;
      for (int j = 0; j < n; ++j) {
        if (S.A[cc + 1](r, j) == 0.0) continue;
        if (slot >= 4) return fail(VFP_EDEVICE, "internal: A^y/A^z row %d has more than 4 entries", r);
        iv[o_ayzc + (cc * 4 + slot) * n + r] = j;
        dv[o_ayzv + (cc * 4 + slot) * n + r] = S.A[cc + 1](r, j);
        ++slot;
      }
      for (; slot < 4; ++slot) iv[o_ayzc + (cc * 4 + slot) * n + r] = r;
    }
    dv[o_cv + r] = S.C[r];
    // (m,s) block of A^x: l' = m..L
    const int bsz = L - m + 1;
    Mat blk(bsz);
    for (int i = 0; i < bsz; ++i)
      for (int j = 0; j < bsz; ++j) blk(i, j) = S.A[0](lms_index(m + i, m, s), lms_index(m + j, m, s));
    std::vector<double> lam;
    Mat W;
    jacobi_eigh(blk, lam, W);
    const int pos = l - m;
    for (int i = 0; i <= L; ++i) {
      if (i < bsz) {
        iv[o_mem + i * n + r] = lms_index(m + i, m, s);
        dv[o_wrow + i * n + r] = W(pos, i);
        dv[o_wcol + i * n + r] = W(i, pos);
      } else {
        iv[o_mem + i * n + r] = r;
      }
    }
    dv[o_lam + r] = lam[pos];
  }

  // point flows: eigenvectors and eigenvalues of A^a per spatial axis (the
  // characteristic speeds U^a + lambda V vary from face point to face point)
  size_t o_wd[3] = {0, 0, 0}, o_lamd[3] = {0, 0, 0};
  if (c->pflow) {
    for (int ax = 0; ax < c->nspace; ++ax) {
      std::vector<double> lam;
      Mat W;
      jacobi_eigh(S.A[c->axes[ax]], lam, W);
      o_wd[ax] = dalloc((size_t)n * n);
      o_lamd[ax] = dalloc(n);
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) dv[o_wd[ax] + (size_t)j * n + k] = W(j, k);
      for (int k = 0; k < n; ++k) dv[o_lamd[ax] + k] = lam[k];
    }
  }

  // uniform-axis face matrices beta^a = U_a + V A^a and |beta^a| (no ln p axis)
  size_t o_fb[3] = {0, 0, 0}, o_fa[3] = {0, 0, 0}, o_fbv[3] = {0, 0, 0}, o_fav[3] = {0, 0, 0};
  int nfb[3] = {0, 0, 0}, nfa[3] = {0, 0, 0};
  const bool adv = c->terms & VFP_TERM_ADVECTION;
  for (int ax = 0; ax < c->nspace; ++ax) {
    if (c->pflow) break;
    if (ax == 0 && c->planar) continue;
    if (c->mom) break;  // with a ln p axis only the profiled x axis is spatial
    const int comp = c->axes[ax];
    const double V = momentum_V(c, c->p_fixed);
    Mat Bm(n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Bm(i, j) = adv ? V * S.A[comp](i, j) : 0.0;
    for (int i = 0; i < n; ++i) Bm(i, i) += adv ? c->U[comp] : 0.0;
    std::vector<double> lam;
    Mat W;
    jacobi_eigh(Bm, lam, W);
    Mat Ab(n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int e = 0; e < n; ++e) acc += W(i, e) * std::fabs(lam[e]) * W(j, e);
        Ab(i, j) = std::fabs(acc) < 1e-14 ? 0.0 : acc;
      }
    auto pack = [&](const Mat& Mx, size_t& oc, size_t& ov, int& cnt) -> int {
      cnt = 0;
      for (int i = 0; i < n; ++i) {
        int nz = 0;
        for (int j = 0; j < n; ++j) nz += (Mx(i, j) != 0.0);
        cnt = std::max(cnt, nz);
      }
      if (cnt > kMaxUniSlots) return fail(VFP_EUNSUPPORTED, "face matrix row has %d > %d entries", cnt, kMaxUniSlots);
      oc = ialloc(size_t(cnt) * n);
      ov = dalloc(size_t(cnt) * n);
      for (int i = 0; i < n; ++i) {
        int slot = 0;
        for (int j = 0; j < n; ++j)
          if (Mx(i, j) != 0.0) {
            iv[oc + size_t(slot) * n + i] = j;
            dv[ov + size_t(slot) * n + i] = Mx(i, j);
            ++slot;
          }
        for (; slot < cnt; ++slot) iv[oc + size_t(slot) * n + i] = i;
      }
      return VFP_OK;
    };
    if (int e = pack(Bm, o_fb[ax], o_fbv[ax], nfb[ax])) return e;
    if (int e = pack(Ab, o_fa[ax], o_fav[ax], nfa[ax])) return e;
  }

  // B . Omega rows for a uniform B (the kernel multiplies by q/(gamma m))
  int nrot = 0;
  {
    Mat RB(n);
    for (int cc = 0; cc < 3; ++cc)
      for (size_t i = 0; i < RB.a.size(); ++i) RB.a[i] += c->B[cc] * S.Om[cc].a[i];
    for (int i = 0; i < n; ++i) {
      int nz = 0;
      for (int j = 0; j < n; ++j) nz += (RB(i, j) != 0.0);
      nrot = std::max(nrot, nz);
    }
    if (nrot > 5) return fail(VFP_EDEVICE, "internal: B.Omega row with %d entries", nrot);
    nrot = (nrot <= 1) ? 1 : 5;
    size_t oc = ialloc(size_t(nrot) * n), ov = dalloc(size_t(nrot) * n);
    for (int i = 0; i < n; ++i) {
      int slot = 0;
      for (int j = 0; j < n; ++j)
        if (RB(i, j) != 0.0) {
          iv[oc + size_t(slot) * n + i] = j;
          dv[ov + size_t(slot) * n + i] = RB(i, j);
          ++slot;
        }
      for (; slot < nrot; ++slot) iv[oc + size_t(slot) * n + i] = i;
    }
    c->o_rot[0] = oc;
    c->o_rot[1] = ov;
  }
  if (int e = upload_vec(c->d_itab, iv)) return e;
  if (int e = upload_vec(c->d_dtab, dv)) return e;
  const int* ib = c->d_itab.as<int>();
  const double* db = c->d_dtab.as<double>();
  RowTables& T = c->tab;
  T = RowTables{};
  T.ax_col = ib + o_axc;
  T.ax_val = db + o_axv;
  T.g1_val = db + o_g1v;
  T.axx_col = ib + o_axxc;
  T.axx_val = db + o_axxv;
  T.g2_val = db + o_g2v;
  T.g1t_val = db + o_g1t;
  T.g2t_val = db + o_g2t;
  T.om_col = ib + o_omc;
  T.om_val = db + o_omv;
  T.ayz_col = ib + o_ayzc;
  T.ayz_val = db + o_ayzv;
  T.c_val = db + o_cv;
  T.blk_mem = ib + o_mem;
  T.w_row = db + o_wrow;
  T.w_col = db + o_wcol;
  T.lam = db + o_lam;
  T.rot_col = ib + c->o_rot[0];
  T.rot_val = db + c->o_rot[1];
  T.nrot = nrot;
  for (int ax = 0; ax < 3; ++ax) {
    T.wd[ax] = (c->pflow && ax < c->nspace) ? db + o_wd[ax] : nullptr;
    T.lamd[ax] = (c->pflow && ax < c->nspace) ? db + o_lamd[ax] : nullptr;
    T.nfb[ax] = nfb[ax];
    T.nfa[ax] = nfa[ax];
    T.fb_col[ax] = nfb[ax] ? ib + o_fb[ax] : nullptr;
    T.fb_val[ax] = nfb[ax] ? db + o_fbv[ax] : nullptr;
    T.fa_col[ax] = nfa[ax] ? ib + o_fa[ax] : nullptr;
    T.fa_val[ax] = nfa[ax] ? db + o_fav[ax] : nullptr;
  }
  return VFP_OK;
}

// ------------------------------------------------- momentum-axis data --

int build_momentum_data(vfp_ctx* c) {
  if (!c->mom || !c->mesh_set) return VFP_OK;
  const int pa = c->naxes - 1, K1 = c->K1;
  const int np = c->ncell[pa];
  const std::vector<double>& nd = c->nodes[pa];
  std::vector<double> g = gauss_points(c->k);
  // beta^p along the axis xi (ln p or p): -(dU/dt ca A^x + U' cu (A^x A^x)_t)
  // with ca = gamma m / p, cu = 1 on ln p (beta^{ln p} = beta^p / p) and
  // ca = gamma m, cu = p on p; -div beta holds -dU/dt idiv A^x with
  // idiv = m/(gamma p) (ln p) or -V (p; d(gamma m)/dp = V), and on p also
  // + U' (A^x A^x)_t (FieldArgs::t_divu)
  std::vector<double> V(np * K1), iV(np * K1), idiv(np * K1), ig(np * K1), iVf(np + 1);
  std::vector<double> ca(np * K1), cu(np * K1), cuf(np + 1);
  c->vmax = 0.0;
  for (int i = 0; i < np; ++i)
    for (int q = 0; q < K1; ++q) {
      double xi = nd[i] + (1.0 + g[q]) * 0.5 * (nd[i + 1] - nd[i]);
      double p = c->linp ? xi : std::exp(xi);
      double gam = std::sqrt(1.0 + (p / c->mass) * (p / c->mass));
      const int j = i * K1 + q;
      V[j] = p / (gam * c->mass);
      iV[j] = gam * c->mass / p;
      idiv[j] = c->linp ? -V[j] : c->mass / (gam * p);
      ig[j] = c->charge / (gam * c->mass);
      ca[j] = c->linp ? gam * c->mass : iV[j];
      cu[j] = c->linp ? p : 1.0;
      c->vmax = std::max(c->vmax, V[j]);
    }
  for (int f = 0; f <= np; ++f) {
    double p = c->linp ? nd[f] : std::exp(nd[f]);
    double gam = std::sqrt(1.0 + (p / c->mass) * (p / c->mass));
    iVf[f] = c->linp ? gam * c->mass : gam * c->mass / p;
    cuf[f] = c->linp ? p : 1.0;
    c->vmax = std::max(c->vmax, p / (gam * c->mass));
  }
  if (int e = upload_vec(c->d_ca_vol, ca)) return e;
  if (int e = upload_vec(c->d_cu_vol, cu)) return e;
  if (int e = upload_vec(c->d_cu_face, cuf)) return e;
  if (int e = upload_vec(c->d_V_vol, V)) return e;
  if (int e = upload_vec(c->d_iV_vol, iV)) return e;
  if (int e = upload_vec(c->d_idiv_vol, idiv)) return e;
  if (int e = upload_vec(c->d_ig_vol, ig)) return e;
  if (int e = upload_vec(c->d_iV_face, iVf)) return e;
  return VFP_OK;
}

// Eigen-decomposition of a small symmetric matrix (cyclic Jacobi), in place:
// on return a[i][i] are the eigenvalues and v the eigenvectors (columns).
constexpr int kBlk = kMaxLmax + 1;
// Converged as jacobi_eigh: off-diagonal entries below 1e-18 of the
// Frobenius norm are set to zero, and the first sweep without a rotation ends.
void small_eigh(int n, double (&a)[kBlk][kBlk], double (&v)[kBlk][kBlk]) {
  double tot = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      v[i][j] = (i == j) ? 1.0 : 0.0;
      tot += a[i][j] * a[i][j];
    }
  const double small = 1e-18 * std::sqrt(tot);
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p][q];
        if (std::fabs(apq) <= small) {
          a[p][q] = a[q][p] = 0.0;
          continue;
        }
        rotated = true;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = cs * akp - sn * akq;
          a[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = cs * apk - sn * aqk;
          a[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = cs * vkp - sn * vkq;
          v[k][q] = sn * vkp + cs * vkq;
        }
      }
    if (!rotated) break;
  }
}

int host_threads() {
  for (const char* name : {"VFP_HOST_THREADS", "OMP_NUM_THREADS"}) {
    const char* e = std::getenv(name);
    if (e && std::atoi(e) > 0) return std::min(std::atoi(e), 64);
  }
  const unsigned hw = std::thread::hardware_concurrency();
  return hw ? (int)std::min(hw, 16u) : 1;
}

// p-face upwind data: beta^{ln p} = a1 A^x + a2 (A^x A^x)_t at each (x point,
// p face); it keeps the (m,s) blocks of A^x (and the s = 0 and s = 1 blocks
// of one m are equal), so each m block is diagonalised once.  Points where
// beta^{ln p} vanishes (no flow gradient) are trivially code -1.  The
// derivative tables of B_+ are built once field gradients have been asked
// for (c->pf_dk); dk_only rebuilds just those (the codes and B_+ rows come
// out the same and stay as uploaded).
int build_pface_data(vfp_ctx* c, bool dk_only = false) {
  if (!c->mom || !c->mesh_set) return VFP_OK;
  const bool dk = c->pf_dk;
  const int pa = c->naxes - 1, K1 = c->K1, n = c->n, L = c->lmax;
  const int nxp = c->ncell[0] * K1, npf = c->ncell[pa] + 1;
  const std::vector<double>& nd = c->nodes[pa];
  const double tm = (c->terms & VFP_TERM_MOMENTUM) ? 1.0 : 0.0;
  // the m blocks of A^x and (A^x A^x)_t
  std::vector<double> ab((size_t)(L + 1) * kBlk * kBlk, 0.0), xb(ab.size(), 0.0);
  for (int m = 0; m <= L; ++m)
    for (int i = 0; i <= L - m; ++i)
      for (int j = 0; j <= L - m; ++j) {
        const int ri = lms_index(m + i, m, 0), rj = lms_index(m + j, m, 0);
        ab[((size_t)m * kBlk + i) * kBlk + j] = c->S.A[0](ri, rj);
        xb[((size_t)m * kBlk + i) * kBlk + j] = c->S.AXX(ri, rj);
      }
  // coefficients of dU/dt and U' in beta^p at each p face (see build_momentum_data)
  std::vector<double> inv_v(npf), cu_f(npf);
  for (int f = 0; f < npf; ++f) {
    const double p = c->linp ? nd[f] : std::exp(nd[f]);
    const double gam = std::sqrt(1.0 + (p / c->mass) * (p / c->mass));
    inv_v[f] = c->linp ? gam * c->mass : gam * c->mass / p;
    cu_f[f] = c->linp ? p : 1.0;
  }
  const size_t rowsz = (size_t)n * (L + 1);
  struct Part {
    std::vector<int> code_ix;            // [ix - lo][f]
    std::vector<double> tab;             // rows of mixed-sign points, in (ix, f) order
    std::vector<double> dtab;            // rows of dB_+[A^x], dB_+[(A^xA^x)_t] of the same points
    double bmax = 0.0;
  };
  const int nth = std::max(1, std::min(host_threads(), nxp));
  std::vector<Part> parts(nth);
  auto work = [&](int t) {
    const int lo = (int)((long long)nxp * t / nth), hi = (int)((long long)nxp * (t + 1) / nth);
    Part& P = parts[t];
    P.code_ix.assign((size_t)(hi - lo) * npf, -1);
    std::vector<double> rows(rowsz), drows(rowsz);
    double a[kBlk][kBlk], v[kBlk][kBlk];
    for (int ix = lo; ix < hi; ++ix) {
      const double av = c->planar ? c->a_vol[ix] : 0.0;
      const double du = c->planar ? c->du_vol[ix] : 0.0;
      for (int f = 0; f < npf; ++f) {
        const double a1 = -tm * av * inv_v[f], a2 = -tm * du * cu_f[f];
        if (a1 == 0.0 && a2 == 0.0) continue;       // beta = 0: code -1
        double bnorm = 0.0;
        double ev[kBlk][kBlk];                       // eigenvalues per block
        double vec[kBlk][kBlk][kBlk];                // eigenvectors per block
        for (int m = 0; m <= L; ++m) {
          const int bsz = L - m + 1;
          for (int i = 0; i < bsz; ++i)
            for (int j = 0; j < bsz; ++j)
              a[i][j] = a1 * ab[((size_t)m * kBlk + i) * kBlk + j] + a2 * xb[((size_t)m * kBlk + i) * kBlk + j];
          small_eigh(bsz, a, v);
          for (int i = 0; i < bsz; ++i) {
            ev[m][i] = a[i][i];
            bnorm = std::max(bnorm, std::fabs(a[i][i]));
            for (int j = 0; j < bsz; ++j) vec[m][i][j] = v[i][j];
          }
        }
        P.bmax = std::max(P.bmax, bnorm);
        // eigenvalues within rounding of zero count as zero
        const double tol = 1e-14 * bnorm;
        bool anypos = false, anyneg = false;
        for (int m = 0; m <= L; ++m)
          for (int i = 0; i <= L - m; ++i) {
            anypos |= ev[m][i] > tol;
            anyneg |= ev[m][i] < -tol;
          }
        int cd = -1;
        if (anyneg && !anypos) cd = -2;
        if (anyneg && anypos) {
          // beta_+ rows, for the s = 0 and s = 1 rows of each m alike
          for (int m = 0; m <= L; ++m) {
            const int bsz = L - m + 1;
            for (int i = 0; i < bsz; ++i)
              for (int j = 0; j < bsz; ++j) {
                double acc = 0.0;
                for (int e = 0; e < bsz; ++e) acc += vec[m][i][e] * std::max(ev[m][e], 0.0) * vec[m][j][e];
                for (int s = 0; s <= (m ? 1 : 0); ++s)
                  rows[(size_t)lms_index(m + i, m, s) * (L + 1) + j] = acc;
              }
          }
          cd = (int)(P.tab.size() / rowsz);     // local index, offset on merge
          P.tab.insert(P.tab.end(), rows.begin(), rows.end());
          // derivatives of B_+ in the directions A^x and (A^xA^x)_t
          // (Daleckii-Krein): Q (Gamma o Q^T dB Q) Q^T with
          // Gamma_kl = (l_k^+ - l_l^+) / (l_k - l_l), H(l_k) where equal;
          // only for field gradients (vfp_field_grad_*)
          for (int dir = 0; dk && dir < 2; ++dir) {
            std::fill(drows.begin(), drows.end(), 0.0);
            for (int m = 0; m <= L; ++m) {
              const int bsz = L - m + 1;
              const double* db = (dir == 0 ? ab.data() : xb.data()) + (size_t)m * kBlk * kBlk;
              const double(&Q)[kBlk][kBlk] = vec[m];
              double W[kBlk][kBlk], D[kBlk][kBlk];
              for (int i = 0; i < bsz; ++i)          // W = dB Q
                for (int l = 0; l < bsz; ++l) {
                  double acc = 0.0;
                  for (int j = 0; j < bsz; ++j) acc += db[i * kBlk + j] * Q[j][l];
                  W[i][l] = acc;
                }
              for (int k = 0; k < bsz; ++k)          // D = Gamma o (Q^T W)
                for (int l = 0; l < bsz; ++l) {
                  double acc = 0.0;
                  for (int i = 0; i < bsz; ++i) acc += Q[i][k] * W[i][l];
                  const double lk = ev[m][k], ll = ev[m][l], dl = lk - ll;
                  const double gam = std::fabs(dl) > 1e-14 * (std::fabs(lk) + std::fabs(ll))
                                         ? (std::max(lk, 0.0) - std::max(ll, 0.0)) / dl
                                         : (lk > 0 ? 1.0 : (lk < 0 ? 0.0 : 0.5));
                  D[k][l] = gam * acc;
                }
              for (int i = 0; i < bsz; ++i)          // W = Q D
                for (int l = 0; l < bsz; ++l) {
                  double acc = 0.0;
                  for (int k = 0; k < bsz; ++k) acc += Q[i][k] * D[k][l];
                  W[i][l] = acc;
                }
              for (int i = 0; i < bsz; ++i)          // rows of W Q^T
                for (int j = 0; j < bsz; ++j) {
                  double acc = 0.0;
                  for (int l = 0; l < bsz; ++l) acc += W[i][l] * Q[j][l];
                  for (int s = 0; s <= (m ? 1 : 0); ++s)
                    drows[(size_t)lms_index(m + i, m, s) * (L + 1) + j] = acc;
                }
            }
            P.dtab.insert(P.dtab.end(), drows.begin(), drows.end());
          }
        }
        P.code_ix[(size_t)(ix - lo) * npf + f] = cd;
      }
    }
  };
  if (nth == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  std::vector<int> code((size_t)nxp * npf, -1);
  std::vector<double> tab, dtab;
  c->beta_pmax = 0.0;
  for (int t = 0; t < nth; ++t) {
    const int lo = (int)((long long)nxp * t / nth), hi = (int)((long long)nxp * (t + 1) / nth);
    const int off = (int)(tab.size() / rowsz);
    const Part& P = parts[t];
    for (int ix = lo; ix < hi; ++ix)
      for (int f = 0; f < npf; ++f) {
        const int cd = P.code_ix[(size_t)(ix - lo) * npf + f];
        code[(size_t)f * nxp + ix] = cd >= 0 ? cd + off : cd;
      }
    tab.insert(tab.end(), P.tab.begin(), P.tab.end());
    dtab.insert(dtab.end(), P.dtab.begin(), P.dtab.end());
    c->beta_pmax = std::max(c->beta_pmax, P.bmax);
  }
  if (dk) {
    if (dtab.empty()) dtab.assign(2 * rowsz, 0.0);
    if (int e = upload_vec(c->d_pf_dtab, dtab)) return e;
  } else {
    c->d_pf_dtab.release();
  }
  if (dk_only) return VFP_OK;
  if (int e = upload_vec(c->d_pf_code, code)) return e;
  std::vector<double> coded(code.begin(), code.end());
  if (int e = upload_vec(c->d_pf_coded, coded)) return e;
  if (tab.empty()) tab.assign(rowsz, 0.0);
  if (int e = upload_vec(c->d_pf_tab, tab)) return e;
  return VFP_OK;
}

// Binds the context to the current device on first use and uploads the
// 1-D basis tables to that device once per process.
int ensure_device(vfp_ctx* c) {
  if (c->device >= 0) return VFP_OK;
  int cnt = 0;
  hipError_t e = hipGetDeviceCount(&cnt);
  if (e != hipSuccess || cnt <= 0) return fail(VFP_EDEVICE, "no HIP device available");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(VFP_EDEVICE, "device ordinal %d", dev);
  if (!g_basis_ready[dev]) {
    Basis1D b[kMaxK];
    for (int k = 1; k <= kMaxK; ++k) b[k - 1] = make_basis(k);
    HIP_TRY(upload_basis(b));
    g_basis_ready[dev] = true;
  }
  c->device = dev;
  const int zero = 0;
  return upload(c->d_flag, &zero, sizeof(int));
}

// Packed per-x-cell and per-p-cell scalar records (see FieldArgs::xrec).
int build_records(vfp_ctx* c) {
  // the records hold three Gauss points per axis; the (x, ln p) and (x, p)
  // kernels that read them exist for k <= 2
  if (!c->mom || !c->mesh_set || c->k > 2) return VFP_OK;
  const int K1 = c->K1, nxc = c->ncell[0], pa = c->naxes - 1, npc = c->ncell[pa];
  const double ta = (c->terms & VFP_TERM_ADVECTION) ? 1.0 : 0.0;
  const double tm = (c->terms & VFP_TERM_MOMENTUM) ? 1.0 : 0.0;
  const double tr = (c->terms & VFP_TERM_ROTATION) ? 1.0 : 0.0;
  std::vector<double> xr((size_t)nxc * kRec, 0.0), pr((size_t)npc * kRec, 0.0);
  for (int i = 0; i < nxc; ++i) {
    const double s2h = 2.0 / (c->nodes[0][i + 1] - c->nodes[0][i]);
    double* x = &xr[(size_t)i * kRec];
    for (int q = 0; q < K1; ++q) {
      x[0 + q] = ta * s2h * c->u_vol[i * K1 + q];
      x[3 + q] = c->du_vol[i * K1 + q];
      x[6 + q] = tm * c->a_vol[i * K1 + q];
    }
    x[9] = ta * c->u_face[i];
    x[10] = ta * c->u_face[i + 1];
    x[11] = s2h;
    // flow gradient present at a Gauss point of this x cell (else every
    // momentum and divergence term of its cells is exactly zero)
    bool g = false;
    for (int q = 0; q < K1; ++q) g |= c->du_vol[i * K1 + q] != 0.0 || c->a_vol[i * K1 + q] != 0.0;
    x[12] = g ? 1.0 : 0.0;
  }
  const std::vector<double>& nd = c->nodes[pa];
  std::vector<double> g = gauss_points(c->k);
  // on a p axis: the m/(gamma p) slot holds -V (-div beta = dU/dt V A^x + ...),
  // the face slots t_mom gamma m, and the extra record gamma m, p (Gauss
  // points) and p (faces)
  std::vector<double> pr2(c->linp ? (size_t)npc * 8 : 0, 0.0);
  for (int j = 0; j < npc; ++j) {
    double* p = &pr[(size_t)j * kRec];
    for (int q = 0; q < K1; ++q) {
      const double xi = nd[j] + (1.0 + g[q]) * 0.5 * (nd[j + 1] - nd[j]);
      const double pp = c->linp ? xi : std::exp(xi);
      const double gam = std::sqrt(1.0 + (pp / c->mass) * (pp / c->mass));
      p[0 + q] = pp / (gam * c->mass);
      p[3 + q] = gam * c->mass / pp;
      p[6 + q] = c->linp ? -pp / (gam * c->mass) : c->mass / (gam * pp);
      p[9 + q] = tr * c->charge / (gam * c->mass);
      if (c->linp) {
        pr2[(size_t)j * 8 + q] = gam * c->mass;
        pr2[(size_t)j * 8 + 3 + q] = pp;
      }
    }
    for (int s = 0; s < 2; ++s) {
      const double pp = c->linp ? nd[j + s] : std::exp(nd[j + s]);
      const double gam = std::sqrt(1.0 + (pp / c->mass) * (pp / c->mass));
      p[12 + s] = tm * gam * c->mass / (c->linp ? 1.0 : pp);
      if (c->linp) pr2[(size_t)j * 8 + 6 + s] = pp;
    }
    p[14] = 2.0 / (nd[j + 1] - nd[j]);
  }
  if (int e = upload_vec(c->d_xrec, xr)) return e;
  if (int e = upload_vec(c->d_prec, pr)) return e;
  if (c->linp)
    if (int e = upload_vec(c->d_prec2, pr2)) return e;
  return VFP_OK;
}

// What a set-up call invalidates.
enum : unsigned { R_TAB = 1, R_MOM = 2, R_PFACE = 4, R_REC = 8, R_ALL = 15 };

int refresh(vfp_ctx* c, unsigned what) {
  if (!c->mesh_set) return VFP_OK;
  if (int e = ensure_device(c)) return e;
  if (what & R_TAB)
    if (int e = build_row_tables(c)) return e;
  if (what & R_MOM)
    if (int e = build_momentum_data(c)) return e;
  if (what & R_PFACE)
    if (int e = build_pface_data(c)) return e;
  if (what & R_REC)
    if (int e = build_records(c)) return e;
  FieldArgs& F = c->fld;
  F = FieldArgs{};
  F.u_vol = c->d_u_vol.as<double>();
  F.du_vol = c->d_du_vol.as<double>();
  F.a_vol = c->d_a_vol.as<double>();
  F.u_face = c->d_u_face.as<double>();
  for (int i = 0; i < 3; ++i) F.U[i] = c->U[i];
  F.V_vol = c->d_V_vol.as<double>();
  F.iV_vol = c->d_iV_vol.as<double>();
  F.idiv_vol = c->d_idiv_vol.as<double>();
  F.ig_vol = c->d_ig_vol.as<double>();
  F.iV_face = c->d_iV_face.as<double>();
  F.ca_vol = c->d_ca_vol.as<double>();
  F.cu_vol = c->d_cu_vol.as<double>();
  F.cu_face = c->d_cu_face.as<double>();
  F.t_divu = c->linp ? 1.0 : 0.0;
  if (!c->mom) {
    double p = c->p_fixed;
    double gam = std::sqrt(1.0 + (p / c->mass) * (p / c->mass));
    F.V0 = p / (gam * c->mass);
    F.iV0 = gam * c->mass / p;
    F.ig0 = c->charge / (gam * c->mass);
    c->vmax = F.V0;
  }
  F.pf_code = c->d_pf_code.as<int>();
  F.pf_coded = c->d_pf_coded.as<double>();
  F.xrec = c->d_xrec.as<double>();
  F.prec = c->d_prec.as<double>();
  F.prec2 = c->linp ? c->d_prec2.as<double>() : nullptr;
  F.pf_tab = c->d_pf_tab.as<double>();
  F.pf_dtab = c->d_pf_dtab.as<double>();
  for (int i = 0; i < 3; ++i) F.B[i] = c->B[i];
  F.B_pts = c->have_Bpts ? c->d_Bpts.as<double>() : nullptr;
  F.nu0 = c->nu0;
  F.nu_cell = c->have_nu_cell ? c->d_nu.as<double>() : nullptr;
  F.nu_pts = c->have_nu_pts ? c->d_nu_pts.as<double>() : nullptr;
  F.u_pts = c->pflow ? c->d_u_pts.as<double>() : nullptr;
  for (int a = 0; a < 3; ++a) F.uf_pts[a] = c->pflow ? c->d_uf_pts[a].as<double>() : nullptr;
  F.src = c->have_src ? c->d_src.as<double>() : nullptr;
  F.t_adv = (c->terms & VFP_TERM_ADVECTION) ? 1.0 : 0.0;
  F.t_mom = (c->terms & VFP_TERM_MOMENTUM) ? 1.0 : 0.0;
  F.t_rot = (c->terms & VFP_TERM_ROTATION) ? 1.0 : 0.0;
  F.t_col = (c->terms & VFP_TERM_COLLISION) ? 1.0 : 0.0;
  if (c->mom && !c->planar) {
    // a momentum axis needs the x profile arrays; a uniform flow is stored as
    // a constant profile
    return VFP_OK;
  }
  c->launcher = nullptr;
  c->shock = false;
  const bool shock_ok = c->naxes == 2 && c->mom && c->planar && !c->have_Bpts && !c->have_nu_pts &&
                        !c->force_general;
  if (shock_ok) {
    if (c->shape && !c->linp) c->launcher = find_shock_launcher_shape(c->k, c->lmax, c->tab.nrot, c->shape);
    if (!c->launcher) {
      c->shape = 0;
      c->launcher = find_shock_launcher(c->k, c->lmax, c->tab.nrot, c->linp);
    }
    c->shock = c->launcher != nullptr;
  }
  const int flow = c->pflow ? 2 : (c->planar ? 1 : 0);
  if (!c->launcher) c->launcher = find_stage_launcher(c->naxes, c->k, c->lmax, c->mom, flow);
  c->adj_launcher = nullptr;
  if (shock_ok) c->adj_launcher = find_shock_adjoint_launcher(c->k, c->lmax, c->tab.nrot, c->linp);
  c->adj_shock = c->adj_launcher != nullptr;
  if (!c->adj_launcher) c->adj_launcher = find_adjoint_launcher(c->naxes, c->k, c->lmax, c->mom, flow);
  c->mass_launcher = find_mass_launcher(c->naxes, c->k);
  // a small run on one axis with constant coefficients (uniform flow, fixed
  // p, uniform B, nu per cell) steps inside one workgroup (VFP_RESIDENT=0
  // turns this off)
  c->resident = nullptr;
  {
    const char* rv = std::getenv("VFP_RESIDENT");
    const bool allow = !(rv && std::atoi(rv) == 0);
    const size_t lds = (size_t)3 * c->ncells * c->nb * c->n * sizeof(double);
    const bool fits = (int64_t)c->ncells * c->n <= kResidentItems && c->tab.nfb[0] <= kResFbCap &&
                      c->tab.nfa[0] <= c->lmax + 2 && c->tab.nrot <= kResRotCap;
    if (allow && fits && c->naxes == 1 && !c->mom && !c->planar && !c->pflow && !c->have_Bpts && !c->have_nu_pts &&
        c->lmax <= kShFullMaxLmax && lds <= resident_max_lds())
      c->resident = find_resident_launcher(c->k, c->lmax);
  }
  return VFP_OK;
}

int check_ready(const vfp_ctx* c) {
  if (!c) return fail(VFP_EINVAL, "null context");
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (!c->mom && !(c->p_fixed > 0)) return fail(VFP_ESTATE, "vfp_set_momentum has not been called");
  if (c->mom && !c->planar) return fail(VFP_ESTATE, "a ln p axis needs vfp_set_flow_planar (a constant profile for uniform flow)");
  if (!c->launcher)
    return fail(VFP_EUNSUPPORTED, "no kernel built for naxes=%d k=%d lmax=%d lnp=%d planar=%d point flow=%d",
                c->naxes, c->k, c->lmax, (int)c->mom, (int)c->planar, (int)c->pflow);
  return VFP_OK;
}

}  // namespace

// ===================================================================== ABI

extern "C" {

const char* vfp_last_error(void) { return g_err.c_str(); }

int vfp_create(vfp_ctx** out, int lmax, int k, int naxes, const int* axis_kinds, unsigned term_mask,
               double mass, double charge) {
  if (!out) return fail(VFP_EINVAL, "out is null");
  *out = nullptr;
  if (lmax < 1 || lmax > kMaxLmax) return fail(VFP_EINVAL, "lmax=%d outside [1,%d]", lmax, kMaxLmax);
  if (k < 1 || k > kMaxK) return fail(VFP_EINVAL, "k=%d outside [1,%d]", k, kMaxK);
  if (naxes < 1 || naxes > 3) return fail(VFP_EINVAL, "naxes=%d outside [1,3]", naxes);
  if (!axis_kinds) return fail(VFP_EINVAL, "axis_kinds is null");
  if (!(mass > 0) || !std::isfinite(mass) || !std::isfinite(charge)) return fail(VFP_EINVAL, "bad mass/charge");
  if (term_mask & ~31u) return fail(VFP_EINVAL, "unknown term bits 0x%x", term_mask);
  int nsp = 0;
  bool mom = false;
  for (int a = 0; a < naxes; ++a) {
    int kd = axis_kinds[a];
    if (kd == VFP_AXIS_LNP || kd == VFP_AXIS_P) {
      if (a != naxes - 1) return fail(VFP_EINVAL, "the ln p (or p) axis must be the last axis");
      mom = true;
    } else if (kd >= VFP_AXIS_X && kd <= VFP_AXIS_Z) {
      if (kd != a) return fail(VFP_EINVAL, "spatial axes must be x, y, z in order");
      ++nsp;
    } else {
      return fail(VFP_EINVAL, "axis kind %d unknown", kd);
    }
  }
  if (mom && nsp > 2) return fail(VFP_EINVAL, "at most two spatial axes with a ln p axis");
  if (nsp == 0) return fail(VFP_EINVAL, "at least one spatial axis is required");
  if ((naxes == 3 && k > 2) || (naxes == 2 && k > 3))
    return fail(VFP_EUNSUPPORTED, "k=%d is built for at most %d axes", k, k > 3 ? 1 : 2);
  if (lmax > kShFullMaxLmax && (naxes != 1 || mom || k > 2))
    return fail(VFP_EUNSUPPORTED, "l_max > %d is built for one spatial axis (x) at fixed p with k <= 2",
                kShFullMaxLmax);
  vfp_ctx* c = new (std::nothrow) vfp_ctx();
  if (!c) return fail(VFP_ENOMEM, "context allocation");
  c->lmax = lmax;
  c->k = k;
  c->naxes = naxes;
  c->n = (lmax + 1) * (lmax + 1);
  c->K1 = k + 1;
  c->nb = 1;
  for (int a = 0; a < naxes; ++a) {
    c->nb *= c->K1;
    c->axes[a] = axis_kinds[a];
  }
  c->terms = term_mask;
  c->mass = mass;
  c->charge = charge;
  c->mom = mom;
  c->linp = mom && axis_kinds[naxes - 1] == VFP_AXIS_P;
  c->nspace = nsp;
  {
    const char* kv = std::getenv("VFP_KERNEL");
    c->force_general = kv && std::strcmp(kv, "general") == 0;
    const char* tm = std::getenv("VFP_TILE_MAP");
    c->tile_map = tm ? (std::atoi(tm) != 0) : 0;
    const char* sh = std::getenv("VFP_SHOCK_SHAPE");   // initial workgroup shape slot (tests)
    c->shape = sh ? std::max(0, std::min(kShockShapes - 1, std::atoi(sh))) : 0;
  }
  c->S = build_sh_matrices(lmax);
  {
    std::vector<double> lam;
    Mat W;
    jacobi_eigh(c->S.A[0], lam, W);
    c->lam_max = *std::max_element(lam.begin(), lam.end());
  }
  *out = c;
  return VFP_OK;
}

void vfp_destroy(vfp_ctx* c) { delete c; }

int vfp_set_mesh(vfp_ctx* c, const int* ncells, const double* const* nodes, const int* bc_lo,
                 const int* bc_hi) {
  if (!c || !ncells || !nodes || !bc_lo || !bc_hi) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  long long tot = 1;
  for (int a = 0; a < c->naxes; ++a) {
    if (ncells[a] < 1) return fail(VFP_EINVAL, "ncells[%d]=%d", a, ncells[a]);
    if (!nodes[a]) return fail(VFP_EINVAL, "nodes[%d] is null", a);
    for (int i = 0; i < ncells[a]; ++i)
      if (!(nodes[a][i + 1] > nodes[a][i]) || !std::isfinite(nodes[a][i + 1]))
        return fail(VFP_EINVAL, "nodes[%d] not strictly increasing at %d", a, i);
    if (c->linp && a == c->naxes - 1 && !(nodes[a][0] > 0.0))
      return fail(VFP_EINVAL, "the p axis must start above p = 0");
    for (int lohi = 0; lohi < 2; ++lohi) {
      int b = lohi ? bc_hi[a] : bc_lo[a];
      if (b < 0 || b > 2) return fail(VFP_EINVAL, "bc kind %d unknown", b);
    }
    if ((bc_lo[a] == VFP_BC_PERIODIC) != (bc_hi[a] == VFP_BC_PERIODIC))
      return fail(VFP_EINVAL, "axis %d: periodic must be set on both ends", a);
    tot *= ncells[a];
  }
  if (tot > (1LL << 31) / 64) return fail(VFP_EINVAL, "too many cells (%lld)", tot);
  c->ncells = (int)tot;
  for (int a = 0; a < 3; ++a) {
    c->ncell[a] = a < c->naxes ? ncells[a] : 1;
    c->bc_lo[a] = a < c->naxes ? bc_lo[a] : 0;
    c->bc_hi[a] = a < c->naxes ? bc_hi[a] : 0;
    c->nodes[a].clear();
    if (a < c->naxes) c->nodes[a].assign(nodes[a], nodes[a] + ncells[a] + 1);
  }
  // reset fields
  c->planar = false;
  for (int i = 0; i < 3; ++i) c->U[i] = c->B[i] = 0.0;
  c->have_Bpts = c->have_nu_cell = c->have_nu_pts = c->have_src = false;
  c->pflow = false;
  c->d_fg_support.release();
  c->d_fg_blocks.release();
  c->fg_nblocks = 0;
  c->nu0 = 0.0;
  c->u_vol.assign(c->ncell[0] * c->K1, 0.0);
  c->du_vol = c->a_vol = c->u_vol;
  c->u_face.assign(c->ncell[0] + 1, 0.0);
  c->mesh_set = true;
  for (int a = 0; a < 3; ++a) {
    c->meshargs.n[a] = c->ncell[a];
    c->meshargs.bc_lo[a] = c->bc_lo[a];
    c->meshargs.bc_hi[a] = c->bc_hi[a];
  }
  c->meshargs.ncells = c->ncells;
  if (c->mom) c->planar = true;   // a ln p axis always uses the x-profile kernels (U = 0 to start)
  if (int e = ensure_device(c)) return e;
  for (int a = 0; a < 3; ++a) {
    std::vector<double> s2h(c->ncell[a], 0.0);
    if (a < c->naxes)
      for (int i = 0; i < c->ncell[a]; ++i) s2h[i] = 2.0 / (c->nodes[a][i + 1] - c->nodes[a][i]);
    if (int e = upload_vec(c->d_s2h[a], s2h)) return e;
    c->meshargs.s2h[a] = c->d_s2h[a].as<double>();
  }
  if (c->mom) {
    if (int e = upload_vec(c->d_u_vol, c->u_vol)) return e;
    if (int e = upload_vec(c->d_du_vol, c->du_vol)) return e;
    if (int e = upload_vec(c->d_a_vol, c->a_vol)) return e;
    if (int e = upload_vec(c->d_u_face, c->u_face)) return e;
  }
  if (!c->mom && !(c->p_fixed > 0)) return VFP_OK;
  return refresh(c, R_ALL);
}

int vfp_set_momentum(vfp_ctx* c, double p) {
  if (!c) return fail(VFP_EINVAL, "null context");
  ++c->gen;
  if (c->mom) return fail(VFP_EINVAL, "context has a ln p axis; momentum is a coordinate");
  if (!(p > 0) || !std::isfinite(p)) return fail(VFP_EINVAL, "p=%g must be positive", p);
  c->p_fixed = p;
  return refresh(c, R_TAB);
}

int vfp_query_points(const vfp_ctx* c, int which, int axis, double* coords, int64_t* count) {
  if (!c || !count) return fail(VFP_EINVAL, "null argument");
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (axis < 0 || axis >= c->naxes) return fail(VFP_EINVAL, "axis %d", axis);
  const int na = c->ncell[axis], K1 = c->K1;
  const std::vector<double>& nd = c->nodes[axis];
  if (which == VFP_PTS_FACE) {
    *count = na + 1;
    if (coords) std::copy(nd.begin(), nd.end(), coords);
    return VFP_OK;
  }
  if (which != VFP_PTS_VOLUME && which != VFP_PTS_NODE) return fail(VFP_EINVAL, "point set %d", which);
  *count = (int64_t)na * K1;
  if (!coords) return VFP_OK;
  std::vector<double> ref = (which == VFP_PTS_VOLUME) ? gauss_points(c->k)
                                                      : (c->k == 1 ? std::vector<double>{-1.0, 1.0}
                                                                   : std::vector<double>{-1.0, 0.0, 1.0});
  for (int i = 0; i < na; ++i)
    for (int q = 0; q < K1; ++q) coords[i * K1 + q] = nd[i] + (1.0 + ref[q]) * 0.5 * (nd[i + 1] - nd[i]);
  return VFP_OK;
}

int vfp_set_flow_uniform(vfp_ctx* c, const double* U) {
  if (!c || !U) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(U[i])) return fail(VFP_EINVAL, "U not finite");
  for (int i = 0; i < 3; ++i) c->U[i] = U[i];
  c->pflow = false;
  if (c->mom) {
    // stored as a constant x profile (grad U = 0, dU/dt = 0)
    std::fill(c->u_vol.begin(), c->u_vol.end(), U[0]);
    std::fill(c->u_face.begin(), c->u_face.end(), U[0]);
    std::fill(c->du_vol.begin(), c->du_vol.end(), 0.0);
    std::fill(c->a_vol.begin(), c->a_vol.end(), 0.0);
    if (int e = upload_vec(c->d_u_vol, c->u_vol)) return e;
    if (int e = upload_vec(c->d_du_vol, c->du_vol)) return e;
    if (int e = upload_vec(c->d_a_vol, c->a_vol)) return e;
    if (int e = upload_vec(c->d_u_face, c->u_face)) return e;
  } else {
    c->planar = false;
  }
  return refresh(c, R_TAB | R_PFACE | R_REC);
}

int vfp_set_flow_planar(vfp_ctx* c, const double* u, const double* dudx, const double* dudt,
                        const double* u_face) {
  if (!c || !u || !dudx || !dudt || !u_face) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (c->axes[0] != VFP_AXIS_X) return fail(VFP_EINVAL, "planar flow needs axis 0 = x");
  const int nq = c->ncell[0] * c->K1;
  for (int i = 0; i < nq; ++i)
    if (!std::isfinite(u[i]) || !std::isfinite(dudx[i]) || !std::isfinite(dudt[i]))
      return fail(VFP_EINVAL, "flow profile not finite at %d", i);
  c->u_vol.assign(u, u + nq);
  c->du_vol.assign(dudx, dudx + nq);
  c->a_vol.assign(dudt, dudt + nq);
  c->u_face.assign(u_face, u_face + c->ncell[0] + 1);
  c->U[0] = 0.0;
  c->planar = true;
  c->pflow = false;
  if (int e = upload_vec(c->d_u_vol, c->u_vol)) return e;
  if (int e = upload_vec(c->d_du_vol, c->du_vol)) return e;
  if (int e = upload_vec(c->d_a_vol, c->a_vol)) return e;
  if (int e = upload_vec(c->d_u_face, c->u_face)) return e;
  return refresh(c, R_PFACE | R_REC);
}

int vfp_set_magnetic_uniform(vfp_ctx* c, const double* B) {
  if (!c || !B) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (c->lmax > kShFullMaxLmax && (B[1] != 0.0 || B[2] != 0.0))
    return fail(VFP_EUNSUPPORTED, "l_max > %d: B must lie along x", kShFullMaxLmax);
  for (int i = 0; i < 3; ++i) c->B[i] = B[i];
  c->have_Bpts = false;
  return refresh(c, R_TAB);
}

int vfp_set_magnetic_points(vfp_ctx* c, const double* B) {
  if (!c || !B) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (c->lmax > kShFullMaxLmax) return fail(VFP_EUNSUPPORTED, "l_max > %d: B must be uniform along x", kShFullMaxLmax);
  if (int e = upload(c->d_Bpts, B, (size_t)c->ncells * c->nb * 3 * sizeof(double))) return e;
  c->have_Bpts = true;
  for (int i = 0; i < 3; ++i) c->B[i] = 0.0;
  return refresh(c, R_TAB);
}

int vfp_set_scattering(vfp_ctx* c, double nu, const double* nu_cell) {
  if (!c) return fail(VFP_EINVAL, "null context");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (nu_cell) {
    for (int i = 0; i < c->ncells; ++i)
      if (!std::isfinite(nu_cell[i])) return fail(VFP_EINVAL, "nu_cell[%d] not finite", i);
    if (c->have_nu_cell && c->d_nu.bytes == (size_t)c->ncells * sizeof(double)) {
      // same size: overwrite in place (ordered after work already queued on
      // the null stream; callers on other streams synchronise first)
      HIP_TRY(hipMemcpy(c->d_nu.p, nu_cell, c->d_nu.bytes, hipMemcpyHostToDevice));
    } else if (int e = upload(c->d_nu, nu_cell, (size_t)c->ncells * sizeof(double))) {
      return e;
    }
    c->have_nu_cell = true;
  } else {
    if (!std::isfinite(nu)) return fail(VFP_EINVAL, "nu not finite");
    c->nu0 = nu;
    c->have_nu_cell = false;
  }
  const bool had_pts = c->have_nu_pts;
  c->have_nu_pts = false;
  if (c->launcher && !had_pts) {
    // only the scattering fields change: no table rebuild
    c->fld.nu0 = c->nu0;
    c->fld.nu_cell = c->have_nu_cell ? c->d_nu.as<double>() : nullptr;
    return VFP_OK;
  }
  return refresh(c, 0);
}

int vfp_set_scattering_points(vfp_ctx* c, const double* nu) {
  if (!c || !nu) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  const size_t cnt = (size_t)c->ncells * c->nb;
  for (size_t i = 0; i < cnt; ++i)
    if (!std::isfinite(nu[i])) return fail(VFP_EINVAL, "nu[%zu] not finite", i);
  if (int e = upload(c->d_nu_pts, nu, cnt * sizeof(double))) return e;
  c->have_nu_pts = true;
  c->have_nu_cell = false;
  c->nu0 = 0.0;
  return refresh(c, 0);
}

int vfp_set_flow_points(vfp_ctx* c, const double* U, const double* gradU, const double* const* U_face) {
  if (!c || !U || !gradU || !U_face) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  if (c->mom)
    return fail(VFP_EUNSUPPORTED, "flow at the points with a momentum axis (use vfp_set_flow_planar)");
  if (c->terms & VFP_TERM_MOMENTUM)
    return fail(VFP_EUNSUPPORTED, "the flow-gradient terms of R need a momentum axis and a planar flow");
  if (c->k > 2) return fail(VFP_EUNSUPPORTED, "flow at the points is built for k <= 2");
  const int nb = c->nb, K1 = c->K1, D = c->naxes;
  const size_t nq = (size_t)c->ncells * nb;
  std::vector<double> up(nq * 4);
  for (size_t i = 0; i < nq; ++i) {
    double div = 0.0;
    for (int a = 0; a < D; ++a) div += gradU[i * 9 + 4 * c->axes[a]];   // dU_a/dx^a
    for (int b = 0; b < 3; ++b) up[i * 4 + b] = U[i * 3 + b];
    up[i * 4 + 3] = div;
    for (int b = 0; b < 4; ++b)
      if (!std::isfinite(up[i * 4 + b])) return fail(VFP_EINVAL, "flow not finite at volume point %zu", i);
  }
  double umax[3] = {0, 0, 0};
  for (size_t i = 0; i < nq; ++i)
    for (int a = 0; a < D; ++a) umax[a] = std::max(umax[a], std::fabs(U[i * 3 + c->axes[a]]));
  std::vector<double> uf[3];
  for (int a = 0; a < D; ++a) {
    if (!U_face[a]) return fail(VFP_EINVAL, "U_face[%d] is null", a);
    size_t nf = 1;
    for (int b = 0; b < D; ++b) nf *= (size_t)(c->ncell[b] + (b == a ? 1 : 0));
    size_t nqf = 1;
    for (int b = 0; b < D - 1; ++b) nqf *= K1;
    uf[a].resize(nf * nqf);
    for (size_t i = 0; i < nf * nqf; ++i) {
      const double v = U_face[a][i * 3 + c->axes[a]];
      if (!std::isfinite(v)) return fail(VFP_EINVAL, "flow not finite at face point %zu of axis %d", i, a);
      uf[a][i] = v;
      umax[a] = std::max(umax[a], std::fabs(v));
    }
    if (c->bc_lo[a] == VFP_BC_PERIODIC) {
      // the wrap-around face is one face: both ends must carry the same flow
      size_t stride = 1;
      for (int b = 0; b < a; ++b) stride *= (size_t)c->ncell[b];
      const size_t na = (size_t)c->ncell[a];
      for (size_t f = 0; f < nf; ++f) {
        if ((f / stride) % (na + 1) != 0) continue;
        const size_t g = f + na * stride;
        for (size_t q = 0; q < nqf; ++q) {
          const double v0 = uf[a][f * nqf + q], v1 = uf[a][g * nqf + q];
          if (std::fabs(v0 - v1) > 1e-12 * std::max(1.0, std::fabs(v0)))
            return fail(VFP_EINVAL, "axis %d is periodic but the flow differs at its two ends (%g vs %g)", a, v0, v1);
        }
      }
    }
  }
  if (int e = upload_vec(c->d_u_pts, up)) return e;
  for (int a = 0; a < 3; ++a) {
    if (a < D) {
      if (int e = upload_vec(c->d_uf_pts[a], uf[a])) return e;
    } else {
      c->d_uf_pts[a].release();
    }
    c->pflow_umax[a] = a < D ? umax[a] : 0.0;
  }
  for (int i = 0; i < 3; ++i) c->U[i] = 0.0;
  c->planar = false;
  c->pflow = true;
  return refresh(c, R_TAB);
}

int vfp_set_source_points(vfp_ctx* c, const double* s) {
  if (!c || !s) return fail(VFP_EINVAL, "null argument");
  ++c->gen;
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  // M^{-1} h per cell: the 000 component of the test contraction of
  // s_000 = sqrt(4 pi) s (the Jacobian cancels against M^{-1})
  Basis1D b = make_basis(c->k);
  const int nb = c->nb, K1 = c->K1, D = c->naxes;
  std::vector<double> out((size_t)c->ncells * nb, 0.0);
  const double s4 = std::sqrt(4.0 * M_PI);
  for (int cell = 0; cell < c->ncells; ++cell) {
    const double* sc = s + (size_t)cell * nb;
    for (int i = 0; i < nb; ++i) {
      double acc = 0.0;
      for (int q = 0; q < nb; ++q) {
        double t = 1.0;
        int ii = i, qq = q;
        for (int a = 0; a < D; ++a) {
          t *= b.tst[ii % K1][qq % K1];
          ii /= K1;
          qq /= K1;
        }
        acc += t * sc[q];
      }
      out[(size_t)cell * nb + i] = s4 * acc;
    }
  }
  if (int e = upload_vec(c->d_src, out)) return e;
  c->have_src = true;
  return refresh(c, 0);
}

int vfp_ndofs(const vfp_ctx* c, int64_t* n) {
  if (!c || !n) return fail(VFP_EINVAL, "null argument");
  if (!c->mesh_set) return fail(VFP_ESTATE, "vfp_set_mesh has not been called");
  *n = (int64_t)c->ncells * c->nb * c->n;
  return VFP_OK;
}

int vfp_cfl_dt(const vfp_ctx* c, double courant, double* dt) {
  if (int e = check_ready(c)) return e;
  if (!dt || !(courant > 0)) return fail(VFP_EINVAL, "bad courant / dt pointer");
  double sum = 0.0;
  const bool adv = c->terms & VFP_TERM_ADVECTION;
  for (int a = 0; a < c->naxes; ++a) {
    double hmin = 1e300;
    for (int i = 0; i < c->ncell[a]; ++i) hmin = std::min(hmin, c->nodes[a][i + 1] - c->nodes[a][i]);
    double bmax = 0.0;
    if (c->mom && a == c->naxes - 1) {
      bmax = c->beta_pmax;
    } else if (adv) {
      double umax = c->pflow ? c->pflow_umax[a] : std::fabs(c->U[c->axes[a]]);
      if (a == 0 && c->planar) {
        for (double v : c->u_vol) umax = std::max(umax, std::fabs(v));
        for (double v : c->u_face) umax = std::max(umax, std::fabs(v));
      }
      bmax = umax + c->lam_max * c->vmax;
    }
    sum += bmax / hmin;
  }
  if (!(sum > 0)) return fail(VFP_EINVAL, "no advection: the CFL step is unbounded");
  *dt = courant / sum;
  return VFP_OK;
}

// c_s dt of stage s (Horner form, c = 1/4, 1/3, 1/2, 1), rounded the same way
// by every caller so that all stepping paths agree bit for bit.
static double stage_cdt(int s, double dt) {
  switch (s) {
    case 0: return 0.25 * dt;
    case 1: return dt / 3.0;
    case 2: return 0.5 * dt;
    default: return dt;
  }
}

static bool overlaps(const double* a, int64_t na, const double* b, int64_t nb) {
  if (!a || !b) return false;
  return a < b + nb && b < a + na;
}

static int launch(vfp_ctx* c, const double* w_in, const double* u, double* w_out, double alpha, double beta,
                  int with_source, void* stream) {
  KernelArgs a{};
  a.mesh = c->meshargs;
  a.fld = c->fld;
  a.tab = c->tab;
  a.st.w_in = w_in;
  a.st.u = u;
  a.st.w_out = w_out;
  a.st.alpha = alpha;
  a.st.beta = beta;
  a.st.with_source = with_source && (c->terms & VFP_TERM_SOURCE);
  a.tile_map = c->tile_map;
  c->launcher(a, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int vfp_autotune(vfp_ctx* c, const double* u, double* work, int reps, int* chosen, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u || !work) return fail(VFP_EINVAL, "null state pointer");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(u, N, work, N)) return fail(VFP_EINVAL, "work overlaps u");
  if (reps < 1) reps = 3;
  if (c->shock && !c->linp) {
    // one temporary vector, so that the later stages' form (reads w_in and
    // u, writes a third vector) is timed without touching u
    DevBuf tmp;
    if (std::getenv("VFP_FAIL_ALLOC")) return fail(VFP_ENOMEM, "allocation refused (VFP_FAIL_ALLOC)");
    if (hipMalloc(&tmp.p, (size_t)N * sizeof(double)) != hipSuccess) {
      tmp.p = nullptr;
      return fail(VFP_ENOMEM, "hipMalloc(%lld doubles)", (long long)N);
    }
    double* t3 = tmp.as<double>();
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(VFP_EDEVICE, "hipEventCreate");
    }
    struct Cand {
      int shape, tm;
      StageLauncher L;
      float best;
    };
    std::vector<Cand> cand;
    for (int shape = 0; shape < kShockShapes; ++shape) {
      StageLauncher L = shape ? find_shock_launcher_shape(c->k, c->lmax, c->tab.nrot, shape)
                              : find_shock_launcher(c->k, c->lmax, c->tab.nrot, false);
      if (L)
        for (int tm : {0, 1}) cand.push_back({shape, tm, L, 1e30f});
    }
    const int bs0 = c->shape, bt0 = c->tile_map;
    int rc = VFP_OK;
    // Each candidate runs what a Runge-Kutta step runs: one stage of the
    // first form (reads u, writes work) and three of the later form (reads
    // work and u, writes the temporary), reps times; two rounds over the
    // candidates, keeping each one's faster round (clocks and neighbours
    // drift within a round)
    for (int round = 0; round < 2 && rc == VFP_OK; ++round)
      for (Cand& cd : cand) {
        c->launcher = cd.L;
        c->tile_map = cd.tm;
        if ((rc = launch(c, u, u, work, 1.0, 1e-3, 1, stream))) break;
        if ((rc = launch(c, work, u, t3, 1.0, 1e-3, 1, stream))) break;
        if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) { rc = fail(VFP_EDEVICE, "event"); break; }
        for (int i = 0; i < reps && rc == VFP_OK; ++i) {
          rc = launch(c, u, u, work, 1.0, 1e-3, 1, stream);
          for (int st = 0; st < 3 && rc == VFP_OK; ++st) rc = launch(c, work, u, t3, 1.0, 1e-3, 1, stream);
        }
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, (hipStream_t)stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(VFP_EDEVICE, "timing events");
          break;
        }
        cd.best = std::min(cd.best, ms);
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int bs = bs0, bt = bt0;
    if (rc == VFP_OK && !cand.empty()) {
      const Cand* b = &cand[0];
      for (const Cand& cd : cand)
        if (cd.best < b->best) b = &cd;
      bs = b->shape;
      bt = b->tm;
    }
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));   // tmp is freed on return
    c->shape = bs;
    c->tile_map = bt;
    c->launcher = bs ? find_shock_launcher_shape(c->k, c->lmax, c->tab.nrot, bs)
                     : find_shock_launcher(c->k, c->lmax, c->tab.nrot, false);
    if (rc) return rc;
  }
  if (chosen) {
    chosen[0] = c->shock ? c->shape : 0;
    chosen[1] = c->shock ? shock_shape_threads(c->lmax, c->shape) : stage_threads_general();
    chosen[2] = c->shock ? c->tile_map : 0;
  }
  return VFP_OK;
}

int vfp_apply(vfp_ctx* c, const double* in, double* out, int with_source, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!in || !out) return fail(VFP_EINVAL, "null state pointer");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(in, N, out, N)) return fail(VFP_EINVAL, "in and out must not overlap");
  return launch(c, in, nullptr, out, 0.0, 1.0, with_source, stream);
}

int vfp_stage(vfp_ctx* c, const double* w_in, const double* u, double* w_out, double cdt, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!w_in || !u || !w_out) return fail(VFP_EINVAL, "null state pointer");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(w_out, N, w_in, N)) return fail(VFP_EINVAL, "w_out must not overlap w_in");
  if (overlaps(w_out, N, u, N) && w_out != u) return fail(VFP_EINVAL, "w_out partially overlaps u");
  if (!std::isfinite(cdt)) return fail(VFP_EINVAL, "cdt not finite");
  return launch(c, w_in, u, w_out, 1.0, cdt, 1, stream);
}

// Opt-in guard (VFP_CHECK_FINITE=1 in the environment): after a compute call
// that advances the state, check it for NaN / Inf on the device and report
// VFP_EDEVICE; synchronises the stream.  Off, it costs one getenv.
static int check_finite(vfp_ctx* c, const double* u, int64_t N, void* stream, const char* who) {
  const char* ev = std::getenv("VFP_CHECK_FINITE");
  if (!(ev && std::atoi(ev) != 0)) return VFP_OK;
  hipStream_t st = (hipStream_t)stream;
  int* flag = c->d_flag.as<int>();
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  kry_nonfinite(u, N, flag, st);
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h) return fail(VFP_EDEVICE, "%s: the state holds NaN or Inf values (VFP_CHECK_FINITE)", who);
  return VFP_OK;
}

int vfp_advance(vfp_ctx* c, double* u, double dt, int64_t nsteps, double* work, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u || !work) return fail(VFP_EINVAL, "null state pointer");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  double* wa = work;
  double* wb = work + N;
  if ((u >= work && u < work + 2 * N) || (work >= u && work < u + N))
    return fail(VFP_EINVAL, "work overlaps u");
  if (c->resident) {
    if (nsteps == 0) return VFP_OK;
    KernelArgs a{};
    a.mesh = c->meshargs;
    a.fld = c->fld;
    a.tab = c->tab;
    a.st.with_source = (c->terms & VFP_TERM_SOURCE) ? 1 : 0;
    c->resident(a, dt, (long long)nsteps, u, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return check_finite(c, u, N, stream, "vfp_advance");
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    if (int e = launch(c, u, u, wa, 1.0, stage_cdt(0, dt), 1, stream)) return e;
    if (int e = launch(c, wa, u, wb, 1.0, stage_cdt(1, dt), 1, stream)) return e;
    if (int e = launch(c, wb, u, wa, 1.0, stage_cdt(2, dt), 1, stream)) return e;
    if (int e = launch(c, wa, u, u, 1.0, stage_cdt(3, dt), 1, stream)) return e;
  }
  return check_finite(c, u, N, stream, "vfp_advance");
}

static int launch_adj(vfp_ctx* c, const double* mu_in, const double* acc_in, double* acc_out, double alpha,
                      double beta, double* t_out, const double* fwd, double* grad_nu, int mass_out,
                      void* stream, const double* add_in = nullptr) {
  if (!c->adj_launcher) return fail(VFP_EUNSUPPORTED, "no adjoint kernel for this configuration");
  KernelArgs a{};
  a.mesh = c->meshargs;
  a.fld = c->fld;
  a.tab = c->tab;
  a.st.w_in = mu_in;
  a.st.u = acc_in;
  a.st.w_out = acc_out;
  a.st.alpha = alpha;
  a.st.beta = beta;
  a.st.with_source = 0;
  a.adj.t_out = t_out;
  a.adj.fwd = fwd;
  a.adj.grad_nu = grad_nu;
  a.adj.mass_out = mass_out;
  a.adj.add_in = add_in;
  a.tile_map = c->tile_map;
  c->adj_launcher(a, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

static int launch_mass(vfp_ctx* c, const double* in, double* out, bool inv, void* stream) {
  if (!c->mass_launcher) return fail(VFP_EUNSUPPORTED, "no mass kernel for this configuration");
  c->mass_launcher(c->meshargs, c->n, in, out, inv, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int vfp_mass(vfp_ctx* c, const double* in, double* out, int inverse, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!in || !out) return fail(VFP_EINVAL, "null state pointer");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(in, N, out, N) && in != out) return fail(VFP_EINVAL, "out partially overlaps in");
  return launch_mass(c, in, out, inverse != 0, stream);
}

int vfp_apply_adjoint(vfp_ctx* c, const double* in, double* out, double* work, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!in || !out || !work) return fail(VFP_EINVAL, "null pointer (in, out and work are required)");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(in, N, out, N)) return fail(VFP_EINVAL, "in and out must not overlap");
  if (overlaps(work, N, in, N) || overlaps(work, N, out, N))
    return fail(VFP_EINVAL, "work must be disjoint from in and out");
  // work receives mu = M^{-1} in; the adjoint kernel then forms -D^T mu with
  // the mass multiply fused (M K M^{-1} = -D^T M^{-1})
  if (int e = launch_mass(c, in, work, true, stream)) return e;
  return launch_adj(c, work, nullptr, out, 0.0, 1.0, nullptr, nullptr, nullptr, 1, stream);
}

int vfp_adjoint_stage(vfp_ctx* c, const double* mu_in, const double* acc_in, const double* fwd, double cdt,
                      double* t_out, double* acc_out, double* grad_nu, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!mu_in || !acc_in || !acc_out) return fail(VFP_EINVAL, "null state pointer");
  if (!std::isfinite(cdt)) return fail(VFP_EINVAL, "cdt not finite");
  if (grad_nu && !fwd) return fail(VFP_EINVAL, "grad_nu needs the forward stage input fwd");
  if (grad_nu && c->have_nu_pts) return fail(VFP_EUNSUPPORTED, "dJ/dnu per cell with nu given at the points");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(acc_out, N, mu_in, N) || overlaps(t_out, N, mu_in, N) || overlaps(t_out, N, acc_in, N) ||
      overlaps(t_out, N, acc_out, N))
    return fail(VFP_EINVAL, "t_out / acc_out alias an input that other cells read");
  if (overlaps(acc_out, N, acc_in, N) && acc_out != acc_in)
    return fail(VFP_EINVAL, "acc_out partially overlaps acc_in");
  if (grad_nu && (overlaps(grad_nu, c->ncells, acc_out, N) || overlaps(grad_nu, c->ncells, t_out, N)))
    return fail(VFP_EINVAL, "grad_nu overlaps an output");
  return launch_adj(c, mu_in, acc_in, acc_out, 1.0, cdt, t_out, grad_nu ? fwd : nullptr, grad_nu, 0, stream);
}

int vfp_advance_tape(vfp_ctx* c, const double* u0, double dt, int64_t nsteps, double* tape, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u0 || !tape) return fail(VFP_EINVAL, "null state pointer");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(u0, N, tape, 4 * nsteps * N)) return fail(VFP_EINVAL, "tape overlaps u0");
  for (int64_t s = 0; s < nsteps; ++s) {
    const double* un = s == 0 ? u0 : tape + (4 * s - 1) * N;
    double* w = tape + 4 * s * N;
    if (int e = launch(c, un, un, w, 1.0, stage_cdt(0, dt), 1, stream)) return e;
    if (int e = launch(c, w, un, w + N, 1.0, stage_cdt(1, dt), 1, stream)) return e;
    if (int e = launch(c, w + N, un, w + 2 * N, 1.0, stage_cdt(2, dt), 1, stream)) return e;
    if (int e = launch(c, w + 2 * N, un, w + 3 * N, 1.0, stage_cdt(3, dt), 1, stream)) return e;
  }
  return VFP_OK;
}

static int field_grad_ready(const vfp_ctx* c) {
  if (!(c->naxes == 2 && c->mom && !c->linp && c->planar))
    return fail(VFP_EUNSUPPORTED, "field gradients need an (x, ln p) context with a planar flow");
  return VFP_OK;
}

// Builds the p-face derivative tables on the first field-gradient call (a
// host computation and an upload); later set-up calls keep them current.
static int ensure_pf_dk(vfp_ctx* c) {
  if (c->pf_dk) return VFP_OK;
  c->pf_dk = true;
  if (int e = build_pface_data(c, true)) {
    c->pf_dk = false;
    return e;
  }
  c->fld.pf_dtab = c->d_pf_dtab.as<double>();
  return VFP_OK;
}

static int launch_fg(vfp_ctx* c, const double* mu, const double* fwd, double cdt, double* slots, double* grad_nu,
                     void* stream) {
  FieldGradLauncher fl = find_field_grad_launcher(c->k, c->lmax);
  if (!fl) return fail(VFP_EUNSUPPORTED, "no field-gradient kernel for k=%d lmax=%d", c->k, c->lmax);
  if (int e = ensure_pf_dk(c)) return e;
  KernelArgs a{};
  a.mesh = c->meshargs;
  a.fld = c->fld;
  a.tab = c->tab;
  const bool listed = c->d_fg_support.as<unsigned char>() != nullptr;
  fl(a, mu, fwd, cdt, slots, c->d_fg_support.as<unsigned char>(), listed ? c->d_fg_blocks.as<int>() : nullptr,
     listed ? c->fg_nblocks : 0, grad_nu, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int vfp_field_grad_support(vfp_ctx* c, const unsigned char* xcells) {
  if (!c) return fail(VFP_EINVAL, "null context");
  ++c->gen;
  if (int e = check_ready(c)) return e;
  if (int e = field_grad_ready(c)) return e;
  if (int e = ensure_pf_dk(c)) return e;
  c->d_fg_blocks.release();
  c->fg_nblocks = 0;
  if (!xcells) {
    c->d_fg_support.release();
    return VFP_OK;
  }
  std::vector<unsigned char> m(xcells, xcells + c->ncell[0]);
  for (auto& v : m) v = v ? 1 : 0;
  // the tiles (runs of consecutive cells) that hold at least one support cell
  const int tc = field_grad_tile_cells(c->lmax), nt = field_grad_tiles((int)c->ncells, c->lmax);
  std::vector<int> blocks;
  for (int t = 0; t < nt; ++t)
    for (int j = 0; j < tc; ++j) {
      const int64_t cell = (int64_t)t * tc + j;
      if (cell < c->ncells && m[cell % c->ncell[0]]) {
        blocks.push_back(t);
        break;
      }
    }
  if (!blocks.empty())
    if (int e = upload_vec(c->d_fg_blocks, blocks)) return e;
  c->fg_nblocks = (int)blocks.size();
  return upload_vec(c->d_fg_support, m);
}

int vfp_field_grad_size(const vfp_ctx* c, int64_t* n) {
  if (int e = check_ready(c)) return e;
  if (!n) return fail(VFP_EINVAL, "null argument");
  if (int e = field_grad_ready(c)) return e;
  *n = (int64_t)c->ncells * field_grad_slots_per_cell(c->k);
  return VFP_OK;
}

int vfp_field_grad_stage(vfp_ctx* c, const double* mu, const double* fwd, double cdt, double* slots,
                         void* stream) {
  if (int e = check_ready(c)) return e;
  if (int e = field_grad_ready(c)) return e;
  if (!mu || !fwd || !slots) return fail(VFP_EINVAL, "null pointer");
  if (!std::isfinite(cdt)) return fail(VFP_EINVAL, "cdt not finite");
  int64_t N = 0, ns = 0;
  vfp_ndofs(c, &N);
  vfp_field_grad_size(c, &ns);
  if (overlaps(slots, ns, mu, N) || overlaps(slots, ns, fwd, N)) return fail(VFP_EINVAL, "slots overlap an input");
  return launch_fg(c, mu, fwd, cdt, slots, nullptr, stream);
}

int vfp_field_grad_reduce(vfp_ctx* c, const double* slots, double* g_u, double* g_dudx, double* g_dudt,
                          double* g_uface, void* stream) {
  if (int e = check_ready(c)) return e;
  if (int e = field_grad_ready(c)) return e;
  if (!slots || !g_u || !g_dudx || !g_dudt || !g_uface) return fail(VFP_EINVAL, "null pointer");
  FieldGradReduce fr = find_field_grad_reduce(c->k);
  if (!fr) return fail(VFP_EUNSUPPORTED, "k=%d", c->k);
  fr(c->meshargs, slots, g_u, g_dudx, g_dudt, g_uface, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int vfp_adjoint_steps(vfp_ctx* c, const double* u0, const double* tape, double dt, int64_t nsteps, double* mu,
                      double* grad_nu, double* field_slots, double* work, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u0 || !tape || !mu || !work) return fail(VFP_EINVAL, "null state pointer");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  if (overlaps(work, 3 * N, mu, N) || overlaps(work, 3 * N, tape, 4 * nsteps * N) || overlaps(work, 3 * N, u0, N) ||
      overlaps(mu, N, tape, 4 * nsteps * N) || overlaps(mu, N, u0, N))
    return fail(VFP_EINVAL, "work / mu overlap the tape or each other");
  if (grad_nu && (overlaps(grad_nu, c->ncells, work, 3 * N) || overlaps(grad_nu, c->ncells, mu, N)))
    return fail(VFP_EINVAL, "grad_nu overlaps a state buffer");
  if (grad_nu && c->have_nu_pts) return fail(VFP_EUNSUPPORTED, "dJ/dnu per cell with nu given at the points");
  if (field_slots) {
    if (int e = field_grad_ready(c)) return e;
    int64_t ns = 0;
    vfp_field_grad_size(c, &ns);
    if (overlaps(field_slots, ns, work, 3 * N) || overlaps(field_slots, ns, mu, N) ||
        overlaps(field_slots, ns, tape, 4 * nsteps * N) || overlaps(field_slots, ns, grad_nu, c->ncells))
      return fail(VFP_EINVAL, "field_slots overlap another buffer");
  }
  double* acc = work;
  double* b1 = work + N;
  double* b2 = work + 2 * N;
  // with the flow sensitivities the dJ/dnu term rides on their launch, which
  // reads the same (adjoint, forward) pair anyway; the adjoint stages then
  // do not read the forward state at all
  double* gnu_fg = field_slots ? grad_nu : nullptr;
  double* gnu_adj = field_slots ? nullptr : grad_nu;
  // each flow-sensitivity launch pairs an adjoint stage input with its
  // forward stage input, before the adjoint stage may overwrite it
  auto stage = [&](const double* m_in, const double* a_in, double* a_out, double* t_out, const double* fw,
                   const double* f_nu, double cdt, double alpha, const double* add_in) -> int {
    if (field_slots)
      if (int e = launch_fg(c, m_in, fw, cdt, field_slots, gnu_fg, stream)) return e;
    return launch_adj(c, m_in, a_in, a_out, alpha, cdt, t_out, f_nu, gnu_adj, 0, stream, add_in);
  };
  // The running sum acc = lambda + t_4 + t_3 + ... starts one stage late
  // where the kernel can add a state to its output: the last stage writes
  // only t_4, and the next one forms lambda + t_4 + t_3 from lambda, its own
  // input t_4 and its result (8 bytes per DoF less than writing lambda + t_4
  // and reading it back).
  const bool late = c->adj_shock;
  for (int64_t s = nsteps - 1; s >= 0; --s) {
    const double* un = s == 0 ? u0 : tape + (4 * s - 1) * N;
    const double* w = tape + 4 * s * N;
    const double* f3 = gnu_adj ? w + 2 * N : nullptr;
    const double* f2 = gnu_adj ? w + N : nullptr;
    const double* f1 = gnu_adj ? w : nullptr;
    const double* f0 = gnu_adj ? un : nullptr;
    if (late) {
      if (int e = stage(mu, nullptr, nullptr, b1, w + 2 * N, f3, stage_cdt(3, dt), 0.0, nullptr)) return e;
      if (int e = stage(b1, mu, acc, b2, w + N, f2, stage_cdt(2, dt), 1.0, b1)) return e;
    } else {
      if (int e = stage(mu, mu, acc, b1, w + 2 * N, f3, stage_cdt(3, dt), 1.0, nullptr)) return e;
      if (int e = stage(b1, acc, acc, b2, w + N, f2, stage_cdt(2, dt), 1.0, nullptr)) return e;
    }
    if (int e = stage(b2, acc, acc, b1, w, f1, stage_cdt(1, dt), 1.0, nullptr)) return e;
    if (int e = stage(b1, acc, mu, nullptr, un, f0, stage_cdt(0, dt), 1.0, nullptr)) return e;
  }
  return VFP_OK;
}

int vfp_forward_checkpoints(vfp_ctx* c, double* u, double dt, int64_t nsteps, int64_t seg, double* ckpt,
                            double* work, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u || !ckpt || !work) return fail(VFP_EINVAL, "null state pointer");
  if (nsteps < 0 || seg < 1 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps / seg");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  const int64_t nseg = (nsteps + seg - 1) / seg;
  if (overlaps(ckpt, nseg * N, u, N) || overlaps(ckpt, nseg * N, work, 2 * N))
    return fail(VFP_EINVAL, "checkpoints overlap u or work");
  for (int64_t j = 0; j < nseg; ++j) {
    HIP_TRY(hipMemcpyAsync(ckpt + j * N, u, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    const int64_t cnt = std::min(seg, nsteps - j * seg);
    if (int e = vfp_advance(c, u, dt, cnt, work, stream)) return e;
  }
  return VFP_OK;
}

int vfp_adjoint_checkpointed(vfp_ctx* c, const double* ckpt, double dt, int64_t nsteps, int64_t seg,
                             double* tape, double* lam, double* grad_nu, double* field_slots, double* work,
                             void* stream) {
  if (int e = check_ready(c)) return e;
  if (!ckpt || !tape || !lam || !work) return fail(VFP_EINVAL, "null state pointer");
  if (nsteps < 0 || seg < 1 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps / seg");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  const int64_t nseg = (nsteps + seg - 1) / seg;
  const int64_t ntape = 4 * std::min(seg, nsteps) * N;
  if (overlaps(tape, ntape, ckpt, nseg * N) || overlaps(lam, N, ckpt, nseg * N) || overlaps(lam, N, tape, ntape) ||
      overlaps(work, 3 * N, tape, ntape) || overlaps(work, 3 * N, lam, N) || overlaps(work, 3 * N, ckpt, nseg * N))
    return fail(VFP_EINVAL, "checkpoint, tape, lam and work buffers must be disjoint");
  if (int e = launch_mass(c, lam, lam, true, stream)) return e;
  for (int64_t j = nseg - 1; j >= 0; --j) {
    const int64_t cnt = std::min(seg, nsteps - j * seg);
    const double* u0 = ckpt + j * N;
    if (int e = vfp_advance_tape(c, u0, dt, cnt, tape, stream)) return e;
    if (int e = vfp_adjoint_steps(c, u0, tape, dt, cnt, lam, grad_nu, field_slots, work, stream)) return e;
  }
  return launch_mass(c, lam, lam, false, stream);
}

}  // extern "C"

// ====================================================== Theta-method steps

namespace {

// Work layout (doubles): V [(m+1) N] Krylov basis, w [N], b [N] right-hand
// side, s [N] = M^{-1} h, z [N] preconditioned vector, partial
// [kKryMaxVectors kKryBlocks], dots [3 kKryMaxVectors].
struct ThetaWork {
  double *V, *w, *b, *s, *z, *partial, *d1, *d2, *d3;
};

int64_t theta_work_len(int64_t N, int m) {
  return (int64_t)(m + 5) * N + (int64_t)kKryMaxVectors * kKryBlocks + 3 * kKryMaxVectors;
}

ThetaWork theta_split(double* work, int64_t N, int m) {
  ThetaWork t;
  t.V = work;
  t.w = t.V + (int64_t)(m + 1) * N;
  t.b = t.w + N;
  t.s = t.b + N;
  t.z = t.s + N;
  t.partial = t.z + N;
  t.d1 = t.partial + (int64_t)kKryMaxVectors * kKryBlocks;
  t.d2 = t.d1 + kKryMaxVectors;
  t.d3 = t.d2 + kKryMaxVectors;
  return t;
}

// device -> host copy of n doubles (through the pinned buffer pin when
// there is one), then wait for the stream
int fetch(double* host, const double* dev, int n, hipStream_t st, double* pin = nullptr) {
  double* dst = pin ? pin : host;
  HIP_TRY(hipMemcpyAsync(dst, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (pin) std::memcpy(host, pin, n * sizeof(double));
  return VFP_OK;
}

// w = A x = x - dt Theta L0(x): the stage kernel with u = w_in = x
int theta_op(vfp_ctx* c, const double* x, double* w, double dt, double theta, void* stream) {
  return launch(c, x, x, w, 1.0, -dt * theta, 0, stream);
}

// One Theta step in place on u by restarted GMRES (iterate from u).
// it: Krylov iterations (accumulated); res: final true relative residual.
// The x-line preconditioner's blocks in the work tail (see xline.hip).
struct XLine {
  double *D = nullptr, *L = nullptr, *U = nullptr;
  int* fail = nullptr;
  int nx = 0, nlines = 0, b = 0, wrapc = 0;
  bool rowwise = false;   // VFP_XLINE_ROWS=1: the one-lane-per-row solve for every block size (tests)
};

XLine xline_layout(const vfp_ctx* c, double* tail) {
  XLine x;
  x.nx = c->ncell[0];
  x.nlines = c->ncells / x.nx;
  x.b = c->nb * c->n;
  x.wrapc = (c->bc_lo[0] == VFP_BC_PERIODIC && x.nx % 3 != 0) ? 1 : 0;
  const char* rw = std::getenv("VFP_XLINE_ROWS");
  x.rowwise = rw && std::atoi(rw) != 0;
  const int64_t blk = (int64_t)c->ncells * x.b * x.b;
  if (tail) {
    x.D = tail;
    x.L = tail + blk;
    x.U = tail + 2 * blk;
    x.fail = reinterpret_cast<int*>(tail + 3 * blk);
  }
  return x;
}

int64_t xline_len(const vfp_ctx* c) {
  const XLine x = xline_layout(c, nullptr);
  return 3 * (int64_t)c->ncells * x.b * x.b + (x.nlines + 1) / 2 + 1;
}

// Blocks of A = I - dt Theta L0 by probing (one colour and one local unknown
// at a time, into t.z, output in t.w), then the block factorisation per line.
int xline_build(vfp_ctx* c, const XLine& x, double dt, double theta, const ThetaWork& t, int64_t N, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int ncol = x.wrapc ? 4 : std::min(3, x.nx);
  // the coupling blocks stay zero where no neighbour exists
  HIP_TRY(hipMemsetAsync(x.L, 0, (size_t)c->ncells * x.b * x.b * sizeof(double), st));
  HIP_TRY(hipMemsetAsync(x.U, 0, (size_t)c->ncells * x.b * x.b * sizeof(double), st));
  for (int col = 0; col < ncol; ++col)
    for (int j = 0; j < x.b; ++j) {
      xl_probe_set(t.z, N, x.nx, x.b, x.wrapc, col, j, st);
      if (int e = theta_op(c, t.z, t.w, dt, theta, stream)) return e;
      xl_probe_get(t.w, x.D, x.L, x.U, N, x.nx, x.b, x.wrapc, col, j, st);
    }
  xl_factor(x.D, x.L, x.U, x.nlines, x.nx, x.b, x.fail, st);
  HIP_TRY(hipGetLastError());
  std::vector<int> fl(x.nlines);
  HIP_TRY(hipMemcpyAsync(fl.data(), x.fail, x.nlines * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int l = 0; l < x.nlines; ++l)
    if (fl[l]) return fail(VFP_EDEVICE, "x-line preconditioner: singular block on line %d", l);
  return VFP_OK;
}

int theta_step(vfp_ctx* c, double* u, double dt, const vfp_theta_opts& o, const ThetaWork& t, int64_t N,
               bool have_s, const XLine& xl, void* stream, int64_t& it, double& res, bool& conv) {
  hipStream_t st = (hipStream_t)stream;
  const int m = o.restart;
  const double th = o.theta;
  const bool pre = o.precond != VFP_PRECOND_NONE;
  const double sp = dt * th * ((c->terms & VFP_TERM_COLLISION) ? 1.0 : 0.0);
  auto precond = [&](double* out, const double* in) {
    if (o.precond == VFP_PRECOND_XLINE)
      xl_apply(in, out, xl.D, xl.L, xl.U, xl.nlines, xl.nx, xl.b, xl.rowwise, st);
    else
      kry_coll_precond(out, in, c->fld.nu_cell, c->fld.nu0, c->tab.c_val, sp, c->ncells, c->nb, c->n, st);
  };
  // right-hand side b = u + dt (1 - Theta) L(u) + dt Theta M^{-1} h
  if (th < 1.0) {
    if (int e = launch(c, u, u, t.b, 1.0, dt * (1.0 - th), 1, stream)) return e;
    if (have_s && th > 0.0) kry_lincomb(t.b, dt * th, t.s, 1.0, t.b, N, st);
  } else if (have_s) {
    kry_lincomb(t.b, 1.0, u, dt, t.s, N, st);
  } else {
    HIP_TRY(hipMemcpyAsync(t.b, u, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  conv = false;
  if (th == 0.0) {   // forward Euler: the system matrix is I
    HIP_TRY(hipMemcpyAsync(u, t.b, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipGetLastError());
    res = 0.0;
    conv = true;
    return VFP_OK;
  }
  double bn2 = 0.0;
  kry_mdot(t.b, N, 1, t.b, N, t.partial, t.d3, st);
  if (int e = fetch(&bn2, t.d3, 1, st, c->h_kry.p)) return e;
  const double bn = std::sqrt(bn2);
  if (bn == 0.0) {
    kry_lincomb(u, 0.0, u, 0.0, nullptr, N, st);
    HIP_TRY(hipGetLastError());
    res = 0.0;
    conv = true;
    return VFP_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), g(m + 1), cs(m), sn(m), y(m), hb(3 * kKryMaxVectors);
  int64_t used = 0;
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { (void)hipEventDestroy(e); }
  } ev_guard{ev};
  for (;;) {
    // true residual r = b - A u into V_0
    if (int e = theta_op(c, u, t.w, dt, th, stream)) return e;
    kry_lincomb(t.V, 1.0, t.b, -1.0, t.w, N, st);
    kry_mdot(t.V, N, 1, t.V, N, t.partial, t.d3, st);
    double rn2 = 0.0;
    if (int e = fetch(&rn2, t.d3, 1, st, c->h_kry.p)) return e;
    const double beta = std::sqrt(rn2);
    res = beta / bn;
    if (!std::isfinite(res)) return fail(VFP_EDEVICE, "non-finite residual in the Theta step");
    if (res <= o.tol) {
      conv = true;
      break;
    }
    if (used >= o.max_iters) break;
    kry_lincomb(t.V, 1.0 / beta, t.V, 0.0, nullptr, N, st);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    // w = A P^{-1} V_j, orthogonalised against V_0..V_j by classical
    // Gram-Schmidt; a second pass only where the first removed most of w
    // (the criterion of Daniel, Gragg, Kaufman and Stewart:
    // |w_new| < |w_old| / sqrt 2).  The decision, the second pass and the
    // normalisation V_{j+1} = w / |w| run on the device (d3[4] the decision,
    // d3[3] = |w|), so that iteration j + 1's launches can be queued before
    // the host has read iteration j's Hessenberg column: the host's round
    // trip then overlaps the next iteration's kernels.  Where the column
    // shows convergence, that queued iteration's results are not used.
    auto front = [&](int jj) -> int {
      const double* vin = t.V + (int64_t)jj * N;
      if (pre) {
        precond(t.z, vin);
        vin = t.z;
      }
      if (int e = theta_op(c, vin, t.w, dt, th, stream)) return e;
      // d1[0..jj] = V^T w and d1[jj+1] = |w|^2 in one pass over w; the
      // update leaves |w_new|^2 in d3[1]
      kry_mdot(t.V, N, jj + 1, t.w, N, t.partial, t.d1, st, true);
      kry_maxpy(t.w, t.V, N, jj + 1, t.d1, -1.0, N, st, t.partial, t.d3 + 1);
      return VFP_OK;
    };
    if (int e = front(0)) return e;
    bool queued = true;   // front(j) is in the stream
    while (j < m && used < o.max_iters) {
      if (!queued)
        if (int e = front(j)) return e;
      kry_decide(t.d1, j, t.d3, st);
      kry_mdot(t.V, N, j + 1, t.w, N, t.partial, t.d2, st, false, t.d3 + 4);
      kry_maxpy(t.w, t.V, N, j + 1, t.d2, -1.0, N, st, t.partial, t.d3 + 2, t.d3 + 4);
      kry_norm_scale(j + 1 < m ? t.V + (int64_t)(j + 1) * N : nullptr, t.w, N, t.d3, st);
      HIP_TRY(hipMemcpyAsync(c->h_kry.p, t.d1, 3 * kKryMaxVectors * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipEventRecord(ev, st));
      // queue the next iteration unless the residual estimate so far is
      // within a factor 100 of the tolerance (then this one may well be the
      // last, and a queued iteration would be wasted work)
      queued = j + 1 < m && used + 1 < o.max_iters && std::fabs(g[j]) > 100.0 * o.tol * bn;
      if (queued)
        if (int e = front(j + 1)) return e;
      HIP_TRY(hipEventSynchronize(ev));
      std::memcpy(hb.data(), c->h_kry.p, 3 * kKryMaxVectors * sizeof(double));
      const bool second = hb[2 * kKryMaxVectors + 4] != 0.0;
      for (int i = 0; i <= j; ++i)
        H[(size_t)i * m + j] = second ? hb[i] + hb[kKryMaxVectors + i] : hb[i];
      const double hn = hb[2 * kKryMaxVectors + 3];
      H[(size_t)(j + 1) * m + j] = hn;
      ++used;
      // previous Givens rotations, then the one that removes H[j+1][j]
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
      const double rr = std::hypot(a, b);
      cs[j] = rr == 0.0 ? 1.0 : a / rr;
      sn[j] = rr == 0.0 ? 0.0 : b / rr;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++j;
      if (std::fabs(g[j]) <= o.tol * bn || hn == 0.0) break;
    }
    // y = H^{-1} g (upper triangular), u += V y
    for (int i = j - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < j; ++l) acc -= H[(size_t)i * m + l] * y[l];
      const double d = H[(size_t)i * m + i];
      y[i] = d != 0.0 ? acc / d : 0.0;
    }
    HIP_TRY(hipMemcpyAsync(t.d1, y.data(), j * sizeof(double), hipMemcpyHostToDevice, st));
    if (pre) {
      // u += P^{-1} V y (z is cleared from V_0, which is finite: z may hold
      // the unused results of a queued iteration)
      kry_lincomb(t.z, 0.0, t.V, 0.0, nullptr, N, st);
      kry_maxpy(t.z, t.V, N, j, t.d1, 1.0, N, st);
      precond(t.z, t.z);
      kry_lincomb(u, 1.0, u, 1.0, t.z, N, st);
    } else {
      kry_maxpy(u, t.V, N, j, t.d1, 1.0, N, st);
    }
    HIP_TRY(hipGetLastError());
  }
  it += used;
  return VFP_OK;
}

}  // namespace

extern "C" {

int vfp_sh_eval(int lmax, int64_t ndir, const double* theta, const double* phi, double* Y) {
  if (lmax < 0 || lmax > kMaxLmax) return fail(VFP_EINVAL, "lmax must be in 0..%d", kMaxLmax);
  if (ndir < 0 || (ndir > 0 && (!theta || !phi || !Y))) return fail(VFP_EINVAL, "bad direction arrays");
  const int n = (lmax + 1) * (lmax + 1);
  for (int64_t d = 0; d < ndir; ++d) real_sh_dir(lmax, theta[d], phi[d], Y + d * n);
  return VFP_OK;
}

int vfp_reconstruct(const vfp_ctx* c, const double* zeta, const double* Y, int64_t ndir, double* out,
                    void* stream) {
  if (!c || !c->mesh_set) return fail(VFP_ESTATE, "context without a mesh");
  if (!zeta || !Y || !out) return fail(VFP_EINVAL, "null pointer");
  if (ndir < 1) return fail(VFP_EINVAL, "ndir must be >= 1");
  const int n = c->n;
  if (n > reconstruct_max_lms()) return fail(VFP_EUNSUPPORTED, "lmax too large for vfp_reconstruct");
  int64_t N = 0;
  vfp_ndofs(c, &N);
  const int64_t rows = N / n;
  if ((ndir + 63) / 64 > 65535) return fail(VFP_EINVAL, "ndir too large");
  if (overlaps(zeta, N, out, rows * ndir)) return fail(VFP_EINVAL, "out overlaps zeta");
  if (overlaps(Y, ndir * n, out, rows * ndir)) return fail(VFP_EINVAL, "out overlaps Y");
  launch_reconstruct(zeta, rows, n, Y, ndir, out, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int vfp_theta_work_size(const vfp_ctx* c, int restart, int64_t* n) {
  if (!c || !n) return fail(VFP_EINVAL, "null argument");
  if (restart < 1 || restart > 64) return fail(VFP_EINVAL, "restart must be in 1..64");
  int64_t N = 0;
  if (int e = vfp_ndofs(c, &N)) return e;
  *n = theta_work_len(N, restart);
  return VFP_OK;
}

int vfp_theta_precond_size(const vfp_ctx* c, int precond, int64_t* n) {
  if (int e = check_ready(c)) return e;
  if (!n) return fail(VFP_EINVAL, "null argument");
  *n = 0;
  if (precond == VFP_PRECOND_XLINE) {
    const int b = c->nb * c->n;
    if (b > kXlMaxBlock)
      return fail(VFP_EUNSUPPORTED, "x-line preconditioner: %d unknowns per cell (at most %d)", b, kXlMaxBlock);
    *n = xline_len(c);
  } else if (precond != VFP_PRECOND_NONE && precond != VFP_PRECOND_COLLISION) {
    return fail(VFP_EINVAL, "precond %d unknown", precond);
  }
  return VFP_OK;
}

int vfp_theta_advance(vfp_ctx* c, double* u, double dt, int64_t nsteps, const vfp_theta_opts* o, double* work,
                      int64_t work_len, vfp_theta_stats* stats, void* stream) {
  if (int e = check_ready(c)) return e;
  if (!u || !work || !o) return fail(VFP_EINVAL, "null argument");
  if (!(o->theta >= 0.0 && o->theta <= 1.0)) return fail(VFP_EINVAL, "theta must be in [0, 1]");
  if (!(o->tol > 0.0)) return fail(VFP_EINVAL, "tol must be positive");
  if (o->restart < 1 || o->restart > 64) return fail(VFP_EINVAL, "restart must be in 1..64");
  if (o->max_iters < 1) return fail(VFP_EINVAL, "max_iters must be >= 1");
  if (o->precond == VFP_PRECOND_COLLISION && c->have_nu_pts)
    return fail(VFP_EUNSUPPORTED, "the collision preconditioner needs nu per cell (not at the points)");
  if (o->precond != VFP_PRECOND_NONE && o->precond != VFP_PRECOND_COLLISION && o->precond != VFP_PRECOND_XLINE)
    return fail(VFP_EINVAL, "precond %d unknown", o->precond);
  if (nsteps < 0 || !std::isfinite(dt)) return fail(VFP_EINVAL, "bad dt / nsteps");
  int64_t pc_len = 0;
  if (int e = vfp_theta_precond_size(c, o->precond, &pc_len)) return e;
  int64_t N = 0;
  vfp_ndofs(c, &N);
  const int64_t need = theta_work_len(N, o->restart) + pc_len;
  if (work_len < need) return fail(VFP_EINVAL, "work holds %lld doubles, %lld needed", (long long)work_len,
                                   (long long)need);
  if (overlaps(u, N, work, need)) return fail(VFP_EINVAL, "work overlaps u");
  const ThetaWork t = theta_split(work, N, o->restart);
  XLine xl;
  if (o->precond == VFP_PRECOND_XLINE && nsteps > 0 && o->theta > 0.0) {
    xl = xline_layout(c, work + theta_work_len(N, o->restart));
    if (int e = xline_build(c, xl, dt, o->theta, t, N, stream)) return e;
  }
  hipStream_t st = (hipStream_t)stream;
  if (!c->h_kry.p && hipHostMalloc((void**)&c->h_kry.p, 3 * kKryMaxVectors * sizeof(double), hipHostMallocDefault) !=
                         hipSuccess) {
    c->h_kry.p = nullptr;      // read-backs go to pageable memory instead
    (void)hipGetLastError();
  }
  const bool have_s = (c->terms & VFP_TERM_SOURCE) && c->have_src && o->theta > 0.0;
  if (have_s) {
    // s = M^{-1} h = L(0)
    HIP_TRY(hipMemsetAsync(t.w, 0, N * sizeof(double), st));
    if (int e = launch(c, t.w, nullptr, t.s, 0.0, 1.0, 1, stream)) return e;
  }
  int64_t it = 0;
  double worst = 0.0;
  bool all = true;
  for (int64_t n = 0; n < nsteps; ++n) {
    double res = 0.0;
    bool conv = false;
    if (int e = theta_step(c, u, dt, *o, t, N, have_s, xl, stream, it, res, conv)) return e;
    worst = std::max(worst, res);
    all = all && conv;
  }
  if (stats) {
    stats->iterations = it;
    stats->residual = worst;
    stats->converged = all ? 1 : 0;
  }
  return check_finite(c, u, N, stream, "vfp_theta_advance");
}

}  // extern "C"

// ================================================================= batches

struct vfp_batch {
  struct Class {
    int k = 0, lmax = 0, nrot = 0;
    bool batched = false;              // one launch per stage for all members
    std::vector<int> members;
    BatchKernel bk;
    DevBuf descs;                      // [stage][member] KernelArgs
    DevBuf start;                      // members + 1 tile offsets
    DevBuf tile_run;                   // run (member index) of every tile
    int total = 0;                     // tiles = workgroups per launch
    int tile_map = 0;                  // tuned
    int shape = 0;                     // tuned workgroup shape slot
  };
  std::vector<vfp_ctx*> runs;
  std::vector<Class> classes;
  std::vector<double*> u, work;
  std::vector<double> dt;
  std::vector<uint64_t> gen;           // each run's set-up generation at vfp_batch_bind
  bool bound = false;
  bool use_graph = false;
  int device = -1;
  hipStream_t stream = nullptr;        // private stream (default priority) for graphs
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // capture: one branch per class (classes share no run, so their stages may
  // run concurrently); streams and events of the fork / join
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~vfp_batch() {
    drop_graph();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (fork) (void)hipEventDestroy(fork);
    for (auto e : joins) (void)hipEventDestroy(e);
    for (auto st : branch) (void)hipStreamDestroy(st);
    if (stream) (void)hipStreamDestroy(stream);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

namespace {

// Stage s of a step (Horner form): (w_in, w_out, c_s dt) with u the step base.
void stage_ptrs(int s, double* u, double* work, int64_t N, double dt, const double*& w_in, double*& w_out,
                double& cdt) {
  double* wa = work;
  double* wb = work + N;
  cdt = stage_cdt(s, dt);
  switch (s) {
    case 0: w_in = u; w_out = wa; break;
    case 1: w_in = wa; w_out = wb; break;
    case 2: w_in = wb; w_out = wa; break;
    default: w_in = wa; w_out = u; break;
  }
}

KernelArgs stage_args(vfp_ctx* c, const double* w_in, const double* u, double* w_out, double beta) {
  KernelArgs a{};
  a.mesh = c->meshargs;
  a.fld = c->fld;
  a.tab = c->tab;
  a.st.w_in = w_in;
  a.st.u = u;
  a.st.w_out = w_out;
  a.st.alpha = 1.0;
  a.st.beta = beta;
  a.st.with_source = (c->terms & VFP_TERM_SOURCE) ? 1 : 0;
  a.tile_map = c->tile_map;
  return a;
}

int batch_launch_stage(vfp_batch* b, vfp_batch::Class& cl, int s, hipStream_t st) {
  if (cl.batched) {
    BatchArgs ba;
    ba.descs = cl.descs.as<KernelArgs>() + (size_t)s * cl.members.size();
    ba.start = cl.start.as<int>();
    ba.tile_run = cl.tile_run.as<int>();
    ba.nruns = (int)cl.members.size();
    ba.total = cl.total;
    ba.tile_map = cl.tile_map;
    cl.bk.launch(ba, st);
  } else {
    for (int r : cl.members) {
      vfp_ctx* c = b->runs[r];
      int64_t N = 0;
      vfp_ndofs(c, &N);
      const double* w_in;
      double* w_out;
      double cdt;
      stage_ptrs(s, b->u[r], b->work[r], N, b->dt[r], w_in, w_out, cdt);
      KernelArgs a = stage_args(c, w_in, b->u[r], w_out, cdt);
      c->launcher(a, st);
    }
  }
  HIP_TRY(hipGetLastError());
  return VFP_OK;
}

int batch_step(vfp_batch* b, hipStream_t st) {
  for (int s = 0; s < 4; ++s)
    for (auto& cl : b->classes)
      if (int e = batch_launch_stage(b, cl, s, st)) return e;
  return VFP_OK;
}

// One step captured as a fork / join: class i's four stages on branch i.
int batch_step_branched(vfp_batch* b, hipStream_t st) {
  HIP_TRY(hipEventRecord(b->fork, st));
  for (size_t i = 0; i < b->classes.size(); ++i) {
    HIP_TRY(hipStreamWaitEvent(b->branch[i], b->fork, 0));
    for (int s = 0; s < 4; ++s)
      if (int e = batch_launch_stage(b, b->classes[i], s, b->branch[i])) return e;
    HIP_TRY(hipEventRecord(b->joins[i], b->branch[i]));
    HIP_TRY(hipStreamWaitEvent(st, b->joins[i], 0));
  }
  return VFP_OK;
}

// Tile tables of a batched class for its current kernel (cells per tile):
// the first tile of every member and the member of every tile.
int class_tiles(vfp_batch* b, vfp_batch::Class& cl) {
  std::vector<int> st(cl.members.size() + 1, 0);
  long long tot = 0;
  for (size_t j = 0; j < cl.members.size(); ++j) {
    st[j] = (int)tot;
    tot += (b->runs[cl.members[j]]->ncells + cl.bk.cells_per_tile - 1) / cl.bk.cells_per_tile;
    if (tot > (1LL << 30)) return fail(VFP_EINVAL, "batch too large (%lld tiles)", tot);
  }
  st.back() = (int)tot;
  cl.total = (int)tot;
  std::vector<int> tr((size_t)tot);
  for (size_t j = 0; j < cl.members.size(); ++j) std::fill(tr.begin() + st[j], tr.begin() + st[j + 1], (int)j);
  if (int e = upload_vec(cl.start, st)) return e;
  return upload_vec(cl.tile_run, tr);
}

// The per-run stage descriptors copy field pointers and values at bind time;
// a set-up call on a run afterwards may free or change them.
int check_bound_current(const vfp_batch* b) {
  if (!b->bound) return fail(VFP_ESTATE, "vfp_batch_bind has not been called");
  for (size_t r = 0; r < b->runs.size(); ++r)
    if (b->runs[r]->gen != b->gen[r])
      return fail(VFP_ESTATE, "run %zu was set up again after vfp_batch_bind; bind again", r);
  return VFP_OK;
}

}  // namespace

extern "C" {

int vfp_batch_create(vfp_batch** out, vfp_ctx* const* runs, int nruns, unsigned flags) {
  if (!out) return fail(VFP_EINVAL, "out is null");
  *out = nullptr;
  if (!runs || nruns < 1) return fail(VFP_EINVAL, "need at least one run");
  if (flags & ~1u) return fail(VFP_EINVAL, "unknown batch flags 0x%x", flags);
  vfp_batch* b = new (std::nothrow) vfp_batch;
  if (!b) return fail(VFP_ENOMEM, "batch");
  b->use_graph = flags & VFP_BATCH_GRAPH;
  for (int i = 0; i < nruns; ++i) {
    if (int e = check_ready(runs[i])) {
      delete b;
      return fail(e, "run %d: %s", i, g_err.c_str());
    }
    if (b->device < 0) b->device = runs[i]->device;
    if (runs[i]->device != b->device) {
      delete b;
      return fail(VFP_EINVAL, "run %d lives on device %d, not %d", i, runs[i]->device, b->device);
    }
    for (int j = 0; j < i; ++j)
      if (runs[j] == runs[i]) {
        delete b;
        return fail(VFP_EINVAL, "run %d repeats run %d", i, j);
      }
    b->runs.push_back(runs[i]);
  }
  for (int i = 0; i < nruns; ++i) {
    vfp_ctx* c = runs[i];
    const int nrot = c->tab.nrot;
    const bool batched = c->shock && !c->linp;   // the batched kernel is built for ln p
    vfp_batch::Class* cl = nullptr;
    for (auto& x : b->classes)
      if (x.batched == batched && x.k == c->k && x.lmax == c->lmax && x.nrot == nrot) cl = &x;
    if (!cl) {
      b->classes.emplace_back();
      cl = &b->classes.back();
      cl->k = c->k;
      cl->lmax = c->lmax;
      cl->nrot = nrot;
      cl->batched = batched;
      if (batched) {
        cl->bk = find_shock_batch_kernel(c->k, c->lmax, nrot);
        if (!cl->bk.launch) {
          delete b;
          return fail(VFP_EUNSUPPORTED, "no batched kernel for k=%d lmax=%d", c->k, c->lmax);
        }
      }
    }
    cl->members.push_back(i);
  }
  for (auto& cl : b->classes) {
    if (!cl.batched) continue;
    if (int e = class_tiles(b, cl)) {
      delete b;
      return e;
    }
  }
  *out = b;
  return VFP_OK;
}

void vfp_batch_destroy(vfp_batch* b) { delete b; }

int vfp_batch_bind(vfp_batch* b, double* const* u, double* const* work, const double* dt) {
  if (!b || !u || !work || !dt) return fail(VFP_EINVAL, "null argument");
  const int nr = (int)b->runs.size();
  for (int r = 0; r < nr; ++r) {
    if (!u[r] || !work[r]) return fail(VFP_EINVAL, "run %d: null buffer", r);
    if (!std::isfinite(dt[r])) return fail(VFP_EINVAL, "run %d: dt not finite", r);
    int64_t N = 0;
    vfp_ndofs(b->runs[r], &N);
    if (overlaps(u[r], N, work[r], 2 * N)) return fail(VFP_EINVAL, "run %d: work overlaps u", r);
  }
  b->u.assign(u, u + nr);
  b->work.assign(work, work + nr);
  b->dt.assign(dt, dt + nr);
  b->gen.resize(nr);
  for (int r = 0; r < nr; ++r) b->gen[r] = b->runs[r]->gen;
  for (auto& cl : b->classes) {
    if (!cl.batched) continue;
    const size_t m = cl.members.size();
    std::vector<KernelArgs> d(4 * m);
    for (int s = 0; s < 4; ++s)
      for (size_t j = 0; j < m; ++j) {
        const int r = cl.members[j];
        vfp_ctx* c = b->runs[r];
        int64_t N = 0;
        vfp_ndofs(c, &N);
        const double* w_in;
        double* w_out;
        double cdt;
        stage_ptrs(s, b->u[r], b->work[r], N, b->dt[r], w_in, w_out, cdt);
        d[s * m + j] = stage_args(c, w_in, b->u[r], w_out, cdt);
      }
    if (int e = upload_vec(cl.descs, d)) return e;
  }
  b->drop_graph();
  b->bound = true;
  return VFP_OK;
}

int vfp_batch_advance(vfp_batch* b, int64_t nsteps, void* stream) {
  if (!b) return fail(VFP_EINVAL, "null batch");
  if (int e = check_bound_current(b)) return e;
  if (nsteps < 0) return fail(VFP_EINVAL, "nsteps < 0");
  hipStream_t st = (hipStream_t)stream;
  if (!b->use_graph) {
    for (int64_t i = 0; i < nsteps; ++i)
      if (int e = batch_step(b, st)) return e;
    return VFP_OK;
  }
  if (!b->stream) {
    HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    for (size_t i = 0; i < b->classes.size(); ++i) {
      hipStream_t bs;
      hipEvent_t je;
      HIP_TRY(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
      b->branch.push_back(bs);
      HIP_TRY(hipEventCreateWithFlags(&je, hipEventDisableTiming));
      b->joins.push_back(je);
    }
  }
  if (!b->exec) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int e = batch_step_branched(b, b->stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (e) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    if (ce != hipSuccess) return fail(VFP_EDEVICE, "graph capture: %s", hipGetErrorString(ce));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  // order after the caller's stream, replay, and order the caller after us
  HIP_TRY(hipEventRecord(b->ev_in, st));
  HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_in, 0));
  for (int64_t i = 0; i < nsteps; ++i) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  HIP_TRY(hipEventRecord(b->ev_out, b->stream));
  HIP_TRY(hipStreamWaitEvent(st, b->ev_out, 0));
  return VFP_OK;
}

// Times every workgroup shape (cells per tile and lanes per workgroup) and
// both tile orders of a class's batched kernel and keeps the fastest.
static int tune_class(vfp_batch* b, vfp_batch::Class& cl, int reps, hipStream_t st, hipEvent_t e0,
                      hipEvent_t e1) {
  // every (shape, tile order) runs a step's mix of stage forms: the first
  // stage (reads u) and three that read a work vector and u (stages 2, 3
  // and 2 again: the last stage, which writes u, is left out so u stays
  // untouched), reps times, over two rounds keeping each candidate's faster
  // one
  struct Cand {
    int shape, tm;
    float best;
  };
  std::vector<Cand> cand;
  for (int shape = 0; shape < kShockShapes; ++shape)
    if (find_shock_batch_kernel(cl.k, cl.lmax, cl.nrot, shape).launch)
      for (int tm : {0, 1}) cand.push_back({shape, tm, 1e30f});
  for (int round = 0; round < 2; ++round)
    for (Cand& cd : cand) {
      cl.bk = find_shock_batch_kernel(cl.k, cl.lmax, cl.nrot, cd.shape);
      cl.shape = cd.shape;
      if (int e = class_tiles(b, cl)) return e;
      cl.tile_map = cd.tm;
      for (int s : {0, 1, 2})
        if (int e = batch_launch_stage(b, cl, s, st)) return e;
      HIP_TRY(hipEventRecord(e0, st));
      for (int i = 0; i < reps; ++i)
        for (int s : {0, 1, 2, 1})
          if (int e = batch_launch_stage(b, cl, s, st)) return e;
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      cd.best = std::min(cd.best, ms);
    }
  int bt = cl.tile_map, bs = cl.shape;
  if (!cand.empty()) {
    const Cand* w = &cand[0];
    for (const Cand& cd : cand)
      if (cd.best < w->best) w = &cd;
    bt = w->tm;
    bs = w->shape;
  }
  cl.tile_map = bt;
  cl.shape = bs;
  cl.bk = find_shock_batch_kernel(cl.k, cl.lmax, cl.nrot, bs);
  return class_tiles(b, cl);
}

int vfp_batch_autotune(vfp_batch* b, int reps, void* stream) {
  if (!b) return fail(VFP_EINVAL, "null batch");
  if (int e = check_bound_current(b)) return e;
  if (reps < 1) reps = 3;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(VFP_EDEVICE, "hipEventCreate");
  }
  int rc = VFP_OK;
  for (auto& cl : b->classes) {
    if (!cl.batched) continue;
    if ((rc = tune_class(b, cl, reps, (hipStream_t)stream, e0, e1))) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->drop_graph();
  return rc;
}

int vfp_batch_nclasses(const vfp_batch* b) { return b ? (int)b->classes.size() : 0; }

int vfp_batch_class_info(const vfp_batch* b, int i, int* info) {
  if (!b || !info) return fail(VFP_EINVAL, "null argument");
  if (i < 0 || i >= (int)b->classes.size()) return fail(VFP_EINVAL, "class %d", i);
  const auto& cl = b->classes[i];
  info[0] = cl.k;
  info[1] = cl.lmax;
  info[2] = cl.nrot;
  info[3] = (int)cl.members.size();
  info[4] = cl.batched ? 1 : 0;
  info[5] = cl.total;
  info[6] = cl.batched ? cl.bk.threads : 0;
  info[7] = cl.tile_map;
  return VFP_OK;
}

}  // extern "C"

namespace vfp {
int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ctx_device(const vfp_ctx* c) { return c ? c->device : -1; }
}  // namespace vfp

