// Small runs on one axis advanced entirely inside one workgroup: the state
// u and the two stage vectors live in LDS (3 N doubles, N <= 2730) and one
// launch takes every Runge-Kutta stage of every step (the four-stage form
// w_i = u + c_i dt L(w_{i-1}), c = 1/4, 1/3, 1/2, 1, as vfp_advance), with a
// workgroup barrier between stages instead of a kernel launch.  For a run of
// a few thousand degrees of freedom a stage is a few hundred cycles of work,
// far below the cost of a launch.  Each thread owns one (cell, lms) item and
// keeps that item's matrix rows in registers, so that a stage reads LDS only.
//
// The operator is that of the general kernel for one spatial axis, a
// uniform flow, fixed p and a uniform B: volume advection in node space
// (2/h) dvol (U w + V A^x w) (the coefficients are constant on the cell), the
// reaction nu C - (q/(gamma m)) B.Omega at the Gauss points, tested with tst,
// and the upwind face flux J = (beta (F1 + F2) + |beta| (F1 - F2)) / 2 at the
// face node, lifted with the 1-D lift (eq. definition-upwind-flux; zero
// inflow, continuous or periodic ends).
#include "kernels.hpp"
#include "launch.hpp"

namespace vfp {
namespace {

constexpr int kResThreads = kResidentItems;

template <int K, int LMAX>
__global__ __launch_bounds__(kResThreads) void resident_kernel(KernelArgs A, double dt, long long nsteps,
                                                               double* __restrict__ u_glob) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr int K1 = K + 1;
  extern __shared__ double lds[];
  const MeshArgs& M = A.mesh;
  const FieldArgs& F = A.fld;
  const RowTables& T = A.tab;
  const Basis1D& bs = c_basis[K - 1];
  const int nc = M.ncells;
  const int tot = nc * K1 * N;
  double* Us = lds;
  double* Wa = lds + tot;
  double* Wb = lds + 2 * tot;
  for (int i = threadIdx.x; i < tot; i += kResThreads) Us[i] = u_glob[i];
  __syncthreads();
  const int items = nc * N;
  const int nfb = T.nfb[0], nfa = T.nfa[0], nrot = T.nrot;
  // One item (cell, lms row) per thread -- the host selects this kernel only
  // then, and only with the row counts within the caps below: the item's
  // rows of the face matrices (their factor 1/2 folded in, exactly), of A^x
  // and of B.Omega, its cell width, collision factor and source stay in
  // registers for all steps, so that a stage reads only LDS.
  constexpr int FBC = kResFbCap, FAC = kResFaCap<LMAX>, RC = kResRotCap;
  const int it0 = threadIdx.x;
  const bool act = it0 < items;
  const int cell = act ? it0 / N : 0, r = act ? it0 - (it0 / N) * N : 0;
  int fbc[FBC], fac[FAC], rc[RC];
  double fbv[FBC], fav[FAC], rv[RC];
#pragma unroll
  for (int s = 0; s < FBC; ++s) {
    fbc[s] = s < nfb ? T.fb_col[0][s * N + r] : 0;
    fbv[s] = s < nfb ? 0.5 * T.fb_val[0][s * N + r] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < FAC; ++s) {
    fac[s] = s < nfa ? T.fa_col[0][s * N + r] : 0;
    fav[s] = s < nfa ? 0.5 * T.fa_val[0][s * N + r] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < RC; ++s) {
    rc[s] = s < nrot ? T.rot_col[s * N + r] : 0;
    rv[s] = s < nrot ? T.rot_val[s * N + r] : 0.0;
  }
  const int c0 = T.ax_col[r], c1 = T.ax_col[N + r];
  const double v0 = T.ax_val[r], v1 = T.ax_val[N + r];
  const double s2h = M.s2h[0][cell];
  const double nu = F.nu_cell ? F.nu_cell[cell] : F.nu0;
  const double cnu = F.t_col * nu * T.c_val[r];
  const double pig = F.t_rot * F.ig0;
  const bool with_src = A.st.with_source && F.src && r == 0;
  double src[K1];
#pragma unroll
  for (int j = 0; j < K1; ++j) src[j] = with_src ? F.src[(size_t)cell * K1 + j] : 0.0;
  // neighbours and boundary kinds of the two faces
  int nbr[2], kind[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int bc = side ? M.bc_hi[0] : M.bc_lo[0];
    int ni = side ? cell + 1 : cell - 1;
    const bool inside = ni >= 0 && ni < nc;
    nbr[side] = (ni + nc) % nc;
    kind[side] = (inside || bc == 0) ? 0 : bc;   // 0 neighbour, 1 zero inflow, 2 continuous
  }
  for (long long step = 0; step < nsteps; ++step) {
#pragma unroll 1
    for (int st = 0; st < 4; ++st) {
      const double* Win = st == 0 ? Us : (st == 2 ? Wb : Wa);
      double* Wout = st == 3 ? Us : (st == 1 ? Wb : Wa);
      // c_s dt, rounded as the host rounds it for the stage launches
      const double cdt = st == 0 ? 0.25 * dt : (st == 1 ? dt / 3.0 : (st == 2 ? 0.5 * dt : dt));
      if (act) {
        const double* own = Win + (size_t)cell * K1 * N;
        double w[K1], res[K1];
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          w[j] = own[j * N + r];
          res[j] = 0.0;
        }
        // faces at the face node
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const double* own_t = own + (side ? K : 0) * N;
          const double* nbr_t = Win + ((size_t)nbr[side] * K1 + (side ? 0 : K)) * N;
          const int kd = kind[side];
          auto f1 = [&](int c) {
            const double o = own_t[c], x = kd == 0 ? nbr_t[c] : (kd == 1 ? 0.0 : o);
            return side ? o : x;
          };
          auto f2 = [&](int c) {
            const double o = own_t[c], x = kd == 0 ? nbr_t[c] : (kd == 1 ? 0.0 : o);
            return side ? x : o;
          };
          double J = 0.0;
#pragma unroll
          for (int s = 0; s < FBC; ++s)
            if (s < nfb) J = fma(fbv[s], f1(fbc[s]) + f2(fbc[s]), J);
#pragma unroll
          for (int s = 0; s < FAC; ++s)
            if (s < nfa) J = fma(fav[s], f1(fac[s]) - f2(fac[s]), J);
          const double sc = (side ? -1.0 : 1.0) * s2h;
#pragma unroll
          for (int j = 0; j < K1; ++j) res[j] = fma(sc * bs.lift[side][j], J, res[j]);
        }
        // advection in node space
        {
          double t[K1];
#pragma unroll
          for (int j = 0; j < K1; ++j)
            t[j] = fma(F.U[0], w[j], F.V0 * (v0 * own[j * N + c0] + v1 * own[j * N + c1]));
          const double sc = F.t_adv * s2h;
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < K1; ++j) acc = fma(bs.dvol[i][j], t[j], acc);
            res[i] = fma(sc, acc, res[i]);
          }
        }
        // reaction at the Gauss points
        {
          double g[K1];
#pragma unroll
          for (int q = 0; q < K1; ++q) {
            double f = 0.0;
#pragma unroll
            for (int j = 0; j < K1; ++j) f = fma(bs.phi[q][j], w[j], f);
            double rot = 0.0;
#pragma unroll
            for (int s = 0; s < RC; ++s)
              if (s < nrot) {
                double fc = 0.0;
#pragma unroll
                for (int j = 0; j < K1; ++j) fc = fma(bs.phi[q][j], own[j * N + rc[s]], fc);
                rot = fma(rv[s], fc, rot);
              }
            g[q] = fma(-pig, rot, cnu * f);
          }
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < K1; ++q) acc = fma(bs.tst[i][q], g[q], acc);
            res[i] -= acc;
          }
        }
        if (with_src) {
#pragma unroll
          for (int j = 0; j < K1; ++j) res[j] += src[j];
        }
        // w_out = u + cdt L(w_in); each item reads its own u entries before
        // the last stage overwrites them
        double* ob = Wout + (size_t)cell * K1 * N + r;
        const double* ub = Us + (size_t)cell * K1 * N + r;
#pragma unroll
        for (int j = 0; j < K1; ++j) ob[j * N] = fma(cdt, res[j], ub[j * N]);
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < tot; i += kResThreads) u_glob[i] = Us[i];
}

template <int K, int LMAX>
void launch_t(const KernelArgs& a, double dt, long long nsteps, double* u, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  const size_t lds = (size_t)3 * a.mesh.ncells * (K + 1) * N * sizeof(double);
  hipLaunchKernelGGL((resident_kernel<K, LMAX>), dim3(1), dim3(kResThreads), lds, s, a, dt, nsteps, u);
}

template <int K>
ResidentLauncher pick(int lmax) {
  switch (lmax) {
    case 1: return &launch_t<K, 1>;
    case 2: return &launch_t<K, 2>;
    case 3: return &launch_t<K, 3>;
    case 4: return &launch_t<K, 4>;
    case 5: return &launch_t<K, 5>;
    case 6: return &launch_t<K, 6>;
    case 7: return &launch_t<K, 7>;
    default: return nullptr;
  }
}

}  // namespace

ResidentLauncher find_resident_launcher(int k, int lmax) {
  if (k == 1) return pick<1>(lmax);
  if (k == 2) return pick<2>(lmax);
  return nullptr;
}

size_t resident_max_lds() { return 64 * 1024; }

hipError_t upload_basis_resident(const Basis1D* b) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_basis), b, sizeof(Basis1D) * kMaxK, 0, hipMemcpyHostToDevice);
}

}  // namespace vfp
