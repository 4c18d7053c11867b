// Host entry points into the general stage kernels (one translation unit
// per family of axes and direction, stage_gen_*.hip) and the cell mass
// kernel.
#include "stage_body.hpp"

namespace vfp {

StageLauncher stage_family_1f(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_1f(const Basis1D* b);
StageLauncher stage_family_1a(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_1a(const Basis1D* b);
StageLauncher stage_family_2f(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_2f(const Basis1D* b);
StageLauncher stage_family_2a(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_2a(const Basis1D* b);
StageLauncher stage_family_3f(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_3f(const Basis1D* b);
StageLauncher stage_family_3a(int k, int lmax, bool mom, int flow);
hipError_t upload_basis_3a(const Basis1D* b);

namespace {

using gen::kThreads;

// Cell mass matrix (or its inverse) applied per (cell, lms) lane.
template <int D, int K, bool INV>
__global__ __launch_bounds__(kThreads) void mass_kernel(MeshArgs M, int n, const double* in, double* out) {
  constexpr int NB = IPow<K + 1, D>::v;
  const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (size_t)M.ncells * n) return;
  const int cell = (int)(t / n);
  const int r = (int)(t - (size_t)cell * n);
  int ic[3];
  {
    int c = cell;
    ic[0] = c % M.n[0];
    c /= M.n[0];
    ic[1] = c % M.n[1];
    ic[2] = c / M.n[1];
  }
  const size_t base = (size_t)cell * NB * n + r;
  double v[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) v[b] = in[base + (size_t)b * n];
  ref_mass<D, K, INV>(v);
  const double jac = cell_jacobian<D>(M, ic);
  const double sc = INV ? 1.0 / jac : jac;
#pragma unroll
  for (int b = 0; b < NB; ++b) out[base + (size_t)b * n] = sc * v[b];
}

template <int D, int K>
void launch_mass_t(const MeshArgs& m, int n, const double* in, double* out, bool inv, hipStream_t s) {
  const size_t lanes = (size_t)m.ncells * n;
  const int blocks = (int)((lanes + kThreads - 1) / kThreads);
  if (inv)
    hipLaunchKernelGGL((mass_kernel<D, K, true>), dim3(blocks), dim3(kThreads), 0, s, m, n, in, out);
  else
    hipLaunchKernelGGL((mass_kernel<D, K, false>), dim3(blocks), dim3(kThreads), 0, s, m, n, in, out);
}


}  // namespace

StageLauncher find_stage_launcher(int D, int k, int lmax, bool mom, int flow) {
  if (D == 1) return stage_family_1f(k, lmax, mom, flow);
  if (D == 2) return stage_family_2f(k, lmax, mom, flow);
  if (D == 3) return stage_family_3f(k, lmax, mom, flow);
  return nullptr;
}

StageLauncher find_adjoint_launcher(int D, int k, int lmax, bool mom, int flow) {
  if (D == 1) return stage_family_1a(k, lmax, mom, flow);
  if (D == 2) return stage_family_2a(k, lmax, mom, flow);
  if (D == 3) return stage_family_3a(k, lmax, mom, flow);
  return nullptr;
}

MassLauncher find_mass_launcher(int D, int k) {
  if (k == 1) return D == 1 ? &launch_mass_t<1, 1> : D == 2 ? &launch_mass_t<2, 1> : &launch_mass_t<3, 1>;
  if (k == 2) return D == 1 ? &launch_mass_t<1, 2> : D == 2 ? &launch_mass_t<2, 2> : &launch_mass_t<3, 2>;
  return nullptr;
}

hipError_t upload_basis(const Basis1D* b) {
  const hipError_t own = hipMemcpyToSymbol(HIP_SYMBOL(c_basis), b, sizeof(Basis1D) * kMaxK, 0,
                                           hipMemcpyHostToDevice);
  if (own != hipSuccess) return own;
  for (auto up : {&upload_basis_1f, &upload_basis_1a, &upload_basis_2f, &upload_basis_2a, &upload_basis_3f,
                   &upload_basis_3a, &upload_basis_resident})
    if (hipError_t e = up(b); e != hipSuccess) return e;
  return hipSuccess;
}

int stage_threads_general() { return kThreads; }

int stage_cells_per_block(int lmax) {
  const int n = (lmax + 1) * (lmax + 1);
  return (kThreads / n) > 0 ? kThreads / n : 1;
}

}  // namespace vfp
