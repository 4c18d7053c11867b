// General forward stage kernels on 1 axis (templates in stage_body.hpp).
#include "stage_body.hpp"

namespace vfp {

StageLauncher stage_family_1f(int k, int lmax, bool mom, int flow) {
  if (mom) return nullptr;
  if (flow == gen::FLOW_XPROF) return gen::pick_k<1, false, gen::FLOW_XPROF, false>(k, lmax);
  if (flow == gen::FLOW_POINTS) return gen::pick_k<1, false, gen::FLOW_POINTS, false>(k, lmax);
  return gen::pick_k<1, false, gen::FLOW_UNIFORM, false>(k, lmax);
}

hipError_t upload_basis_1f(const Basis1D* b) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_basis), b, sizeof(Basis1D) * kMaxK, 0, hipMemcpyHostToDevice);
}

}  // namespace vfp
