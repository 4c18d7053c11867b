// General forward stage kernels on 2 axes (templates in stage_body.hpp).
#include "stage_body.hpp"

namespace vfp {

StageLauncher stage_family_2f(int k, int lmax, bool mom, int flow) {
  if (!mom && flow == gen::FLOW_UNIFORM) return gen::pick_k<2, false, gen::FLOW_UNIFORM, false>(k, lmax);
  if (!mom && flow == gen::FLOW_POINTS) return gen::pick_k<2, false, gen::FLOW_POINTS, false>(k, lmax);
  if (mom && flow == gen::FLOW_XPROF) return gen::pick_k<2, true, gen::FLOW_XPROF, false>(k, lmax);
  return nullptr;
}

hipError_t upload_basis_2f(const Basis1D* b) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_basis), b, sizeof(Basis1D) * kMaxK, 0, hipMemcpyHostToDevice);
}

}  // namespace vfp
