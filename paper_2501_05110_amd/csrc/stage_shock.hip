// Single-run (x, ln p) and (x, p) stage kernels: forward
// (w_out = alpha u + beta L(w_in)) and adjoint, one launch per stage over all
// cells of one run.
#include "shock_body.hpp"

namespace vfp {
namespace {

using namespace shock;

template <int K, int LMAX, int NROT, bool ADJ, bool LINP, int TPB>
__global__ __launch_bounds__((Launch<(LMAX + 1) * (LMAX + 1), TPB>::kThreads)) __attribute__((amdgpu_waves_per_eu(VFP_SHOCK_WAVES)))
void shock_kernel(KernelArgs A) {
  const int blk = A.tile_map ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  shock_body<K, LMAX, NROT, ADJ, LINP, TPB>(A, blk);
}

template <int K, int LMAX, int NROT, bool ADJ, bool LINP, int TPB = 0>
void launch_shock_t(const KernelArgs& a, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  using L = Launch<N, TPB>;
  const int blocks = (a.mesh.ncells + L::kCells - 1) / L::kCells;
  hipLaunchKernelGGL((shock_kernel<K, LMAX, NROT, ADJ, LINP, TPB>), dim3(blocks), dim3(L::kThreads), 0, s, a);
}

template <int K, int NROT, bool ADJ, bool LINP>
StageLauncher pick(int lmax) {
  switch (lmax) {
    case 1: return &launch_shock_t<K, 1, NROT, ADJ, LINP>;
    case 2: return &launch_shock_t<K, 2, NROT, ADJ, LINP>;
    case 3: return &launch_shock_t<K, 3, NROT, ADJ, LINP>;
    case 4: return &launch_shock_t<K, 4, NROT, ADJ, LINP>;
    case 5: return &launch_shock_t<K, 5, NROT, ADJ, LINP>;
    case 6: return &launch_shock_t<K, 6, NROT, ADJ, LINP>;
    case 7: return &launch_shock_t<K, 7, NROT, ADJ, LINP>;
    default: return nullptr;
  }
}

template <bool ADJ, bool LINP>
StageLauncher pick_shock(int k, int lmax, int nrot) {
  if (nrot != 1 && nrot != 5) return nullptr;
  if (k == 1) return nrot == 1 ? pick<1, 1, ADJ, LINP>(lmax) : pick<1, 5, ADJ, LINP>(lmax);
  if (k == 2) return nrot == 1 ? pick<2, 1, ADJ, LINP>(lmax) : pick<2, 5, ADJ, LINP>(lmax);
  return nullptr;
}

}  // namespace

StageLauncher find_shock_launcher(int k, int lmax, int nrot, bool linp) {
  return linp ? pick_shock<false, true>(k, lmax, nrot) : pick_shock<false, false>(k, lmax, nrot);
}

StageLauncher find_shock_adjoint_launcher(int k, int lmax, int nrot, bool linp) {
  return linp ? pick_shock<true, true>(k, lmax, nrot) : pick_shock<true, false>(k, lmax, nrot);
}

}  // namespace vfp
