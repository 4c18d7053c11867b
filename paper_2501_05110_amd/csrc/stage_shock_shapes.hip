// The forward (x, ln p) stage kernel in its other workgroup shapes, for the
// autotuner (vfp_autotune): 128 and 256 lanes where n divides 64 (several
// wavefronts of whole cells), 64 and 128 lanes otherwise (one or a few
// cells).  The default shape is in stage_shock.hip.
#include "shock_body.hpp"

namespace vfp {
namespace {

using namespace shock;

template <int K, int LMAX, int NROT, int TPB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(VFP_SHOCK_WAVES)))
void shock_kernel_shaped(KernelArgs A) {
  const int blk = A.tile_map ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  shock_body<K, LMAX, NROT, false, false, TPB>(A, blk);
}

template <int K, int LMAX, int NROT, int TPB>
void launch_t(const KernelArgs& a, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  using L = Launch<N, TPB>;
  const int blocks = (a.mesh.ncells + L::kCells - 1) / L::kCells;
  hipLaunchKernelGGL((shock_kernel_shaped<K, LMAX, NROT, TPB>), dim3(blocks), dim3(TPB), 0, s, a);
}

template <int K, int LMAX, int NROT>
StageLauncher by_shape(int slot) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  constexpr bool whole = (64 % N) == 0;
  if (slot == 1) return &launch_t<K, LMAX, NROT, whole ? 128 : 64>;
  if (slot == 2) return &launch_t<K, LMAX, NROT, whole ? 256 : 128>;
  return nullptr;
}

template <int K, int NROT>
StageLauncher by_lmax(int lmax, int slot) {
  switch (lmax) {
    case 1: return by_shape<K, 1, NROT>(slot);
    case 2: return by_shape<K, 2, NROT>(slot);
    case 3: return by_shape<K, 3, NROT>(slot);
    case 4: return by_shape<K, 4, NROT>(slot);
    case 5: return by_shape<K, 5, NROT>(slot);
    case 6: return by_shape<K, 6, NROT>(slot);
    case 7: return by_shape<K, 7, NROT>(slot);
    default: return nullptr;
  }
}

}  // namespace

// Built for a B along x (one entry per row of B.Omega), the field of the
// shock runs.
StageLauncher find_shock_launcher_shape(int k, int lmax, int nrot, int slot) {
  if (nrot != 1) return nullptr;
  if (k == 1) return by_lmax<1, 1>(lmax, slot);
  if (k == 2) return by_lmax<2, 1>(lmax, slot);
  return nullptr;
}

}  // namespace vfp
