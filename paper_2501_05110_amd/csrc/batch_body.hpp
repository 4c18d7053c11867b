// Batched (x, ln p) stage kernel: one launch per Runge-Kutta stage covers
// the tiles of many independent runs of one (k, l_max) class, each with its
// own mesh, fields, time step and state buffers.  One workgroup per tile: a
// loop over several tiles per workgroup keeps more values live across the
// iterations and costs a wave per SIMD.  TPB selects the workgroup shape
// (see shock::Launch); the tile size follows it.
#pragma once
#include "shock_body.hpp"

namespace vfp {
namespace shock {

template <int K, int LMAX, int NROT, int TPB>
__global__ __launch_bounds__((Launch<(LMAX + 1) * (LMAX + 1), TPB>::kThreads)) __attribute__((amdgpu_waves_per_eu(VFP_SHOCK_WAVES)))
void shock_batch_kernel(const KernelArgs* __restrict__ descs, const int* __restrict__ start,
                        const int* __restrict__ tile_run, int total, int tile_map) {
  // descs, start and tile_run are read only and alias nothing the kernel
  // writes, so their loads (uniform addresses) stay scalar like kernel
  // arguments; tile_run[t] names the run of tile t in one load
  const int t = tile_map ? xcd_tile(blockIdx.x, total) : (int)blockIdx.x;
  const int run = __builtin_amdgcn_readfirstlane(tile_run[t]);
  shock_body<K, LMAX, NROT, false, false, TPB>(descs[run], t - start[run]);
}

template <int K, int LMAX, int NROT, int TPB>
void launch_batch_t(const BatchArgs& b, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  hipLaunchKernelGGL((shock_batch_kernel<K, LMAX, NROT, TPB>), dim3(b.total), dim3(Launch<N, TPB>::kThreads), 0, s,
                     b.descs, b.start, b.tile_run, b.total, b.tile_map);
}

template <int K, int LMAX, int NROT, int TPB>
BatchKernel batch_entry() {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  return {&launch_batch_t<K, LMAX, NROT, TPB>, Launch<N, TPB>::kCells, Launch<N, TPB>::kThreads};
}

template <int K, int NROT, int TPB>
BatchKernel batch_pick(int lmax) {
  switch (lmax) {
    case 1: return batch_entry<K, 1, NROT, TPB>();
    case 2: return batch_entry<K, 2, NROT, TPB>();
    case 3: return batch_entry<K, 3, NROT, TPB>();
    case 4: return batch_entry<K, 4, NROT, TPB>();
    case 5: return batch_entry<K, 5, NROT, TPB>();
    case 6: return batch_entry<K, 6, NROT, TPB>();
    case 7: return batch_entry<K, 7, NROT, TPB>();
    default: return {};
  }
}

}  // namespace shock
}  // namespace vfp
