// Batched (x, ln p) stage kernel: one launch per Runge-Kutta stage covers
// the tiles of many independent runs of one (k, l_max) class, each with its
// own mesh, fields, time step and state buffers.  One workgroup per tile: a
// loop over several tiles per workgroup keeps more values live across the
// iterations and costs a wave per SIMD.
#include "shock_body.hpp"

namespace vfp {
namespace {

using namespace shock;

template <int K, int LMAX, int NROT>
__global__ __launch_bounds__(Launch<(LMAX + 1) * (LMAX + 1)>::kThreads) __attribute__((amdgpu_waves_per_eu(VFP_SHOCK_WAVES)))
void shock_batch_kernel(const KernelArgs* __restrict__ descs, const int* __restrict__ start,
                        const int* __restrict__ tile_run, int total, int tile_map) {
  // descs, start and tile_run are read only and alias nothing the kernel
  // writes, so their loads (uniform addresses) stay scalar like kernel
  // arguments; tile_run[t] names the run of tile t in one load
  const int t = tile_map ? xcd_tile(blockIdx.x, total) : (int)blockIdx.x;
  const int run = __builtin_amdgcn_readfirstlane(tile_run[t]);
  shock_body<K, LMAX, NROT, false>(descs[run], t - start[run]);
}

template <int K, int LMAX, int NROT>
void launch_batch_t(const BatchArgs& b, hipStream_t s) {
  constexpr int N = (LMAX + 1) * (LMAX + 1);
  hipLaunchKernelGGL((shock_batch_kernel<K, LMAX, NROT>), dim3(b.total), dim3(Launch<N>::kThreads), 0, s, b.descs,
                     b.start, b.tile_run, b.total, b.tile_map);
}

template <int K, int NROT>
BatchKernel pick(int lmax) {
  switch (lmax) {
    case 1: return {&launch_batch_t<K, 1, NROT>, Launch<4>::kCells};
    case 2: return {&launch_batch_t<K, 2, NROT>, Launch<9>::kCells};
    case 3: return {&launch_batch_t<K, 3, NROT>, Launch<16>::kCells};
    case 4: return {&launch_batch_t<K, 4, NROT>, Launch<25>::kCells};
    case 5: return {&launch_batch_t<K, 5, NROT>, Launch<36>::kCells};
    case 6: return {&launch_batch_t<K, 6, NROT>, Launch<49>::kCells};
    case 7: return {&launch_batch_t<K, 7, NROT>, Launch<64>::kCells};
    default: return {};
  }
}

}  // namespace

BatchKernel find_shock_batch_kernel(int k, int lmax, int nrot) {
  if (nrot != 1 && nrot != 5) return {};
  if (k == 1) return nrot == 1 ? pick<1, 1>(lmax) : pick<1, 5>(lmax);
  if (k == 2) return nrot == 1 ? pick<2, 1>(lmax) : pick<2, 5>(lmax);
  return {};
}

int shock_cells_per_tile(int lmax) {
  const int n = (lmax + 1) * (lmax + 1);
  const int threads = (64 % n) == 0 ? 64 : 256;
  return threads / n > 0 ? threads / n : 1;
}

}  // namespace vfp
