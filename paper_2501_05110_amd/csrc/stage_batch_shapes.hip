// The batched (x, ln p) stage kernel in its other workgroup shapes, for the
// batch autotuner: 128 and 256 lanes where n divides 64 (several wavefronts
// of whole cells), 64 and 128 lanes otherwise.  Built for a B along x (one
// entry per row of B.Omega), the field of the shock runs.
#include "batch_body.hpp"

namespace vfp {
namespace {

using namespace shock;

template <int K>
BatchKernel shape_pick(int lmax, int slot) {
  // slot 1: 128 lanes (n | 64) or 64; slot 2: 256 lanes (n | 64) or 128
  const int n = (lmax + 1) * (lmax + 1);
  const bool whole = (64 % n) == 0;
  if (slot == 1) return whole ? batch_pick<K, 1, 128>(lmax) : batch_pick<K, 1, 64>(lmax);
  if (slot == 2) return whole ? batch_pick<K, 1, 256>(lmax) : batch_pick<K, 1, 128>(lmax);
  return {};
}

}  // namespace

BatchKernel find_shock_batch_kernel_shape(int k, int lmax, int nrot, int slot) {
  if (nrot != 1) return {};
  if (k == 1) return shape_pick<1>(lmax, slot);
  if (k == 2) return shape_pick<2>(lmax, slot);
  return {};
}

}  // namespace vfp
