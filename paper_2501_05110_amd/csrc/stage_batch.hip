// Batched (x, ln p) stage kernel in its default workgroup shape (the kernel
// template is in batch_body.hpp, the other shapes in stage_batch_shapes.hip).
#include "batch_body.hpp"

namespace vfp {

using shock::batch_pick;

BatchKernel find_shock_batch_kernel(int k, int lmax, int nrot, int slot) {
  if (slot != 0) return find_shock_batch_kernel_shape(k, lmax, nrot, slot);
  if (nrot != 1 && nrot != 5) return {};
  if (k == 1) return nrot == 1 ? batch_pick<1, 1, 0>(lmax) : batch_pick<1, 5, 0>(lmax);
  if (k == 2) return nrot == 1 ? batch_pick<2, 1, 0>(lmax) : batch_pick<2, 5, 0>(lmax);
  return {};
}

int shock_shape_threads(int lmax, int slot) {
  const int n = (lmax + 1) * (lmax + 1);
  const bool whole = (64 % n) == 0;
  if (slot == 1) return whole ? 128 : 64;
  if (slot == 2) return whole ? 256 : 128;
  return whole ? 64 : 256;
}

int shock_shape_cells(int lmax, int slot) {
  const int n = (lmax + 1) * (lmax + 1);
  const int t = shock_shape_threads(lmax, slot);
  return t / n > 0 ? t / n : 1;
}

int shock_cells_per_tile(int lmax) { return shock_shape_cells(lmax, 0); }

}  // namespace vfp
