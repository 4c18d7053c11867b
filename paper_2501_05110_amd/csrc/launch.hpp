// Host-side entry points into the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace vfp {

using StageLauncher = void (*)(const KernelArgs&, hipStream_t);

// Kernel for (axes D, degree k, l_max, ln-p axis present, planar-x flow
// profile), or nullptr if that combination is not built.
StageLauncher find_stage_launcher(int D, int k, int lmax, bool mom, bool xprof);

hipError_t upload_basis(const Basis1D* b);

int stage_cells_per_block(int lmax);

}  // namespace vfp
