// Host-side entry points into the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace vfp {

using StageLauncher = void (*)(const KernelArgs&, hipStream_t);

// Kernel for (axes D, degree k, l_max, ln-p axis present, flow kind: 0
// uniform, 1 planar x profile, 2 given at the points), or nullptr if that
// combination is not built.
StageLauncher find_stage_launcher(int D, int k, int lmax, bool mom, int flow);

// Adjoint kernel (K = -M^{-1} D^T on mu = M^{-1} lambda) for the same families.
StageLauncher find_adjoint_launcher(int D, int k, int lmax, bool mom, int flow);

// out = M in (inv = false) or M^{-1} in per cell, n coefficients per node.
using MassLauncher = void (*)(const MeshArgs&, int n, const double* in, double* out, bool inv, hipStream_t);
MassLauncher find_mass_launcher(int D, int k);

// Specialised kernel for two axes (x, ln p) with a planar x flow and a
// uniform B; nrot = padded non-zeros per row of B.Omega (1 or 5).
// linp: the momentum axis is p itself instead of ln p.
StageLauncher find_shock_launcher(int k, int lmax, int nrot, bool linp = false);
StageLauncher find_shock_adjoint_launcher(int k, int lmax, int nrot, bool linp = false);
// The forward ln p kernel in workgroup shape slot 1 or 2 (slot 0 is the
// default of find_shock_launcher): 128 / 256 lanes where n divides 64, else
// 64 / 128 lanes; built for nrot = 1.  nullptr where not built.
StageLauncher find_shock_launcher_shape(int k, int lmax, int nrot, int slot);
constexpr int kShockShapes = 3;
// Cells per workgroup (tile) and lanes of shape slot 0..2 for l_max.
int shock_shape_cells(int lmax, int slot);
int shock_shape_threads(int lmax, int slot);

// Batched (x, ln p) forward stage over many runs of one (k, l_max, nrot)
// class: one workgroup per tile, in workgroup shape slot 0..2 (as above).
struct BatchKernel {
  void (*launch)(const BatchArgs&, hipStream_t) = nullptr;
  int cells_per_tile = 0;
  int threads = 0;
};
BatchKernel find_shock_batch_kernel(int k, int lmax, int nrot, int slot = 0);
BatchKernel find_shock_batch_kernel_shape(int k, int lmax, int nrot, int slot);
int shock_cells_per_tile(int lmax);

// Field sensitivities of one stage (planar flow of an (x, ln p) run):
// accumulate cdt <mu, d(h - D fwd)/dfield> into per-cell slots; reduce the
// slots to dJ/dU, dJ/dU', dJ/d(dU/dt) at the x Gauss points and dJ/dU at the
// x faces.
// support: per x cell, 0 where the U' and dU/dt sensitivities are not
// wanted (null: everywhere).  p1_blocks: the np1 tiles (field_grad_tiles
// numbering) that hold a support cell, or null for every tile.  grad_nu:
// per cell, receives the same dJ/dnu term the adjoint stage would add for
// this (mu, fwd, cdt), or null.
using FieldGradLauncher = void (*)(const KernelArgs&, const double* mu, const double* fwd, double cdt,
                                   double* slots, const unsigned char* support, const int* p1_blocks, int np1,
                                   double* grad_nu, hipStream_t);
using FieldGradReduce = void (*)(const MeshArgs&, const double* slots, double* g_u, double* g_du, double* g_a,
                                 double* g_uf, hipStream_t);
FieldGradLauncher find_field_grad_launcher(int k, int lmax);
FieldGradReduce find_field_grad_reduce(int k);
int field_grad_slots_per_cell(int k);
// cells per tile of the field-gradient kernel, and tiles of a mesh
int field_grad_tile_cells(int lmax);
int field_grad_tiles(int ncells, int lmax);

// Krylov-basis vector arithmetic (restarted GMRES of the Theta-method).
// Vectors j of a basis are V + j ldv.  kry_mdot: out[j] = V_j . w for j < k,
// and with self also out[k] = w . w from the same pass (partial:
// kKryMaxVectors * kKryBlocks doubles of scratch, k + self <= kKryMaxVectors);
// kry_maxpy: w += sign sum_j coef[j] V_j (coef on the device), and with norm2
// also *norm2 = |w|^2 of the result (partial: kKryBlocks doubles);
// kry_lincomb: out = a x + b y.
constexpr int kKryMaxVectors = 72;
constexpr int kKryBlocks = 1024;
// enable (device, may be null): the pass is skipped where *enable == 0.
void kry_mdot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial, double* out,
              hipStream_t s, bool self = false, const double* enable = nullptr);
void kry_maxpy(double* w, const double* V, int64_t ldv, int k, const double* coef, double sign, int64_t n,
               hipStream_t s, double* partial = nullptr, double* norm2 = nullptr, const double* enable = nullptr);
// d3[4] = 1 where the first Gram-Schmidt pass left less than half of |w|^2
// (d3[1] against d1[j + 1]), else 0
void kry_decide(const double* d1, int j, double* d3, hipStream_t s);
// d3[3] = hn = |w| after the passes (d3[2] if d3[4], else d3[1]); out = w / hn
// unless out is null
void kry_norm_scale(double* out, const double* w, int64_t n, double* d3, hipStream_t s);
void kry_lincomb(double* out, double a, const double* x, double b, const double* y, int64_t n, hipStream_t s);
// flag[0] = 1 if x (n doubles) holds a NaN or an infinity (flag left as is otherwise)
void kry_nonfinite(const double* x, int64_t n, int* flag, hipStream_t s);
// out = in / (1 + s nu_c c_lms) on a [cell][nb][n] vector (nu per cell, or nu0 if null)
void kry_coll_precond(double* out, const double* in, const double* nu, double nu0, const double* cval, double s,
                      int64_t ncells, int nb, int n, hipStream_t st);

// Block-tridiagonal preconditioner along axis 0 (xline.hip).  Blocks of
// b = nb n unknowns per cell (b <= kXlMaxBlock), three per cell, column-major:
// D (own), L (towards ix - 1), U (towards ix + 1).  Lines are the cells
// line nx .. line nx + nx - 1.  wrapc: axis 0 periodic with nx % 3 != 0 (the
// last cell gets a colour of its own).
constexpr int kXlMaxBlock = 48;
void xl_probe_set(double* v, int64_t ndofs, int nx, int b, int wrapc, int color, int j, hipStream_t s);
void xl_probe_get(const double* w, double* D, double* L, double* U, int64_t ndofs, int nx, int b, int wrapc,
                  int color, int j, hipStream_t s);
void xl_factor(double* D, double* L, double* U, int nlines, int nx, int b, int* fail, hipStream_t s);
// rowwise: one lane per row for every b (else four lanes per row where b <= 16)
void xl_apply(const double* r, double* x, const double* D, const double* L, const double* U, int nlines, int nx,
              int b, bool rowwise, hipStream_t s);

// out[row][d] = sum_j zeta[row][j] Y[d][j] for rows x ndir outputs, n <= 64.
void launch_reconstruct(const double* zeta, int64_t rows, int n, const double* Y, int64_t ndir, double* out,
                        hipStream_t s);
int reconstruct_max_lms();

hipError_t upload_basis(const Basis1D* b);

// A small run on one axis (uniform flow, fixed p, uniform B; 3 ndofs doubles
// within resident_max_lds() bytes) advanced nsteps Runge-Kutta steps in one
// launch of one workgroup holding the state in LDS; u in place.
using ResidentLauncher = void (*)(const KernelArgs&, double dt, long long nsteps, double* u, hipStream_t);
ResidentLauncher find_resident_launcher(int k, int lmax);
// The resident kernel keeps one item (cell, lms row) per thread, with the
// item's rows in registers; it serves runs of at most kResidentItems items
// whose face rows have at most kResFbCap (B) and kResFaCap<l_max> (|B|)
// entries and whose rotation row at most kResRotCap.
constexpr int kResidentItems = 1024;
constexpr int kResFbCap = 4;
template <int LMAX>
constexpr int kResFaCap = LMAX + 2;
constexpr int kResRotCap = 5;
size_t resident_max_lds();
hipError_t upload_basis_resident(const Basis1D* b);

int stage_cells_per_block(int lmax);
int stage_threads_general();

}  // namespace vfp
