/*
 * vfp.h -- C ABI of the MI355X library that applies and time-steps the
 * discontinuous-Galerkin discretisation of the spherical-harmonic expanded
 * Vlasov-Fokker-Planck system (Schween, Schulze & Reville, arXiv 2501.05110).
 *
 * The operator.  For the coefficient vector zeta of f_h (eq.
 * dg-discrete-representation-solution) the library evaluates
 *
 *     L(zeta) = M^{-1} ( h - D zeta )                 (eq. matrix-formulation-system-odes)
 *
 * with M, D, h as in eq. definition-mass-and-dg-matrix: volume terms
 * phi.(R - div beta) f - (grad phi . beta) f, upwind interior fluxes
 * (eq. definition-upwind-flux), weak boundary fluxes (zero inflow,
 * eq. definition-boundary-flux; "continuous", eq. continuous-bc; or periodic),
 * advection matrices beta and reaction matrix R of
 * eq. definitions-advection-reaction-eq built from the real spherical-harmonic
 * matrices A^a, Omega^a, C of Sec. 2.1 (products formed at l_max+1, then
 * truncated).  Integrals use Gauss-Legendre quadrature with k+1 points per
 * axis; the basis is the tensor Lagrange basis on Gauss-Lobatto nodes
 * (eq. lagrange-polynomial).  The momentum axis, when present, is ln p, with
 * beta^{ln p} = beta^p / p.
 *
 * Units: the code units of Table 1 (c = 1); gamma = sqrt(1 + (p/m)^2),
 * V = p/(gamma m), omega_a = q B_a / (gamma m).
 *
 * State layout (device, FP64, contiguous): zeta[cell][basis][lms] with
 *   cell  = i0 + N0 (i1 + N1 i2)          (axis 0 fastest)
 *   basis = j0 + (k+1)(j1 + (k+1) j2)      (j = Gauss-Lobatto node index per axis)
 *   lms   = l(l+1) + (-1)^(s+1) m          (eq. ordering-expansion-coefficients)
 *
 * Conventions.
 *   - Every function returns 0 on success or a negative VFP_E* code; the
 *     message of the last failure on the calling thread is vfp_last_error().
 *     Nothing is thrown across the ABI and nothing exits the process.
 *   - Set-up calls (vfp_create .. vfp_set_*) take HOST arrays, copy them, and
 *     are synchronous.  The library owns only its own tables and copies;
 *     vfp_destroy frees them.
 *   - Compute calls take DEVICE pointers owned by the caller and a stream
 *     (a hipStream_t passed as void*; NULL = the default stream).  They only
 *     enqueue work and never synchronise.
 *   - Pointers to state vectors must not alias unless a call says so.
 */
#ifndef VFP_H
#define VFP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VFP_OK            0
#define VFP_EINVAL       -1   /* bad argument */
#define VFP_ENOMEM       -2   /* allocation failed */
#define VFP_EDEVICE      -3   /* HIP runtime error */
#define VFP_ESTATE       -4   /* call out of order (e.g. apply before set_mesh) */
#define VFP_EUNSUPPORTED -5   /* valid request the library does not handle */

/* axis kinds (reduced phase space xi, Sec. 2.2) */
#define VFP_AXIS_X   0
#define VFP_AXIS_Y   1
#define VFP_AXIS_Z   2
#define VFP_AXIS_LNP 3        /* logarithmic momentum; must be the last axis */
#define VFP_AXIS_P   4        /* momentum magnitude p > 0 itself (Sec. 4: p or ln p);
                                 must be the last axis.  beta^p = -gamma m dU_a/dt A^a
                                 - p dU_b/dx^a (A^a A^b)_t (eq. definitions-advection-
                                 reaction-eq); the (x, ln p) specialisation and the
                                 flow-sensitivity calls need VFP_AXIS_LNP */

/* term switches (eq. vfp-terms-names) */
#define VFP_TERM_ADVECTION 1u  /* (U^a 1 + V A^a) d_a f                       */
#define VFP_TERM_MOMENTUM  2u  /* momentum derivative and the dU terms of R    */
#define VFP_TERM_ROTATION  4u  /* -omega_a Omega^a f                           */
#define VFP_TERM_COLLISION 8u  /* nu C f                                       */
#define VFP_TERM_SOURCE   16u  /* s                                            */

/* boundary kinds per axis end */
#define VFP_BC_PERIODIC    0
#define VFP_BC_ZERO_INFLOW 1   /* eq. definition-boundary-flux */
#define VFP_BC_CONTINUOUS  2   /* eq. continuous-bc            */

/* point sets reported by vfp_query_points (1-D coordinates along one axis) */
#define VFP_PTS_VOLUME 0      /* N_a (k+1) Gauss points, cell-major       */
#define VFP_PTS_FACE   1      /* N_a + 1 cell faces                       */
#define VFP_PTS_NODE   2      /* N_a (k+1) Gauss-Lobatto nodes, cell-major */

typedef struct vfp_ctx vfp_ctx;

/* Message of the last failed call on this thread ("" if none).  The string
 * stays valid until the next failing call on the same thread. */
const char* vfp_last_error(void);

/* Create a context.
 *   lmax       expansion degree l_max, 1..11 (n = (l_max+1)^2 coefficients);
 *              above 7 for one spatial axis x at fixed p, k <= 2, a uniform
 *              flow and B along x (the closure example of Sec. 4.3; forward
 *              operator), VFP_EUNSUPPORTED otherwise
 *   k          DG degree 1..5 (Gauss-Lobatto nodes, eq. lagrange-polynomial);
 *              k <= 3 with two axes and k <= 2 with three.  The (x, ln p)
 *              kernels, the adjoint, the mass and the flow-sensitivity calls
 *              are built for k <= 2 (VFP_EUNSUPPORTED above)
 *   naxes      1..3 axes of the reduced phase space (Sec. 4 term list: at most
 *              three; with VFP_AXIS_LNP at most two spatial axes)
 *   axis_kinds naxes kinds; spatial axes in x, y, z order, VFP_AXIS_LNP last
 *   term_mask  OR of VFP_TERM_*
 *   mass, charge  particle mass m > 0 and charge q in code units
 * Errors: VFP_EINVAL for any value outside these ranges; VFP_EUNSUPPORTED
 * for k above the limit of the number of axes. */
int vfp_create(vfp_ctx** out, int lmax, int k, int naxes, const int* axis_kinds,
               unsigned term_mask, double mass, double charge);

/* Free the context and every table it owns.  NULL is accepted. */
void vfp_destroy(vfp_ctx* ctx);

/* Rectilinear tensor mesh (Sec. 3.1: lines, rectangles or cuboids).
 *   ncells[a]  cells along axis a (>= 1)
 *   nodes[a]   host array of ncells[a]+1 strictly increasing cell boundaries
 *              (for VFP_AXIS_LNP the boundaries are values of ln p)
 *   bc_lo[a], bc_hi[a]  VFP_BC_* ; periodic must be set on both ends
 * Resets all fields to zero. */
int vfp_set_mesh(vfp_ctx* ctx, const int* ncells, const double* const* nodes,
                 const int* bc_lo, const int* bc_hi);

/* Momentum magnitude p > 0 for contexts without a ln p axis (mono-energetic
 * runs, Sec. 4.1-4.3). */
int vfp_set_momentum(vfp_ctx* ctx, double p);

/* 1-D coordinates of a point set along one axis (see VFP_PTS_*).  If coords
 * is NULL only *count is written.  Volume points of a cell (i0,i1,i2) and
 * point index q = q0 + (k+1)(q1 + (k+1) q2) sit at coordinates
 * VOLUME[a][i_a (k+1) + q_a]. */
int vfp_query_points(const vfp_ctx* ctx, int which, int axis, double* coords,
                     int64_t* count);

/* Uniform background flow U (3 components, c = 1 units): grad U = 0 and
 * dU/dt = 0. */
int vfp_set_flow_uniform(vfp_ctx* ctx, const double* U);

/* Planar flow U = U_x(x) e_x along axis 0 (which must be VFP_AXIS_X), given
 * at the axis-0 VOLUME points (u, dudx, dudt: N0(k+1) values each; dudt is
 * the material derivative dU_x/dt of eq. real-system-of-equations) and at the
 * axis-0 FACE points (u_face: N0+1 values). */
int vfp_set_flow_planar(vfp_ctx* ctx, const double* u, const double* dudx,
                        const double* dudt, const double* u_face);

/* Flow U(x) at every point, for contexts without a momentum axis and with
 * the momentum term off (U enters through beta^a = U^a 1 + V A^a and the
 * divergence term (div U) 1 of eq. definitions-advection-reaction-eq; the
 * flow-gradient terms of R and of beta^p need a momentum axis, which takes
 * vfp_set_flow_planar).  Host arrays:
 *   U      [cell][q][3] at the volume points (q as in vfp_query_points)
 *   gradU  [cell][q][3][3], gradU[..][a][b] = dU_b/dx^a; only the diagonal
 *          entries of the run's spatial axes are used (div U over those axes)
 *   U_face naxes arrays; U_face[a] is [face][qf][3] at the Gauss points of
 *          the faces normal to axis a: faces numbered over (N_a + 1)
 *          positions on axis a and N_b cells on the other axes (axis 0
 *          fastest), qf over the (k+1) Gauss points of each other axis in
 *          increasing axis order (first fastest).  Only U^a is used.  At a
 *          periodic axis both end positions are given and must agree (one
 *          face; VFP_EINVAL otherwise).
 * Upwinding uses the characteristic speeds U^a + lambda V with the constant
 * eigenvectors of A^a (eq. definition-upwind-flux).  k <= 2.  VFP_EUNSUPPORTED
 * with a momentum axis, the momentum term or k > 2; VFP_EINVAL for a value
 * that is not finite. */
int vfp_set_flow_points(vfp_ctx* ctx, const double* U, const double* gradU,
                        const double* const* U_face);

/* Uniform magnetic field B (3 components). */
int vfp_set_magnetic_uniform(vfp_ctx* ctx, const double* B);

/* Magnetic field at every volume point: host array [cell][q][3]
 * (ncells (k+1)^naxes 3 values; with a momentum axis the points span it
 * too, and omega = q B / (gamma m) takes each point's p).  The (x, ln p)
 * specialised kernels need a uniform B, so this selects the general ones. */
int vfp_set_magnetic_points(vfp_ctx* ctx, const double* B);

/* Scattering frequency nu of the collision term: nu_cell (host, one value
 * per cell) if not NULL, else the uniform value nu. */
int vfp_set_scattering(vfp_ctx* ctx, double nu, const double* nu_cell);

/* Scattering frequency at every volume point: host array [cell][q]
 * (ncells (k+1)^naxes values), integrated by the same Gauss rule as the
 * other variable coefficients, so nu may vary inside a cell.  Selects the
 * general kernels.  With nu at the points the per-cell gradient dJ/dnu
 * (grad_nu of the adjoint calls) and VFP_PRECOND_COLLISION are
 * VFP_EUNSUPPORTED. */
int vfp_set_scattering_points(vfp_ctx* ctx, const double* nu);

/* Isotropic source s (the s of eq. monoenergetic-point-source, so that
 * s_000 = sqrt(4 pi) s) at every volume point: host array [cell][q]. */
int vfp_set_source_points(vfp_ctx* ctx, const double* s);

/* Number of degrees of freedom N = cells n (k+1)^naxes (Sec. 3.1). */
int vfp_ndofs(const vfp_ctx* ctx, int64_t* n);

/* Stable explicit step dt = courant / sum_a (beta_a,max / dxi_a,min), where
 * beta_a,max bounds the spectral radius of beta^a over the mesh (the CFL rule
 * of the convergence study, Sec. 4.1, summed over axes). */
int vfp_cfl_dt(const vfp_ctx* ctx, double courant, double* dt);

/* Choose the fastest launch shape of this context's stage kernel by timing:
 * for the specialised (x, ln p) kernel, every built workgroup shape (lanes
 * per workgroup, and so cells per tile) and both tile orders (launch order,
 * or each of the 8 XCDs taking one contiguous range of tiles), each timed on
 * reps repetitions of a Runge-Kutta step's stage forms: one stage that reads
 * u and writes work (device, ndofs doubles, disjoint from u) and three that
 * read work and u and write a temporary vector of ndofs doubles that the
 * call allocates and frees (VFP_ENOMEM if it cannot); two rounds over the
 * candidates, each keeping its faster round.  u is unchanged.  The choice stays with the context (a
 * later set-up call keeps it where the kernel exists) and changes no result:
 * every shape computes each cell with the same arithmetic.  chosen (host,
 * 3 ints, may be NULL):
 * shape slot, lanes per workgroup, tile order.  Other kernels have one
 * shape: nothing is timed.  Synchronises `stream`. */
int vfp_autotune(vfp_ctx* ctx, const double* u, double* work, int reps, int* chosen, void* stream);

/* out = M^{-1}( h [with_source] - D in ).  in, out: device, ndofs doubles,
 * must not overlap (VFP_EINVAL). */
int vfp_apply(vfp_ctx* ctx, const double* in, double* out, int with_source,
              void* stream);

/* One fused Runge-Kutta stage: w_out = u + cdt * L(w_in) (with the source).
 * All three are device arrays of ndofs doubles.  w_in may equal u.  w_out may
 * equal u (each lane reads its own u before writing w_out), but w_out must
 * not overlap w_in, because neighbouring cells still read w_in, and must
 * otherwise be disjoint from u: those cases are rejected with VFP_EINVAL. */
int vfp_stage(vfp_ctx* ctx, const double* w_in, const double* u, double* w_out,
              double cdt, void* stream);

/* Advance u by nsteps explicit fourth-order Runge-Kutta steps of size dt
 * (the four-stage form w_i = u + c_i dt L(w_{i-1}), c = 1/4, 1/3, 1/2, 1,
 * whose step map on this linear, autonomous system is the degree-4 Taylor
 * polynomial of exp(dt L), as for classical RK4).  work: device scratch of
 * 2*ndofs doubles.  u is updated in place.
 * With VFP_CHECK_FINITE=1 in the environment, vfp_advance and
 * vfp_theta_advance check the state for NaN or Inf after their last step
 * (one extra kernel, then a synchronisation of `stream`) and return
 * VFP_EDEVICE if one is found; unset (the default) they do not synchronise. */
int vfp_advance(vfp_ctx* ctx, double* u, double dt, int64_t nsteps,
                double* work, void* stream);

/* ------------------------------------------------------------------ adjoint
 *
 * The linear part of L is  L_lin = -M^{-1} D  (eq. matrix-formulation-system-odes
 * without h).  Its Euclidean transpose is  L_lin^T = -D^T M^{-1}  (M is
 * symmetric).  The reverse-mode calls below run in the variable
 * mu = M^{-1} lambda, where the transposed operator reads
 *     K = M^{-1} L_lin^T M = -M^{-1} D^T,
 * which couples cells through face-node traces only, like the forward
 * operator.  D^T: volume blocks transposed (beta^a symmetric, R^T with
 * Omega^T = -Omega), and on a face from T1 to T2 with B = n.beta (eq.
 * definition-upwind-flux) the blocks B_+ and B_- trade places between the
 * rows: T1 receives B_+ (mu_1 - mu_2), T2 receives -B_- (mu_1 - mu_2).
 *
 * Scattering enters L as -nu_c l(l+1)/2 per coefficient of cell c (the GL(k+1)
 * mass matrix of the collision term cancels against M^{-1}), so
 *     d L(w) / d nu_c = -C w  on the degrees of freedom of cell c.
 */

/* out = M in (inverse = 0) or M^{-1} in (inverse != 0), cell by cell, with M
 * the DG mass matrix of eq. definition-mass-and-dg-matrix.  in may equal out;
 * a partial overlap is rejected with VFP_EINVAL. */
int vfp_mass(vfp_ctx* ctx, const double* in, double* out, int inverse, void* stream);

/* out = -D^T M^{-1} in  (the transpose of the linear part of vfp_apply; the
 * source does not enter).  in, out: device, ndofs doubles, must not overlap.
 * work: caller-owned device scratch of ndofs doubles, disjoint from both; it
 * receives M^{-1} in.  VFP_EINVAL for a NULL pointer or an overlap.  Nothing
 * is allocated. */
int vfp_apply_adjoint(vfp_ctx* ctx, const double* in, double* out, double* work, void* stream);

/* vfp_apply_adjoint without a work argument, for callers that cannot
 * allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc).  The scratch vector M^{-1} in is a fixed
 * library array of VFP_NOALLOC_MAX_NDOFS doubles (64 MiB) per device, held
 * until the process ends; the call allocates and frees nothing.  Results
 * equal vfp_apply_adjoint's to the bit.  VFP_EINVAL if ndofs exceeds
 * VFP_NOALLOC_MAX_NDOFS or the context lives on another device than the
 * current one.  Every call on one device shares that array: calls that
 * overlap in time on a device (other streams, other threads, other
 * contexts) race on it. */
#define VFP_NOALLOC_MAX_NDOFS 8388608
int vfp_apply_adjoint_noalloc(vfp_ctx* ctx, const double* in, double* out, void* stream);

/* One adjoint Runge-Kutta stage in mu variables:
 *     t = cdt K(mu_in);   t_out = t (if t_out != NULL);   acc_out = acc_in + t.
 * If grad_nu != NULL (fwd must then be given), also
 *     grad_nu[c] += -cdt sum_{b, lms in c} (l(l+1)/2) (M mu_in)_{b,lms} fwd_{b,lms}
 * which is d/dnu_c of <M mu_in, cdt L(fwd)>: fwd is the forward stage input
 * that this adjoint stage transposes.  acc_in may equal mu_in; acc_out may
 * equal acc_in; t_out and acc_out must not overlap mu_in, and t_out must not
 * overlap acc_in or acc_out (VFP_EINVAL). */
int vfp_adjoint_stage(vfp_ctx* ctx, const double* mu_in, const double* acc_in, const double* fwd,
                      double cdt, double* t_out, double* acc_out, double* grad_nu, void* stream);

/* Forward steps as vfp_advance, keeping every stage vector: tape holds
 * 4 nsteps ndofs doubles, step s storing w_1, w_2, w_3 and u_{s+1} in slots
 * 4s .. 4s+3.  u0 is read only; the final state is slot 4 nsteps - 1. */
int vfp_advance_tape(vfp_ctx* ctx, const double* u0, double dt, int64_t nsteps, double* tape,
                     void* stream);

/* Reverse sweep over a taped run of nsteps steps from u0 (the same u0, dt and
 * tape as vfp_advance_tape).  On entry mu = M^{-1} dJ/du_nsteps; on exit
 * mu = M^{-1} dJ/du_0.  Because every 4-stage fourth-order scheme has the
 * step map P(dt L_lin) = 1 + dt L_lin + ... + (dt L_lin)^4/24 on this
 * linear autonomous system, each step maps mu to P(dt K) mu.
 * grad_nu (ncells doubles, may be NULL) accumulates dJ/dnu_c; field_slots
 * (vfp_field_grad_size doubles, may be NULL) accumulates the planar-flow
 * sensitivities (see vfp_field_grad_stage).  With both, the dJ/dnu term of
 * each stage is added by the flow-sensitivity launch, which reads the same
 * stage inputs, and the adjoint stages skip the forward state: the per-cell
 * terms are those of vfp_adjoint_stage, added in the same order.
 * work: 3 ndofs doubles. */
int vfp_adjoint_steps(vfp_ctx* ctx, const double* u0, const double* tape, double dt, int64_t nsteps,
                      double* mu, double* grad_nu, double* field_slots, double* work, void* stream);

/* vfp_advance with checkpoints: before each segment of seg steps the current
 * u is copied into ckpt[j] (ckpt: ceil(nsteps/seg) ndofs doubles).  work:
 * 2 ndofs doubles. */
int vfp_forward_checkpoints(vfp_ctx* ctx, double* u, double dt, int64_t nsteps, int64_t seg,
                            double* ckpt, double* work, void* stream);

/* Reverse pass over a checkpointed run: for each segment, last first, the
 * forward steps are replayed from its checkpoint into tape
 * (4 min(seg, nsteps) ndofs doubles) and swept back with vfp_adjoint_steps.
 * lam: on entry dJ/du_nsteps, on exit dJ/du_0 (Euclidean gradients).
 * grad_nu (ncells doubles) and field_slots (vfp_field_grad_size doubles)
 * accumulate, either may be NULL.  work: 3 ndofs doubles.  All buffers must
 * be disjoint. */
int vfp_adjoint_checkpointed(vfp_ctx* ctx, const double* ckpt, double dt, int64_t nsteps, int64_t seg,
                             double* tape, double* lam, double* grad_nu, double* field_slots,
                             double* work, void* stream);

/* Sensitivities to the planar flow of an (x, ln p) context: the arrays
 * u, dudx, dudt (x Gauss points) and u_face (x faces) of
 * vfp_set_flow_planar.  For a stage w_out = u + cdt L(fwd) whose output has
 * the adjoint lambda = M mu, the contribution to dJ/dfield is
 *     cdt <mu, d(h - D fwd)/dfield>,
 * differentiating the volume terms, the upwind x-face flux (speeds
 * U_F + lambda V; Heaviside 1/2 where a speed is exactly 0) and the ln p
 * face flux B_+ f1 + B_- f2 (spectral derivative of B_+) of
 * eq. definition-mass-and-dg-matrix.  vfp_field_grad_stage accumulates it
 * into per-cell slots (device, *n doubles from vfp_field_grad_size,
 * zeroed by the caller before the first stage); vfp_field_grad_reduce sums
 * the slots into g_u, g_dudx, g_dudt (N0 (k+1) doubles each) and g_uface
 * (N0 + 1 doubles), overwriting them.  VFP_EUNSUPPORTED for contexts without
 * an (x, ln p) planar flow.  The derivative tables of B_+ at the ln p faces
 * are built by the context's first vfp_field_grad_support or field-gradient
 * launch (vfp_field_grad_stage, or vfp_adjoint_steps /
 * vfp_adjoint_checkpointed with field_slots): a synchronous host computation
 * and allocation, so make that first call outside stream capture; later
 * set-up calls keep the tables current. */
int vfp_field_grad_size(const vfp_ctx* ctx, int64_t* n);
/* Restrict the U' and dU/dt sensitivities (volume and ln p faces) to the x
 * cells with xcells[i] != 0 (host array of N0 flags; NULL: every cell, the
 * default): they are formed on every such cell and on the cells that share
 * a kernel tile (a run of consecutive cells) with one, and the slots of the
 * other cells are left untouched; dJ/dU and dJ/dU_face are formed
 * everywhere.  For a caller whose
 * parameters move U' and dU/dt only on some cells (a tanh shock: its U' and
 * every parameter derivative of U' and U U' vanish exactly where
 * 1 - tanh^2(x/w) rounds to 0), the skipped contributions are multiplied
 * by zero in the chain rule anyway.  Set-up call (synchronous); a new mesh
 * drops it. */
int vfp_field_grad_support(vfp_ctx* ctx, const unsigned char* xcells);
int vfp_field_grad_stage(vfp_ctx* ctx, const double* mu, const double* fwd, double cdt, double* slots,
                         void* stream);
int vfp_field_grad_reduce(vfp_ctx* ctx, const double* slots, double* g_u, double* g_dudx, double* g_dudt,
                          double* g_uface, void* stream);

/* ------------------------------------------------------ reconstruction
 *
 * The distribution function from its coefficients (eq. spherical-harmonic-exp):
 * f(x, p, theta, phi) = sum_lms f_lms(x, p) Y_lms(theta, phi), with the real
 * spherical harmonics of App. A (eq. spherical-harmonics,
 * eq. normalisation-spherical-harmonics, Condon-Shortley phase inside P_l^m
 * as in eq. associated-legendre-polynomials), theta measured from the x axis
 * and phi about it: p/p = (cos theta, sin theta cos phi, sin theta sin phi).
 */

/* Host only: Y[d n + lms] = Y_lms(theta[d], phi[d]) for d < ndir,
 * n = (lmax+1)^2, 0 <= lmax <= 11 (host arrays). */
int vfp_sh_eval(int lmax, int64_t ndir, const double* theta, const double* phi, double* Y);

/* f at every basis node of every cell in ndir directions:
 * out[row ndir + d] = sum_lms zeta[row n + lms] Y[d n + lms], row = cell nb + basis
 * (nb = (k+1)^naxes).  zeta (ndofs doubles), Y (ndir n doubles, e.g. from
 * vfp_sh_eval) and out (ncells nb ndir doubles) are device arrays. */
int vfp_reconstruct(const vfp_ctx* ctx, const double* zeta, const double* Y, int64_t ndir, double* out,
                    void* stream);

/* --------------------------------------------------- implicit time steps
 *
 * The Theta-method of eq. theta-method: each step solves the linear system
 * of eq. system-matrix-rhs,
 *     (M + dt Theta D) zeta^n = (M - dt (1 - Theta) D) zeta^{n-1} + dt h,
 * (fields, and so D and h, constant in time), Theta in [0, 1]: 0 forward
 * Euler, 1/2 Crank-Nicolson, 1 backward Euler.  The library solves the same
 * system multiplied by the block-diagonal M^{-1} (exact per cell),
 *     (I - dt Theta L0) zeta^n = zeta^{n-1} + dt (1 - Theta) L(zeta^{n-1}) + dt Theta M^{-1} h,
 * with L0 = L without the source, by restarted GMRES (classical
 * Gram-Schmidt, repeated for a Krylov vector where the first pass removes
 * more than half of its squared norm) whose operator is the fused
 * stage kernel; the iterate starts at zeta^{n-1}.  A step is accepted when
 * the true residual norm is at most tol times the right-hand side's
 * (Euclidean norms).
 */
#define VFP_PRECOND_NONE      0
#define VFP_PRECOND_COLLISION 1   /* right preconditioner 1 / (1 + dt Theta nu_c l(l+1)/2) per
                                     DoF: the exact inverse of the scattering part of the
                                     system (the inverse mass reduces it to that factor) */
#define VFP_PRECOND_XLINE     2   /* right preconditioner: the exact inverse of the system's
                                     block-tridiagonal part along axis 0 (each cell's own
                                     block and its blocks towards its two neighbours along
                                     axis 0; a periodic wrap is left out), one block
                                     recurrence per line of cells along axis 0.  The blocks
                                     are taken from the operator itself at the start of the
                                     call (3 ncolours (k+1)^d n stage applications) and
                                     factorised on the device.  Needs (k+1)^d n <= 48 and
                                     vfp_theta_precond_size extra doubles of work */

typedef struct vfp_theta_opts {
  double theta;       /* in [0, 1]                                            */
  double tol;         /* relative residual, > 0                               */
  int restart;        /* Krylov vectors per cycle, 1 .. 64                    */
  int max_iters;      /* Krylov iterations per step, >= 1                     */
  int precond;        /* VFP_PRECOND_*                                        */
} vfp_theta_opts;

typedef struct vfp_theta_stats {
  int64_t iterations; /* Krylov iterations over all steps                     */
  double residual;    /* largest final relative residual over the steps       */
  int converged;      /* 1 if every step met tol within max_iters             */
} vfp_theta_stats;

/* Doubles of device work space for vfp_theta_advance with `restart` vectors:
 * (restart + 5) ndofs plus a fixed reduction area. */
int vfp_theta_work_size(const vfp_ctx* ctx, int restart, int64_t* n);

/* Extra doubles of work a preconditioner needs, after the vfp_theta_work_size
 * part: 0 for VFP_PRECOND_NONE and VFP_PRECOND_COLLISION; for
 * VFP_PRECOND_XLINE three b x b blocks per cell (b = (k+1)^d n) and a flag per
 * line; VFP_EUNSUPPORTED where b > 48. */
int vfp_theta_precond_size(const vfp_ctx* ctx, int precond, int64_t* n);

/* Advance u (device, ndofs doubles, in place) by nsteps Theta-method steps.
 * work: device, at least vfp_theta_work_size + vfp_theta_precond_size doubles
 * (work_len), disjoint from u; with VFP_PRECOND_XLINE the call first builds
 * the preconditioner for its dt and Theta (synchronising `stream` once) and
 * fails with VFP_EDEVICE if a block is singular.  Unlike the other compute calls this one synchronises `stream`
 * once per Krylov iteration (the Hessenberg least-squares problem is solved
 * on the host; the first call on a context also allocates a 1.7 KB pinned
 * host buffer for those read-backs, kept until vfp_destroy).  stats (host,
 * may be NULL) reports the iterations and residuals; a step that does not
 * reach tol within max_iters keeps its last iterate, the run continues, and
 * stats->converged is 0.  Calls on one context that overlap in time race on
 * that buffer. */
int vfp_theta_advance(vfp_ctx* ctx, double* u, double dt, int64_t nsteps, const vfp_theta_opts* opts,
                      double* work, int64_t work_len, vfp_theta_stats* stats, void* stream);

/* ------------------------------------------------------------------ batches
 *
 * Many independent runs (each its own context: mesh, l_max, k, fields, time
 * step) advanced together.  The runs are grouped into classes of equal
 * (k, l_max, rows of B.Omega); for the (x, ln p) runs of Sec. 4.4 one launch
 * per Runge-Kutta stage and class walks the (run, tile) items of all its
 * runs, other runs are launched one by one.  Each run's arithmetic is the
 * same as vfp_advance's, so results agree with the runs advanced alone to
 * the last bit.
 */
typedef struct vfp_batch vfp_batch;

#define VFP_BATCH_GRAPH 1u   /* replay each step as a captured HIP graph */

/* Group nruns ready contexts (all on one device, none repeated).  The batch
 * borrows the contexts: they must outlive it.  A set-up call (vfp_set_*) on
 * a run after vfp_batch_bind makes vfp_batch_advance and vfp_batch_autotune
 * return VFP_ESTATE, before any launch, until the batch is bound again. */
int vfp_batch_create(vfp_batch** out, vfp_ctx* const* runs, int nruns, unsigned flags);

void vfp_batch_destroy(vfp_batch* b);

/* Bind the state u[r] (ndofs_r doubles) and work[r] (2 ndofs_r doubles,
 * disjoint from u[r]) device buffers and the time step dt[r] of every run
 * (host arrays of nruns entries).  Synchronous (uploads the per-run stage
 * descriptors); drops a captured graph. */
int vfp_batch_bind(vfp_batch* b, double* const* u, double* const* work, const double* dt);

/* Advance every bound run by nsteps Runge-Kutta steps (as vfp_advance).
 * With VFP_BATCH_GRAPH the first call captures one step into a graph on a
 * private stream, ordered after `stream` by events, and later calls replay
 * it; `stream` waits for the replays. */
int vfp_batch_advance(vfp_batch* b, int64_t nsteps, void* stream);

/* Time the batched kernel of every class over the bound buffers, on a
 * step's mix of stage forms (the first stage, which reads u and writes the
 * first work vector, and three that read a work vector and u and write the
 * other; u is unchanged), reps repetitions per candidate over two rounds
 * keeping each candidate's faster one, for each workgroup shape (lanes per workgroup:
 * 64 / 128 / 256 where n = (l_max+1)^2 divides 64, else 256 / 64 / 128;
 * cells per tile follow) and each tile order -- launch order, or each of the
 * 8 XCDs taking one contiguous range of tiles -- and keep the fastest.
 * Results do not depend on the choice (each cell's arithmetic is the same).
 * Synchronises `stream`; drops a captured graph. */
int vfp_batch_autotune(vfp_batch* b, int reps, void* stream);

/* Number of classes, and for class i: info[0..7] = k, l_max, rows of B.Omega,
 * runs, batched (1/0), tiles (= workgroups per launch), lanes per workgroup
 * (the tuned shape; 0 for runs launched one by one), tile order (1: XCD
 * ranges). */
int vfp_batch_nclasses(const vfp_batch* b);
int vfp_batch_class_info(const vfp_batch* b, int i, int* info);

#ifdef __cplusplus
}
#endif

#endif /* VFP_H */
