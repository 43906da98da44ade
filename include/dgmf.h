/*
 * dgmf: matrix-free discontinuous Galerkin operators on tensor-product
 * hexahedra for AMD Instinct MI355X (gfx950).
 *
 * The operations follow Krank, Fehn, Wall & Kronbichler, "A high-order
 * semi-explicit discontinuous Galerkin solver for 3D incompressible flow with
 * application to DNS and LES of turbulent channel flow" (arXiv:1607.01323):
 *   - nodal Lagrange basis of tensor degree k on Gauss-Lobatto nodes
 *     (Sec. 3.1), Gauss quadrature with k+1 points per direction for the
 *     linear forms and over-integration for the convective term (Sec. 5);
 *   - the symmetric interior penalty (SIPG) Laplace operator of the pressure
 *     Poisson step and the Helmholtz operator of the viscous step in its
 *     scalar form (Sec. 3.2, eqs. poissonspat, ipflux, taue, tau; matrix
 *     form Sec. 4.4, eqs. poissonmat and viscous);
 *   - preconditioned conjugate gradients with matrix-free products, point
 *     Jacobi, a Chebyshev polynomial preconditioner or a geometric multigrid
 *     V-cycle with Chebyshev smoothing, in single precision, and the
 *     zero-mean projection of singular problems (Sec. 5.1);
 *   - the divergence-form convective operator with the local Lax-Friedrichs
 *     flux, Lambda evaluated per face quadrature point (Sec. 3.2, eq.
 *     convstepspat; matrix form eq. advect), its vector-Jacobian product,
 *     and the explicit convective substep with the tensorial inverse of the
 *     block-diagonal mass matrix (Sec. 4 matrix formulation, Sec. 5);
 *   - the divergence and gradient operators, the div-div penalty and the
 *     element-local projection of variant V3c (Sec. 4.2, Sec. 5.1).
 *
 * Conventions shared by every entry point
 *   Reference cell [0,1]^3, n = k+1 nodes per direction.
 *   Cell index c = (cz*ny + cy)*nx + cx.
 *   DoF index g = c*n^3 + (l*n + j)*n + i (x node index i fastest).
 *   Vector fields are component-major: [3][N], N = n_cells * n^3.
 *   All vector arguments are DEVICE pointers on the device that was current
 *   when the handle was created, contiguous, of the dtype the call states,
 *   owned by the caller.  The library never keeps a pointer past the work it
 *   enqueues; the caller keeps buffers alive until the stream passes it.
 *   Work is enqueued on the given hipStream_t (0 = the null stream) and the
 *   call returns without waiting unless it says otherwise.
 *   Calls that build something on first use (a multigrid hierarchy, the
 *   curved-cell metric of the V3c operators) change the handle: the first
 *   such call on one handle must not overlap another call on it from a
 *   different host thread; later calls only read the handle.
 *
 * Errors: every function returns a dgmf_status; no exception crosses the
 * ABI.  Argument errors are detected before anything is enqueued and leave
 * outputs untouched.  dgmf_last_error() returns a thread-local message for
 * the last non-OK status of the calling thread.  Launch failures are reported
 * as DGMF_HIP_ERROR; device faults surface at the next synchronising call.
 */
#ifndef DGMF_H
#define DGMF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DGMF_OK = 0,
  DGMF_INVALID = 1,        /* bad argument: null/misaligned pointer, size, degree, dtype */
  DGMF_HIP_ERROR = 2,      /* a HIP runtime call or kernel launch failed */
  DGMF_OOM = 3,            /* device allocation failed */
  DGMF_NOT_CONVERGED = 4,  /* CG reached max_iter; outputs hold the last iterate */
  DGMF_BREAKDOWN = 5,      /* CG: <r,z> <= 0 or <p,Ap> <= 0 (preconditioner/operator not SPD) */
  DGMF_NONFINITE = 6,      /* CG: NaN/Inf in the data or in a scalar of the iteration */
  DGMF_UNSUPPORTED = 7     /* valid request outside what the library implements */
} dgmf_status;

typedef enum { DGMF_F64 = 0, DGMF_F32 = 1 } dgmf_dtype;

typedef struct dgmf_mesh_* dgmf_mesh;  /* opaque, library-owned */
typedef struct dgmf_op_* dgmf_op;      /* opaque, library-owned */

/* Thread-local text of the last error of the calling thread ("" if none). */
const char* dgmf_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int dgmf_version(void);

/* ---------------------------------------------------------------- mesh --- */
/* Box [0,lx] x [y0,y0+ly] x [0,lz] of nx*ny*nz affine hexahedra (Sec. 3.1).
 * periodic[d] = 1: faces at both ends of direction d are identified and
 * treated as interior faces; 0: both ends are Dirichlet boundaries.
 * y_tanh_gamma > 0 grades the y vertices with the hyperbolic mapping of
 * Sec. 7.1, y = y0 + ly/2 (1 + tanh(gamma (2t-1)) / tanh(gamma)), t in [0,1].
 * store_qp_metric = 1 makes SIPG operators on this mesh store and stream the
 * geometry at every quadrature point (w detJ J^{-1}J^{-T}, w detJ; on faces
 * w dA and J^{-1}n w dA of both cells) instead of using the per-cell constant
 * metric of axis-aligned cells (then periodic directions need >= 2 cells).
 * shear: row-major 3x3 matrix S applied to every point of the box, x = S p
 * (a constant affine lattice, so cells are parallelepipeds); all zeros means
 * the identity.  A non-identity shear needs store_qp_metric = 1 and is not
 * supported by the convective operator.
 * neumann[2d+s] = 1 makes the boundary side s (0 low, 1 high) of a
 * non-periodic direction d a homogeneous Neumann boundary, 0 (default) a
 * Dirichlet one; ignored in periodic directions.  Sec. 3.2: on such faces the
 * flux takes the cell's own trace and the gradient flux is data, so the SIPG
 * operator has no face term there (the pressure Poisson operator on the walls
 * of a velocity-Dirichlet domain, the viscous operator on an outflow); their
 * area still counts in tau_e (eq. taue).  For the convective operator such a
 * side is an outflow: the flux is F^c of the own trace (exterior state u+ = u-).
 * The divergence and gradient operators take the own trace on both boundary
 * parts (the ND average of Sec. 3.1), and the viscous operator in the
 * symmetric-gradient form has no term on a Neumann side either (U* = u_h
 * there, the flux F^nu* is data); every operator accepts Neumann sides.
 * curve_amp = a != 0 makes the cells iso-parametric and curved (Sec. 5): the
 * box point p (after the tanh grading) moves to
 *   x = p + a (lx s(t_y) s(t_z), ly s(t_z) s(t_x), lz s(t_x) s(t_y)),
 * s(t) = sin(2 pi t), t = (p - (0, y0, 0)) / (lx, ly, lz), and each cell's map is
 * the degree-k interpolant of x at its GLL nodes.  The map is periodic in every
 * direction; walls of non-periodic directions become curved.  |a| <= 0.1;
 * needs store_qp_metric = 1 and no shear.  Curved meshes serve the SIPG
 * operator, its diagonal, CG with every preconditioner (multigrid keeps the
 * curved operator on the finest level and rediscretises the coarse levels on
 * the undeformed box), the mass matrix and its inverse (with the point
 * weights w_q det J_q), the convective operator and its VJP, the V3c
 * divergence, gradient, div-div penalty and local projection, the viscous
 * operator in the symmetric-gradient form and its CG (with the Jacobian at
 * every quadrature point), node and quadrature-point coordinates and load
 * vectors; the fused convective substep returns DGMF_UNSUPPORTED on them.
 * degree k in 1..7; every cell count >= 1; lengths > 0. */
typedef struct {
  int degree;
  int nx, ny, nz;
  double lx, ly, lz;
  double y0;
  int periodic[3];
  double y_tanh_gamma;
  int store_qp_metric;
  double shear[9];
  int neumann[6];
  double curve_amp;
} dgmf_box_desc;

/* Allocates device geometry on the current device.  *out receives the handle. */
dgmf_status dgmf_mesh_create(const dgmf_box_desc* desc, dgmf_mesh* out);
/* Host outputs (either may be NULL). */
dgmf_status dgmf_mesh_info(dgmf_mesh mesh, int64_t* n_cells, int64_t* n_dofs_per_field);
/* Physical coordinates of every DoF: xyz is a device double array [3][N]
 * (on curved cells the deformed node positions, which the cell maps
 * interpolate). */
dgmf_status dgmf_mesh_node_coords(dgmf_mesh mesh, double* xyz, hipStream_t stream);
/* dst = M^{-1} src for n_fields consecutive scalar fields ([n_fields][N],
 * dtype DGMF_F64 or DGMF_F32), M the block-diagonal DG mass matrix of the
 * nodal basis, (phi_i, phi_j)_K with k+1 Gauss points per direction (exact on
 * these affine cells).  Applied per cell through the tensorial inverse of
 * Sec. 5 (implementation): the inverted 1D node-to-Gauss-point transform and
 * inverse weights, Mh^{-1} = S^{-1} W^{-1} S^{-T} along each direction, times
 * 1/|det J|.  This is the M^{-1} of the explicit convective step (Sec. 4,
 * matrix formulation, eq. advect) and of the inverse-mass preconditioners of
 * Sec. 5.1.  n_fields in 1..64; src == dst (in place) is allowed, any other
 * overlap is DGMF_INVALID.  Asynchronous. */
dgmf_status dgmf_inverse_mass_apply(dgmf_mesh mesh, dgmf_dtype dtype, int n_fields, const void* src, void* dst,
                                    hipStream_t stream);
/* dst = M src, the block-diagonal mass matrix of dgmf_inverse_mass_apply
 * itself (|det J| (Mh (x) Mh (x) Mh) per cell); the M U-hat term of the
 * projection's right-hand side (Sec. 4, eq. project).  Same arguments and
 * rules as dgmf_inverse_mass_apply.  Asynchronous. */
dgmf_status dgmf_mass_apply(dgmf_mesh mesh, dgmf_dtype dtype, int n_fields, const void* src, void* dst,
                            hipStream_t stream);

/* ------------------------------------------------- variant V3c (fp64) --- */
/* Operators of the projection and pressure steps of variant V3c (Sec. 4.2,
 * V3b/V3c; matrix form Sec. 4, eqs. poissonmat and project) on axis-aligned
 * meshes (sheared meshes: DGMF_UNSUPPORTED).  Averages are central on
 * interior faces; on boundary faces the cell's own trace is used (the ND
 * extension of Sec. 3.1).  All vectors are device fp64; [3][N] for vector
 * fields, [N] for scalar fields, [n_cells] for per-cell values. */
/* out = A u, the divergence of eq. av3 without the factor gamma_0/dt:
 * (A u)_i = sum_K (grad phi_i, u)_K - (phi_i, {{u}}.n)_dK.  u [3][N],
 * out [N]; must not overlap.  Asynchronous, except that on a mesh with
 * curved cells the first call of this or dgmf_gradient_apply fills (on the
 * device, synchronously) a per-point metric of 8 (9 n^3 + 18 n^2) bytes per
 * cell, n = k+1, held by the mesh: there both operators integrate with k+1
 * Gauss points per direction and the Jacobian at every point. */
dgmf_status dgmf_divergence_apply(dgmf_mesh mesh, const double* u, double* out, hipStream_t stream);
/* out = B p, the gradient of eq. bv3 without the factor dt/gamma_0:
 * (B p)_{i,a} = sum_K (d_a phi_i, p)_K - (phi_i, {{p}} n_a)_dK.  p [N],
 * out [3][N]; must not overlap.  On periodic affine meshes B = -A^T (on
 * curved cells only up to the quadrature error).  Asynchronous, with the
 * first-call metric fill on curved meshes as for dgmf_divergence_apply. */
dgmf_status dgmf_gradient_apply(dgmf_mesh mesh, const double* p, double* out, hipStream_t stream);
/* tau[c] = zeta |u_bar_c| V_c^(1/3) dt (eq. tauD), u_bar_c the volume average
 * of the velocity u [3][N] on cell c; zeta, dt finite and >= 0 (the paper
 * takes zeta = 1/CFL).  Asynchronous (curved meshes: k+1 Gauss points per
 * direction with w |det J| per point, and the first-call metric fill of
 * dgmf_divergence_apply). */
dgmf_status dgmf_divdiv_penalty(dgmf_mesh mesh, const double* u, double zeta, double dt, double* tau,
                                hipStream_t stream);
/* Solves the local projection of eq. project with the div-div penalty only
 * (V3, tau_C = 0): on every cell (M_e + tau[c] D_e) x_e = rhs_e with
 * D_e = (div v, div u)_K (eq. div-div), by CG preconditioned with the inverse
 * cell mass, one independent iteration per cell (Sec. 5.1, projection
 * solver), started from x on entry and stopped when that cell's residual is
 * at most rtol times its right-hand side or after max_iter iterations.  rhs,
 * x [3][N] (x in/out; must not overlap rhs); tau [n_cells] >= 0;
 * iterations: device int [n_cells] receiving each cell's iteration count, or
 * NULL.  Degrees k <= 6.  Asynchronous.  On curved meshes M_e and D_e take
 * k+1 Gauss points per direction and the Jacobian at every point, the
 * preconditioner is the point inverse mass S^{-1} diag(1/(w |det J|)) S^{-T}
 * per direction, and the first call fills the metric as
 * dgmf_divergence_apply does. */
dgmf_status dgmf_projection_solve(dgmf_mesh mesh, const double* tau, const double* rhs, double* x, double rtol,
                                  int max_iter, int* iterations, hipStream_t stream);

/* Frees the mesh; operators created on it must be destroyed first (DGMF_INVALID otherwise). */
dgmf_status dgmf_mesh_destroy(dgmf_mesh mesh);

/* ------------------------------------------------------------ SIPG op --- */
/* Operator H = mass_coeff * M + diff_coeff * A, A the SIPG Laplacian of
 * Sec. 3.2 with homogeneous Dirichlet data on Dirichlet faces (boundary
 * penalty 2 tau); tau_e = penalty_scale (k+1)^2 (A_int/2 + A_Dir)/V
 * (eq. taue), tau_F = max over the two cells (eq. tau).  The paper's choice is
 * penalty_scale = 1.  n_q must be 0 or k+1 (Sec. 5: k+1 Gauss points). */
typedef struct {
  double mass_coeff;     /* mu = gamma_0 / dt; 0 for the Laplacian */
  double diff_coeff;     /* nu; 1 for the Laplacian */
  double penalty_scale;  /* s in tau_e */
  int n_q;               /* 0 -> k+1 */
} dgmf_sipg_desc;

dgmf_status dgmf_sipg_create(dgmf_mesh mesh, const dgmf_sipg_desc* desc, dgmf_op* out);
/* dst = H src.  src, dst: device arrays of N values of the given dtype;
 * must not alias.  Asynchronous on stream. */
dgmf_status dgmf_operator_apply(dgmf_op op, dgmf_dtype dtype, const void* src, void* dst, hipStream_t stream);
/* out = H_eps u for a velocity u [3][N] (fp64): the viscous operator of the
 * implicit viscous step in its symmetric-gradient form (Sec. 3.2, s = 1,
 * F^nu(u) = 2 nu eps(u), fluxes U* and F^nu* with penalty tau nu, boundary
 * faces with g_u = 0 and penalty 2 tau nu), plus mass_coeff M, with the
 * operator's coefficients and penalty.  Computed as this operator applied to
 * every component plus nu times the component coupling.  Axis-aligned and
 * curved cells (curved: the stored-metric apply per component, the coupling
 * with the Jacobian of the cell map evaluated at every Gauss point of cells
 * and faces; sheared: DGMF_UNSUPPORTED).  u, out must not overlap.
 * Asynchronous (curved meshes upload small tables on the first call). */
dgmf_status dgmf_viscous_apply(dgmf_op op, const double* u, double* out, hipStream_t stream);

/* diag = diag(H), N values of dtype.  Asynchronous. */
dgmf_status dgmf_operator_diagonal(dgmf_op op, dgmf_dtype dtype, void* diag, hipStream_t stream);
/* Cell quadrature points of the operator's rule: xyz device double [3][n_cells*n_q^3],
 * point index c*n_q^3 + (qz*n_q + qy)*n_q + qx (curved cells: the cell map
 * at the Gauss points).  Asynchronous. */
dgmf_status dgmf_quadrature_points(dgmf_op op, double* xyz, hipStream_t stream);
/* b_i = sum_K (f, phi_i)_K by the operator's Gauss rule, f given at the
 * quadrature points (layout of dgmf_quadrature_points), fp64.  This is the
 * load vector of the right-hand sides in Sec. 4.4; on curved cells with the
 * point weights w_q det J_q.  Asynchronous. */
dgmf_status dgmf_integrate(dgmf_op op, const double* f_qp, double* b, hipStream_t stream);

/* ------------------------------------------------------------------ CG --- */
/* Preconditioned CG on H x = b (Sec. 5.1).  Convergence when
 * ||r_k||_2 <= rtol ||b||_2 on the recursive residual (b projected first when
 * project_mean).  precond 0: point Jacobi in fp64.  precond 1: Chebyshev
 * acceleration of point Jacobi, error polynomial of degree cheb_degree on
 * [lambda/smoothing_range, lambda] started from zero (cheb_degree-1 operator
 * products in precond_dtype), lambda = lambda_safety * the largest Ritz value
 * of lanczos_steps Lanczos steps on D^{-1/2} H D^{-1/2} in precond_dtype from
 * a SplitMix64(seed) start vector (mean removed when project_mean); the Ritz
 * value is kept with the operator and reused by later solves with the same
 * precond_dtype, lanczos_steps, seed and project_mean.  With
 * precond_dtype DGMF_F32 the preconditioner runs in fp32 while residual, dot
 * products and updates stay fp64 (mixed precision).  project_mean = 1
 * projects b and every operator product onto zero-mean vectors (singular
 * periodic Laplacian).  check_every: iterations between host reads of the
 * convergence flag (the iteration count is exact regardless).  flexible
 * selects the Polak-Ribiere beta (flexible CG, Notay 2000), which tolerates
 * the slight non-linearity of a preconditioner evaluated in fp32.
 * precond 2: one V-cycle of geometric multigrid in precond_dtype (Sec. 5.1,
 * Poisson solver) over the hierarchy that halves every even cell count until
 * none is even, the operator discretised anew on every level (coarse levels
 * use the per-cell metric of axis-aligned cells; sheared meshes are
 * DGMF_UNSUPPORTED).  Smoother before and after the coarse correction: the
 * Chebyshev-Jacobi polynomial above (cheb_degree, smoothing_range,
 * lanczos_steps, lambda_safety; level l uses seed + l).  Coarse solver:
 * Chebyshev-Jacobi from zero on [theta_min / lambda_safety, lambda_safety
 * theta_max] (fp64 Lanczos with full re-orthogonalisation, at most 64 steps,
 * the null vector deflated when project_mean) with the smallest degree whose
 * Chebyshev error estimate 1/T_m((b+a)/(b-a)) is below mg_coarse_tol
 * (0 -> 1e-3; at most 2000).  Transfers: the mother cell's polynomial
 * evaluated at its children's nodes (reference-cell embedding) and its
 * transpose.  The hierarchy (level meshes, operators, vectors, eigenvalue
 * estimates) is built on the first call and kept with the operator until
 * dgmf_op_destroy or a call with different preconditioner parameters. */
typedef struct {
  double rtol;
  int max_iter;
  int check_every;
  int precond;           /* 0 Jacobi, 1 Chebyshev, 2 geometric multigrid V-cycle, 3 inverse mass
                            matrix (fp64; the viscous-step preconditioner of Sec. 5.1) */
  int precond_dtype;     /* dgmf_dtype of the Chebyshev preconditioner */
  int cheb_degree;       /* >= 1 */
  double smoothing_range;/* > 1 */
  int lanczos_steps;     /* 2..64 */
  double lambda_safety;  /* >= 1 */
  uint64_t seed;
  int project_mean;
  int flexible;          /* 0: beta = <r+,z+>/<r,z> (Fletcher-Reeves); 1: beta = <z+, r+ - r>/<r,z>
                            (Polak-Ribiere, flexible CG: robust to the rounding of an fp32 preconditioner) */
  double mg_coarse_tol;  /* precond 2: coarse Chebyshev error estimate target, 0 -> 1e-3 */
  int mg_graph;          /* precond 2: 1 replays the V-cycle from a captured HIP graph (kept with the
                            hierarchy, one per workspace), 0 launches it kernel by kernel */
} dgmf_cg_params;

typedef struct {
  int iterations;
  double rel_residual;   /* ||r_k|| / ||b|| of the recursive residual */
  double lambda_max;     /* lambda used by the Chebyshev preconditioner (0 for Jacobi) */
  int status;            /* dgmf_status of the solve */
  double setup_s;        /* seconds in diagonal + eigenvalue estimate */
  double solve_s;        /* seconds in the iteration */
} dgmf_cg_result;

/* Bytes of device workspace dgmf_cg_solve needs for these parameters. */
dgmf_status dgmf_cg_workspace_bytes(dgmf_op op, const dgmf_cg_params* params, size_t* bytes);
/* b: device fp64 [N]; x: device fp64 [N], initial guess on entry, solution on
 * exit.  workspace: device memory of at least the queried size, 256-byte
 * aligned.  Synchronous: returns after the work on stream has finished;
 * *out (host) is filled on every path past argument validation, and the
 * returned status equals out->status. */
dgmf_status dgmf_cg_solve(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params,
                          void* workspace, size_t workspace_bytes, hipStream_t stream,
                          dgmf_cg_result* out);
/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation):
 * dgmf_cg_solve with its workspace taken from a static buffer of the library
 * (DGMF_CG_NOALLOC_MAX_BYTES per device, held by every device the library
 * runs on from module load to the end of the process), so the call allocates
 * no device memory.  Arguments, results and synchronisation as for
 * dgmf_cg_solve, without the workspace.  precond 0, 1 and 3 only (the
 * multigrid hierarchy of precond 2 is allocated on first use:
 * DGMF_UNSUPPORTED); a workspace need (dgmf_cg_workspace_bytes) above
 * DGMF_CG_NOALLOC_MAX_BYTES is DGMF_INVALID.  Every call on one device shares
 * that device's buffer and leaves its contents behind; calls on one device
 * are serialised by a lock held for the whole (synchronous) solve, so calls
 * from several host threads run one after the other, and the buffer is
 * rewritten before it is read.  b and x must not lie in the buffer. */
#define DGMF_CG_NOALLOC_MAX_BYTES ((size_t)64 << 20)
dgmf_status dgmf_cg_solve_noalloc(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params,
                                  hipStream_t stream, dgmf_cg_result* out);
/* The implicit viscous step in the symmetric-gradient form (Sec. 3.2; the
 * solver of Sec. 5.1): H_eps x = b with H_eps the operator of
 * dgmf_viscous_apply, by fp64 CG preconditioned with the inverse diagonal of
 * this operator's scalar part on every component (precond 0) or with the
 * inverse mass matrix on every component (precond 3, the paper's viscous
 * preconditioner).  params: rtol (stop on ||r|| <= rtol ||b||), max_iter,
 * check_every, precond (0 or 3, else DGMF_UNSUPPORTED); the other fields
 * are ignored.  b, x: device fp64 [3][N]
 * (x: initial guess in, solution out); workspace: device memory of at least
 * dgmf_viscous_cg_workspace_bytes, 256-byte aligned; none may overlap.
 * Curved cells: the curved operator, and for precond 3 the point-weight
 * inverse mass.  Meshes with shear: DGMF_UNSUPPORTED.
 * Synchronous like dgmf_cg_solve: *out is filled and the returned status
 * equals out->status (NOT_CONVERGED, BREAKDOWN, NONFINITE on failure). */
dgmf_status dgmf_viscous_cg_workspace_bytes(dgmf_op op, size_t* bytes);
dgmf_status dgmf_viscous_cg_solve(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params,
                                  void* workspace, size_t workspace_bytes, hipStream_t stream,
                                  dgmf_cg_result* out);

/* z = B r, one application of the multigrid preconditioner (params->precond
 * must be 2; other fields as for dgmf_cg_solve), no mean projection.  r, z:
 * device fp64 [N], must not overlap.  Builds the hierarchy synchronously on
 * first use, then asynchronous on stream. */
dgmf_status dgmf_precond_apply(dgmf_op op, const dgmf_cg_params* params, const double* r, double* z,
                               hipStream_t stream);
/* Host outputs of the operator's multigrid hierarchy (any may be NULL):
 * number of levels, lambda of every level's smoother (host array of at
 * least 32 entries; the coarsest entry is the upper end of its interval), the
 * coarse Chebyshev degree and interval [lo, hi].  DGMF_INVALID before the
 * hierarchy exists. */
dgmf_status dgmf_precond_info(dgmf_op op, int* levels, double* lambdas, int* coarse_degree,
                              double* coarse_interval);

/* ---------------------------------------------------------- convective --- */
/* Convective operator C(U)_{i,a} = -sum_K (d_b phi_i, u_a u_b)_K
 *   + sum_K (phi_i, R_a)_{dK}, R = 1/2 (u-(u-.n) + u+(u+.n)) + lam (u- - u+),
 * lam = max(|u-.n|, |u+.n|) per face quadrature point (Sec. 3.2); Dirichlet
 * faces use the mirror state u+ = 2g - u- with g = 0, outflow (Neumann) sides
 * the own state u+ = u- (flux F^c(u-).n).  n_q Gauss points per direction on
 * cells and faces; 0 -> floor(3(k+1)/2).  On curved cells (Sec. 5) create
 * fills, on the device and synchronously, a per-point metric: w |det J| J^{-1}
 * at every cell point and the weighted normal w dA n at every face point, of
 * 8 (9 n_q^3 + 18 n_q^2) bytes per cell, owned by the operator. */
typedef struct { int n_q; } dgmf_conv_desc;

dgmf_status dgmf_convective_create(dgmf_mesh mesh, const dgmf_conv_desc* desc, dgmf_op* out);
/* out = C(u); u, out: device fp64 [3][N], must not alias.  Asynchronous. */
dgmf_status dgmf_convective_apply(dgmf_op op, const double* u, double* out, hipStream_t stream);
/* out = u - dt M^{-1} C(u): one explicit convective substep of the matrix
 * form (Sec. 4, matrix formulation, eq. advect, with gamma_0 = alpha_0 =
 * beta_0 = 1 and no body force), M the block-diagonal mass matrix as in
 * dgmf_inverse_mass_apply.  Fused: C(u) stays on chip.  Higher-order
 * combinations sum_i alpha_i U^{n-i} - dt M^{-1} sum_i beta_i F^c(U^{n-i})
 * follow from dgmf_convective_apply, dgmf_inverse_mass_apply and vector
 * sums.  u, out: device fp64 [3][N], must not overlap; dt finite.
 * Curved cells (no block-diagonal mass): DGMF_UNSUPPORTED; there the same
 * step is dgmf_convective_apply followed by dgmf_inverse_mass_apply.
 * Asynchronous. */
dgmf_status dgmf_convective_step(dgmf_op op, double dt, const double* u, double* out, hipStream_t stream);
/* grad = (dC/du)^T w; u, w, grad: device fp64 [3][N]; grad must not alias
 * u or w.  Tie rule of the max: the minus side is active when
 * |u-.n| >= |u+.n|; sgn(0) = 0.  Asynchronous. */
dgmf_status dgmf_convective_vjp(dgmf_op op, const double* u, const double* w, double* grad,
                                hipStream_t stream);

/* Frees any operator handle. */
dgmf_status dgmf_op_destroy(dgmf_op op);

#ifdef __cplusplus
}
#endif
#endif /* DGMF_H */
