/*
 * feti.h — C ABI of the MI355X FETI solver library (libfeti.so).
 *
 * The library solves the torn linear(ised) elasticity systems of the
 * classical and the all-floating FETI methods of Augustin, Holzapfel and
 * Steinbach, "Classical and all-floating FETI methods for the simulation of
 * arterial tissues" (IJNME 99, 2014):
 *
 *   K_i u_i + B_i^T lambda = f_i  (every subdomain i),   sum_i B_i u_i = b,
 *
 * section 4, eqs. (classicalFetiLGS) and (AFFETI), by the projected
 * preconditioned CG on the dual problem P^T F lambda = P^T d (eq.
 * (dualProblem)) with F = sum B_i K_i^+ B_i^T, G = [B_i R_i] and the
 * projection P = I - G (G^T G)^{-1} G^T (eq. (projection)).  Nonlinear
 * problems (Holzapfel-Gasser-Ogden tissue, section 2) are linearised by Newton
 * (section 3.2, eqs. (NewtonRecursion), (LGS), (loadStepping)); every Newton
 * step is one FETI solve.
 *
 * All arithmetic runs on one AMD Instinct MI355X (gfx950).  Every call returns
 * a feti_status; the library never aborts and never prints.  A call fails with
 * FETI_EDEVICE if no HIP device is usable: there is no CPU fallback.
 *
 * Ownership: the caller owns every array it passes in; feti_setup copies what
 * it needs and keeps no caller pointer.  The library owns the problem object
 * and all device memory it allocates (through the allocator callback of
 * feti_options, or hipMalloc when that is NULL).  Output arrays belong to the
 * caller: host memory by default, device memory with FETI_DEVICE_PTRS.
 *
 * Concurrency: one problem must not be used by two calls at the same time;
 * distinct problems may run concurrently (each has its own HIP stream).
 */
#ifndef FETI_H
#define FETI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FETI_OK = 0,
  FETI_EINVAL = -1,      /* bad sizes/ids, empty or disconnected subdomain, non-finite
                            input, all-floating problem without Dirichlet data      */
  FETI_ENOMEM = -2,      /* device memory could not be reserved                       */
  FETI_EDEVICE = -3,     /* no usable HIP device, or a HIP runtime error              */
  FETI_ENOTSPD = -4,     /* non-positive pivot in a local or coarse factor (non-finite
                            only, where a refined step replaces non-positive local
                            pivots); feti_last_error names the subdomain              */
  FETI_ENOCONV = -5,     /* max_it reached; outputs are still written,
                            stats.converged = 0                                        */
  FETI_ESTATE = -6,      /* feti_solve called before feti_factor                      */
  FETI_EBREAKDOWN = -7   /* PCG breakdown: s.Fs <= 0                                   */
} feti_status;

/* Tearing variant: classical FETI eliminates Dirichlet DOFs from the local
 * systems (section 4.1); all-floating FETI enforces them with extra
 * multipliers so every subdomain is floating (section 4.2). */
typedef enum { FETI_CLASSICAL = 0, FETI_ALL_FLOATING = 1 } feti_variant;

/* Preconditioner sum_i B_D,i Y_i B_D,i^T (eq. (feti_preconditioner)): Y_i = I,
 * Y_i = K_i (lumped, eq. (LumpedVK)) or the interface Schur complement
 * (Dirichlet, eq. (DirichletVK)).  Rows of B_D: weight 1/m on the gluing rows
 * of a DOF with m subdomain copies; at a Dirichlet DOF of all-floating FETI,
 * weight 1 on its Dirichlet rows and 0 on its gluing rows. */
typedef enum { FETI_PREC_IDENTITY = 0, FETI_PREC_LUMPED = 1, FETI_PREC_DIRICHLET = 2 } feti_precond;

/* FETI_FP64: every step in FP64.  FETI_MIXED: local factors and local solves
 * in FP32 (MFMA, FP32 accumulation); PCG recurrences, dot products, coarse
 * problem and rigid-body kernels in FP64; accuracy recovered by iterative
 * refinement against FP64 residuals. */
typedef enum { FETI_FP64 = 0, FETI_MIXED = 1 } feti_precision;

/* Material: kind 0 = isotropic linear elasticity (E, nu);
 * kind 1 = Holzapfel-Gasser-Ogden (section 2, eqs. (iso), (aniso_1),
 * (aniso_2)) with neo-Hooke parameter c, fibre parameters k1, k2 and the
 * volumetric penalty kappa of Psi_vol = kappa/2 (J-1)^2, the pressure being
 * condensed per element (P0). */
typedef struct {
  int32_t kind;
  double E, nu, c, k1, k2, kappa;
} feti_material;

/* The torn problem (section 4, eq. (decomposition)): a Q1 or Q2 hexahedral
 * mesh, a non-overlapping element partition, materials, Dirichlet data (eq.
 * (Dirichlet)), a body force and a follower pressure (eq. (Neumann)).
 * Node-major DOF numbering: dof = 3*node + component.  Q2 elements are the
 * 27-node triquadratic hexahedra of section 3.2 (with the HGO material, the
 * Q2-P0 pair: a pressure constant per element, condensed). */
typedef struct {
  int64_t n_nodes;
  const double* xyz;           /* [n_nodes][3] reference coordinates                   */
  int64_t n_elems;
  const int64_t* hex8;         /* element nodes, lexicographic (x fastest).  Q1:
                                  [n_elems][8], corner i+2j+4k at reference point
                                  (2i-1,2j-1,2k-1).  Q2: [n_elems][27], node i+3j+9k
                                  at reference point (i-1,j-1,k-1)                      */
  int32_t n_sub;
  const int32_t* elem_sub;     /* [n_elems] subdomain id in [0, n_sub); every subdomain
                                  must own at least one element                         */
  int32_t n_mat;
  const feti_material* mat;    /* [n_mat]                                               */
  const int32_t* elem_mat;     /* [n_elems] material id                                 */
  const double* elem_fibers;   /* [n_elems][2][3] unit fibre directions a01, a02 (HGO)
                                  or NULL when no element is HGO                        */
  int64_t n_dir;
  const int64_t* dir_dof;      /* [n_dir] Dirichlet DOFs (unique)                       */
  const double* dir_val;       /* [n_dir] prescribed displacement                       */
  const double* body_force;    /* [n_elems][3] force per unit reference volume, or NULL */
  int64_t n_pfaces;
  const int64_t* pface;        /* Q1: [n_pfaces][4] quadrilateral corners, (x1-x0)x(x3-x0)
                                  points out of the body.  Q2: [n_pfaces][9], node i+3j
                                  at face point (s,t) = (i-1,j-1), dx/ds x dx/dt points
                                  out of the body                                       */
  double pressure;             /* follower pressure on pface, current geometry           */
  int32_t order;               /* element order: 1 (Q1; 0 is read as 1) or 2 (Q2)       */
} feti_mesh;

#define FETI_DEVICE_PTRS 0x1ull /* U / u / dU arguments are device pointers */
#define FETI_PROFILE 0x2ull     /* time the dual-operator GEMV and factor-update kernels with
                                   HIP events (reported in feti_stats.kernel_*)              */
#define FETI_AUTOTUNE 0x4ull    /* pick the form of each factor-update launch (64x64 tiles,
                                   128x64 tiles, or 64x64 tiles with double-buffered direct
                                   global-to-LDS loads in 32- or 16-wide chunks) by timing
                                   each in one of the first four factorisations; the factors
                                   do not depend on it                                        */
#define FETI_KERNEL6 0x8ull     /* take all six rigid-body modes as the kernel of every floating
                                   subdomain, as the paper does (section 4.3).  Exact for
                                   stress-free tangents.  For stressed ones (Newton steps away
                                   from U = 0) the dual solve is of an approximate tangent,
                                   which stays definite where compressive stress makes a local
                                   tangent indefinite, and the result is refined against the
                                   exact sparse tangent (corrections as for FETI_MIXED, up to
                                   ir_tol / ir_max).  Default: translations, plus each rotation
                                   that passes the exactness test
                                   ||K r|| <= 1e-12 ||K||_F ||r|| (a direct exact solve)     */

#define FETI_LOAD_STIFFNESS 0x10ull /* feti_newton_step solves the exact linearisation of the
                                   follower-pressure problem, (K'(U) - tau d f_p / dU) dU =
                                   tau f_ext - f_int, whose load stiffness the paper neglects
                                   and notes to be non-symmetric (section 3.2, last paragraph):
                                   flexible GMRES on the assembled FP64 system, preconditioned
                                   by the FETI solve of the symmetric tangent K'(U), up to
                                   ir_tol / ir_max preconditioner applications                */

#define FETI_WARM_START 0x20ull  /* the first dual solve of feti_solve / feti_newton_step starts
                                   from the previous call's multipliers: lambda_0 = G (G^T G)^{-1} e
                                   + c P lambda_prev, which keeps the constraint G^T lambda = e,
                                   with the scale c that minimises the F-norm of the error along
                                   P lambda_prev (one extra F application).  For sequences of
                                   related solves: load ramps, Newton steps, request streams  */

#define FETI_DUAL_GMRES 0x40ull  /* the dual problem is solved by projected GMRES (restarted every
                                   100 vectors, right-preconditioned by P M^{-1} P) instead of PCG:
                                   for local operators that are not positive definite, such as the
                                   stressed tangents of a floating subdomain whose rotations are
                                   not in its kernel (section 3.2 notes that the FETI methods work
                                   with GMRES).  Same stopping rule; kappa_est is not computed  */

typedef struct {
  feti_variant variant;
  feti_precond precond;
  feti_precision precision;
  double rtol;                 /* PCG stop: ||P r_k||_2 <= rtol ||P r_0||_2 (0 => 1e-8)  */
  int32_t max_it;              /* PCG iteration cap (0 => 1000)                           */
  double ir_tol;               /* target of the refinement (FETI_MIXED, FETI_KERNEL6 at a
                                  stressed state, FETI_LOAD_STIFFNESS): flexible GMRES on
                                  the assembled FP64 system until ||b - A u||_2 <=
                                  ir_tol ||b||_2 over free DOFs (0 => 1e-10)              */
  int32_t ir_max;              /* max preconditioner applications (dual solves) of the
                                  refinement (negative => 6); restart every 30;
                                  0: none (the residual is still reported in res_primal)  */
  int32_t graph_block;         /* PCG iterations captured per HIP graph (0 => 8)          */
  void* hip_stream;            /* hipStream_t to run on, or NULL for a library stream    */
  void* (*dev_alloc)(size_t bytes, void* stream, void* ctx);   /* optional allocator     */
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
  uint64_t flags;              /* FETI_DEVICE_PTRS | FETI_PROFILE | FETI_AUTOTUNE |
                                  FETI_KERNEL6 | FETI_LOAD_STIFFNESS | FETI_WARM_START |
                                  FETI_DUAL_GMRES                                         */
  double kernel_tol;           /* rotation test of stressed floating subdomains: a rotation
                                  r joins the kernel if ||K r|| <= kernel_tol ||K||_F ||r||
                                  (0 => 1e-12, an exact kernel).  A larger value treats
                                  rotations of small stress-induced stiffness as kernel
                                  modes (an approximate tangent, refined by the flexible
                                  GMRES against the exact operator as with FETI_KERNEL6)  */
} feti_options;

typedef struct {
  int32_t iters;               /* PCG iterations (summed over refinement sweeps)          */
  int32_t converged;           /* 1 if the stopping rule was met                          */
  int32_t ir_sweeps;           /* refinement: preconditioner applications (dual solves)
                                  after the first solve                                   */
  int32_t n_coarse;            /* dimension of the coarse space (columns of G)            */
  int64_t n_lambda;            /* number of Lagrange multipliers                          */
  double rel_res;              /* final ||P r|| / ||P r_0||                               */
  double kappa_est;            /* Lanczos estimate of the preconditioned condition number */
  double t_assemble, t_factor, t_pcg, t_total;   /* seconds, from HIP events              */
  size_t device_bytes;         /* device memory held by the problem                       */
  /* kernel_gemv_launches: interface GEMV launches of F in this solve (one per PCG
     iteration and one for the initial residual, over all refinement sweeps);
     kernel_update_launches: tile-update launches of the last feti_factor.
     With FETI_PROFILE: mean duration (ms, HIP events on the problem's stream) of
     one GEMV launch, from back-to-back launches after the solve, and of one
     update launch, from events around each launch of the last factorisation.
     gemv_bytes: algorithmic bytes of one GEMV launch (packed symmetric interface
     inverses); update_flops: flops of all update launches of one factorisation */
  int32_t kernel_gemv_launches, kernel_update_launches;
  double kernel_gemv_ms, kernel_update_ms;
  double gemv_bytes, update_flops;
  double res_primal;           /* ||f - K u||_2 / ||f||_2 of the returned u (FP64, assembled,
                                  free DOFs): always for FETI_MIXED, with FETI_PROFILE for
                                  FETI_FP64, else 0                                         */
  int32_t autotune_wide;       /* FETI_AUTOTUNE: update launches that use 128x64 tiles once
                                  tuned; -1 while tuning or without FETI_AUTOTUNE          */
  int32_t autotune_db;         /* FETI_AUTOTUNE: update launches that use the double-buffered
                                  form once tuned; -1 while tuning or without it          */
  int32_t modified_pivots;     /* local pivots of the last factorisation that were not
                                  positive and were replaced (modified Cholesky).  Allowed
                                  only where the factors precondition a refinement against
                                  the exact FP64 operator (FETI_MIXED, FETI_KERNEL6 at a
                                  stressed state, FETI_LOAD_STIFFNESS), so the result stays
                                  the exact solution; elsewhere such a pivot is
                                  FETI_ENOTSPD                                            */
} feti_stats;

typedef struct feti_problem feti_problem;   /* opaque, owned by the library */

/* Decompose the mesh, build multiplier rows, their weights and index maps,
 * reserve device memory and upload the static data.  *out receives a new
 * problem (NULL on failure).  opts may be NULL (defaults: all-floating,
 * lumped, FP64).  Errors: EINVAL, ENOMEM, EDEVICE. */
feti_status feti_setup(const feti_mesh* mesh, const feti_options* opts, feti_problem** out);

/* Device memory held by the problem, for admission control. */
feti_status feti_footprint(const feti_problem* p, size_t* device_bytes);

/* Assemble the local tangents at displacement U ([3*n_nodes], NULL => 0),
 * compute the rigid-body kernels, factor every K_i (interior-first dense
 * Cholesky, regularised interface Schur complement, its explicit inverse) and
 * the coarse matrix G^T G.  These are the generalised inverses K_i^+ and the
 * kernels R_i of section 4.3, eq. (localSolutions), and the coarse operator of
 * eq. (projection).  Errors: EINVAL, ENOTSPD (the message names the
 * subdomain), EDEVICE. */
feti_status feti_factor(feti_problem* p, const double* U);

/* Solve the linear problem K u = lf f_ext with u = lf u_D on the Dirichlet
 * boundary, using the factors of the last feti_factor (which must have been
 * called with U = NULL): the dual problem of section 4.3, eq. (dualProblem),
 * by projected preconditioned CG from lambda_0 = G (G^T G)^{-1} e, then the
 * recovery of u_i by eq. (localSolutions).  u [3*n_nodes] receives the global nodal
 * displacements (shared nodes: mean of the subdomain copies; Dirichlet DOFs:
 * their prescribed values).  stats may be NULL.
 * Errors: ESTATE, ENOCONV (u still written), EBREAKDOWN, EDEVICE. */
feti_status feti_solve(feti_problem* p, double load_factor, double* u, feti_stats* stats);

/* feti_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, with the dual iteration's scratch (CG state, reduction ticket
 * counters, block partial sums, alpha/beta history) taken from a static device
 * array of 512 KiB that each device holds until the process ends, instead of
 * the problem's own buffers, and the PCG iterations launched one by one
 * instead of through an instantiated HIP graph.  It calls no hipMalloc or
 * hipFree.  The problem must have been set up with FETI_DEVICE_PTRS (u is a
 * device array) and max_it <= 8192 (the history the array holds); otherwise
 * FETI_EINVAL.  All calls on one device share the array, which keeps the last
 * call's contents: calls that overlap on one device race.  Results equal
 * those of feti_solve.  Errors: as feti_solve, and FETI_EDEVICE if the array's
 * address could not be obtained at set-up. */
feti_status feti_solve_noalloc(feti_problem* p, double load_factor, double* u, feti_stats* stats);

/* One Newton step of the nonlinear problem (eqs. (LGS), (loadStepping)):
 * factor at U_k, then solve K'(U_k) dU = tau f_ext(U_k) - f_int(U_k) with
 * dU = tau u_D - U_k on the Dirichlet boundary.  The follower pressure acts on
 * the current geometry and its load stiffness is neglected (section 3.2).
 * res_norm (may be NULL) receives ||tau f_ext - f_int||_2 over free DOFs.
 * Errors: as feti_factor and feti_solve. */
feti_status feti_newton_step(feti_problem* p, const double* U_k, double tau, double* dU,
                             double* res_norm, feti_stats* stats);

/* Change the dual stopping tolerance rtol and the refinement target ir_tol
 * of later calls (same meaning as in feti_options), e.g. to solve each
 * Newton step only as accurately as the Newton iteration needs (an inexact
 * Newton method).  The factors and the captured iteration graph are kept.
 * Errors: EINVAL (a tolerance outside (0, 1)). */
feti_status feti_set_tolerances(feti_problem* p, double rtol, double ir_tol);

/* Message of the last failed call on p (or of the last failed feti_setup when
 * p is NULL); valid until the next call on that problem. */
const char* feti_last_error(const feti_problem* p);

/* Release the problem and every device allocation it holds.  NULL is ignored. */
void feti_destroy(feti_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* FETI_H */
