/* fsi.h - C ABI of the MI355X (gfx950) monolithic Newton-Krylov-Schwarz FSI step.
 *
 * Method: Kong, Kheyfets, Finol, Cai, "Simulation of unsteady blood flows in a
 * patient-specific compliant pulmonary artery with a highly parallel monolithically
 * coupled fluid-structure interaction algorithm" (arXiv 1810.04289).
 *
 * One implicit backward-Euler step (§2.2, eq. (9)) is the root of F(y) = 0 (eq. (10)).
 * It is found by inexact Newton with backtracking (§3, eq. (11)); each Newton direction
 * solves J dy = -F (eq. (12)) with restarted GMRES (eq. (13)), right-preconditioned by
 * restricted additive Schwarz (eq. (16)) whose subdomain solver is a block incomplete LU
 * factorization ILU(l) (§3, §4.3).
 *
 * Unknowns: vertex-major, 7 per vertex [u_x u_y u_z p d_x d_y d_z], n = 7 * nverts.
 *   u  fluid velocity at fluid vertices, wall velocity at wall vertices, shared at
 *      interface vertices (strong coupling, §2.2 eqs. (6)-(7));
 *   p  pressure (a dummy row p = 0 at wall-only vertices);
 *   d  mesh displacement at fluid vertices, wall displacement at wall vertices, shared at
 *      interface vertices.
 * Jacobian: block CSR with 7x7 row-major FP64 blocks, int32 indices, sorted columns,
 * diagonal always present, block (a,b) present iff a and b share a tetrahedron.
 *
 * Conventions for every entry point:
 *  - returns fsi_status; no exception, exit or abort crosses this boundary;
 *  - pointers marked (dev) are device pointers owned by the caller, valid for the call;
 *    pointers marked (host) are host pointers owned by the caller;
 *  - all device work is ordered on the HIP stream given to fsi_create; every entry point
 *    returns after the stream work it issued has finished (host-side decisions of Newton
 *    and GMRES need the results anyway);
 *  - a failed call leaves a message readable through fsi_last_error.
 */
#ifndef FSI_H
#define FSI_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSI_OK = 0,
  FSI_ERR_ARG = 1,        /* bad argument, or a call out of order */
  FSI_ERR_MESH = 2,       /* inconsistent mesh (index out of range, orphan vertex, ...) */
  FSI_ERR_OOM = 3,        /* device or host allocation failed */
  FSI_ERR_HIP = 4,        /* a HIP runtime call failed */
  FSI_ERR_INVERTED = 5,   /* a fluid element with non-positive current volume, or det F <= 0 */
  FSI_ERR_ZERO_PIVOT = 6, /* a singular 7x7 pivot block in the subdomain factorization */
  FSI_ERR_DIVERGED = 7    /* Newton reached its iteration limit or the line search failed */
} fsi_status;

/* Boundary face tags. */
enum { FSI_TAG_NONE = 0, FSI_TAG_FLUID_INLET = 1, FSI_TAG_FLUID_OUTLET = 2,
       FSI_TAG_SOLID_RING_IN = 3, FSI_TAG_SOLID_RING_OUT = 4, FSI_TAG_WALL_OUTER = 5 };

/* Mesh (§2.1, §4.8): reference coordinates, positively oriented tetrahedra split into
 * fluid and wall elements, tagged boundary triangles.  Deep-copied by fsi_create. */
typedef struct {
  int32_t nverts, ntets, nbfaces;
  const double *X;           /* (host) [nverts][3] reference coordinates, cm */
  const int32_t *tets;       /* (host) [ntets][4] */
  const int8_t *tet_domain;  /* (host) [ntets] 0 fluid, 1 wall */
  const int32_t *bfaces;     /* (host) [nbfaces][3] */
  const int8_t *bface_tag;   /* (host) [nbfaces] FSI_TAG_* */
} fsi_mesh;

/* Material constants (cgs; §2.1 and §4.1): fluid density and dynamic viscosity, wall
 * density, Young's modulus, Poisson ratio, damping, and the inverse-estimate constant of
 * the stabilization parameter. */
typedef struct { double rho_f, mu_f, rho_s, E_s, nu_s, eta_s, C_I; } fsi_physics;

/* Subdomain orderings (§4.5, Table 4).  RCM: reverse Cuthill-McKee of the subdomain's
 * vertex graph from a George-Liu pseudo-peripheral vertex.  1WD: one-way dissection -- the
 * BFS levels from that vertex, every (ilu_level + 3)-th level a separator; the connected
 * blocks between separators first, each in RCM order, then the separator levels, each in
 * RCM order.  With ILU(l) no fill joins two separators, and rows of different blocks are
 * independent in the triangular sweeps. */
enum { FSI_ORDER_RCM = 0, FSI_ORDER_1WD = 1 };

/* Solver options (§3, §4).  Defaults of the paper: overlap 1, Newton rtol 1e-6, GMRES
 * rtol 1e-3, Jacobian lag 1, subdomain ILU(1), RCM subdomain ordering. */
typedef struct {
  int32_t nsub;             /* number of Schwarz subdomains (>= 1) */
  int32_t overlap;          /* delta: layers of vertex-graph neighbours added (>= 0) */
  int32_t ilu_level;        /* l of ILU(l), 0..8 */
  int32_t ordering;         /* FSI_ORDER_RCM or FSI_ORDER_1WD (§4.5, Table 4) */
  const int32_t *part;      /* (host) [nverts] subdomain of each vertex, or NULL for
                               recursive coordinate bisection */
  int32_t gmres_restart;    /* 1..200 */
  int32_t gmres_maxit;      /* total GMRES iterations per solve */
  double gmres_rtol;
  double newton_rtol, newton_atol;
  int32_t newton_maxit, jac_lag;
  double ls_c;              /* Armijo constant of the backtracking line search */
  int32_t ls_max_halvings;
  int32_t precision;        /* FSI_PREC_*: arithmetic of the Schwarz triangular sweeps */
} fsi_opts;

/* Precision of the preconditioner application (the mixed-precision variant of §3's
 * Schwarz preconditioner).  The factorization is FP64 in every mode; FP32 and BF16 round
 * the factors (to nearest, ties to even) into the front of the FP64 factors' own buffer, so
 * they take no memory of their own, and run both triangular sweeps in FP32 arithmetic,
 * including accumulation.  The input v and output z of
 * fsi_pc_apply stay FP64, as do residuals, GMRES and the Newton update. */
/* FSI_PREC_FP32_FACTOR: the factorization itself runs in FP32 (the FP64 Jacobian rounded
 * to FP32 in the gather, the same operations in the same order as the FP64 factorization),
 * its factors are stored in FP32 only (half the FP64 memory), and the sweeps are the FP32
 * ones. */
enum { FSI_PREC_FP64 = 0, FSI_PREC_FP32 = 1, FSI_PREC_BF16 = 2, FSI_PREC_FP32_FACTOR = 3 };

typedef struct {
  int32_t iters, restarts, converged, pad;
  double rnorm0, rnorm_est, rnorm_true;
} fsi_lin_stats;

#define FSI_MAX_NEWTON 64
/* Per-step statistics; the six phase timers carry the paper's event names (Table 7).
 * t_kspsolve includes t_pcapply and t_kspsetup (each GMRES solve's set-up before its first
 * Arnoldi step: the initial vector, the norm of the right-hand side; the workspace itself
 * is allocated once, at create). */
typedef struct {
  int32_t newton_iters, linear_iters, line_search_cuts, converged;
  double fnorm0, fnorm;
  double t_funceval, t_jaceval, t_pcsetup, t_pcapply, t_kspsolve, t_kspsetup; /* seconds */
  double fnorm_hist[FSI_MAX_NEWTON];
  double alpha_hist[FSI_MAX_NEWTON];
  int32_t lin_hist[FSI_MAX_NEWTON];
} fsi_step_stats;

typedef struct fsi_solver fsi_solver;

/* Build the solver: copies the mesh, classifies vertices (interface triangles by the
 * interface reconstruction of §4.8, Algorithm 1), builds the block pattern, the element
 * scatter maps, the partition, the overlapping subdomains (§3), their RCM order (§4.5),
 * the ILU(l) fill pattern and level schedules, and allocates device memory.
 * hip_stream: a hipStream_t (NULL = the null stream).  Errors: ARG, MESH, OOM, HIP. */
fsi_status fsi_create(const fsi_mesh *mesh, const fsi_physics *phys, const fsi_opts *opts,
                      void *hip_stream, fsi_solver **out);
fsi_status fsi_destroy(fsi_solver *s);
/* Sizes of the discrete problem: n = 7 nverts unknowns (the state y of §2.2 eq. (8), one
 * 7-vector per vertex) and nnzb, the number of 7x7 blocks of the Jacobian of eq. (12)
 * (vertex pairs that share a tetrahedron, plus the diagonal).  Either pointer (host) may
 * be NULL.  Error ARG on a NULL solver. */
fsi_status fsi_sizes(const fsi_solver *s, int64_t *n, int64_t *nnzb);
const char *fsi_last_error(const fsi_solver *s);

/* Data of one backward-Euler step (§2.2 eq. (9)): time t_n, step dt > 0, previous state
 * y_old (dev, n), Dirichlet values g (dev, n; used on Dirichlet rows, forced to zero on
 * clamped wall rings), nodal body force (dev, [nverts][3], or NULL), and an optional
 * extra Dirichlet mask (host, n bytes, 1 = Dirichlet with value g; NULL = none).
 * Dirichlet rows from the tags: inlet u = g and d = 0, outlets d = 0, wall rings u = d = 0. */
fsi_status fsi_set_step(fsi_solver *s, double t_n, double dt, const double *y_old,
                        const double *g, const double *body_force, const uint8_t *extra_mask);

/* Step setup (a Newton guess with the Dirichlet values and the dummy pressures written). */
fsi_status fsi_impose_dirichlet(fsi_solver *s, double *y /* dev, n, in/out */);

/* F(y) (eq. (10)): dt * (element residual) on equation rows, y - g on Dirichlet rows,
 * (d - d_old) - dt u on kinematic rows, p on dummy rows.  Error INVERTED if an element
 * inverts. */
fsi_status fsi_residual(fsi_solver *s, const double *y /* dev, n */, double *F /* dev, n */);

/* Exact Jacobian J = dF/dy at y (§3) into the solver's block matrix. */
fsi_status fsi_jacobian(fsi_solver *s, const double *y /* dev, n */);
/* Copy the block matrix to host arrays sized by fsi_sizes (any pointer may be NULL). */
fsi_status fsi_jacobian_get(const fsi_solver *s, int32_t *rowptr /* host, nverts+1 */,
                            int32_t *colind /* host, nnzb */, double *vals /* host, nnzb*49 */);

/* Replace the values of the solver's block matrix by caller-supplied ones (same pattern as
 * fsi_jacobian_get reports): a Jacobian of eq. (12) assembled elsewhere, for instance to
 * apply and factor exactly the same matrix as another implementation.  Marks the matrix
 * ready for fsi_spmv / fsi_pc_setup.  Error ARG on a NULL pointer. */
fsi_status fsi_jacobian_set(fsi_solver *s, const double *vals /* host, nnzb*49 */);

/* y = J x with the current Jacobian: the matrix-vector product of each GMRES iteration on
 * the preconditioned Jacobian system (§3 eqs. (12)-(13)).  Rows of the block CSR are
 * summed in ascending column order.  Error ARG before a Jacobian exists. */
fsi_status fsi_spmv(fsi_solver *s, const double *x /* dev, n */, double *y /* dev, n */);

/* Schwarz setup (§3 eqs. (15)-(16)): gather every subdomain matrix from J and factor it
 * by block ILU(l).  Error ZERO_PIVOT on a singular pivot block; error HIP if a row of the
 * factorization waited on its pivot rows beyond a fixed bound (the factors are then invalid;
 * a correct schedule never comes near it). */
fsi_status fsi_pc_setup(fsi_solver *s);
/* z = B^{-1} v = sum_i (R_i^0)^T (L_i U_i)^{-1} R_i^delta v. */
fsi_status fsi_pc_apply(fsi_solver *s, const double *v /* dev, n */, double *z /* dev, n */);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fsi_pc_apply with the sweeps' work
 * values and error flags in a static per-GPU scratch array of the library instead of the
 * solver's buffers.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); like fsi_pc_apply it waits for its stream work and reads one error
 * flag back.  The scratch holds 32 MiB of sweep values: 7 values per local (overlapped)
 * subdomain row, FP64 with FSI_PREC_FP64 and FP32 otherwise, i.e. up to 599,186 local
 * rows in FP64.  Larger solvers get ERR_ARG with a message that says so.  Every call on
 * one GPU, from any solver, uses that GPU's one copy of the array and leaves its contents
 * there: calls that overlap on one GPU (on different streams or host threads) race.
 * Results equal fsi_pc_apply's bit for bit (same kernels, same order).  Errors as
 * fsi_pc_apply, and HIP if the scratch's address could not be taken at fsi_create. */
fsi_status fsi_pc_apply_noalloc(fsi_solver *s, const double *v /* dev, n */, double *z /* dev, n */);

/* Schedule of the Schwarz sweeps.  Every subdomain's forward and backward sweep runs in one
 * launch per sweep, one workgroup per subdomain; rows are cut into tasks of at most mb
 * blocks, and the kernel for mb prefetches a matching number of tasks.  The candidates are
 * mb = 8, 16, 24 and 32; at create a rule on the longest row picks one.
 * fsi_pc_tune (after fsi_pc_setup) times every candidate on the current factors, reps
 * applications each after one untimed, and keeps the fastest: *best_mb (may be NULL)
 * receives it and us[4] (may be NULL) the microseconds per application of each candidate,
 * in the order above.  fsi_pc_select sets mb directly (ERR_ARG if not a candidate).  The
 * schedule changes the order of floating-point sums, not the operator. */
fsi_status fsi_pc_tune(fsi_solver *s, int32_t reps, int32_t *best_mb, double *us);
fsi_status fsi_pc_select(fsi_solver *s, int32_t mb);

/* GMRES's inner step as captured graphs (on != 0): the preconditioner, the SpMV, both
 * Gram-Schmidt passes and the norm of each Arnoldi step j are captured into one graph on
 * first use and replayed afterwards, one launch instead of nine.  Results are identical
 * to the eager path (same kernels, same order).  Graphs are dropped when the sweep
 * schedule changes or graphs are switched off; while kernel profiling (fsi_prof_enable) is
 * on, GMRES runs eagerly.  In graph mode the preconditioner's time in fsi_step_stats is
 * not measured separately.  Default off. */
fsi_status fsi_set_graphs(fsi_solver *s, int32_t on);

/* GMRES on J x = rhs (§3 eq. (12)), preconditioned from the right by the Schwarz
 * operator B^{-1} of eq. (16) as eq. (13) allows ("GMRES(fGMRES)", §4 set-up): restarted
 * every gmres_restart iterations, from x0 = 0, classical Gram-Schmidt applied twice,
 * Givens rotations, stopping when the residual estimate reaches gmres_rtol ||rhs|| (the
 * paper's linear tolerance, 1e-3 by default) or after gmres_maxit iterations.
 * Non-convergence is reported in st->converged, not as an error.  Error ARG before the
 * preconditioner exists; HIP if a sweep exceeded its wait bound. */
fsi_status fsi_gmres(fsi_solver *s, const double *rhs /* dev, n */, double *x /* dev, n */,
                     fsi_lin_stats *st /* host, may be NULL */);

/* One implicit step: inexact Newton with backtracking (§3 eq. (11)) on F(y) = 0 of
 * eq. (10), from the guess y (Dirichlet values imposed first) to
 * ||F|| <= max(newton_rtol ||F_0||, newton_atol) (the paper's nonlinear tolerance 1e-6,
 * §4 set-up).  Each Newton direction comes from fsi_gmres on eq. (12); the Jacobian and
 * the Schwarz factors are rebuilt every jac_lag iterations (§4.4); the line search halves
 * the step until the Armijo condition holds (an inverted element counts as a rejection).
 * y (dev, n) is overwritten with the result.  Error DIVERGED if the iteration limit is hit
 * or the line search fails. */
fsi_status fsi_newton_solve(fsi_solver *s, double *y, fsi_step_stats *st /* host, may be NULL */);

/* Replace the Newton tolerances of fsi_opts (rtol >= 0, atol >= 0, not both 0) for the
 * following solves.  A fixed absolute target (rtol = 0) lets solves from different initial
 * guesses of one step be compared at equal accuracy. */
fsi_status fsi_set_newton_tol(fsi_solver *s, double rtol, double atol);

/* Bound of the waits inside the factorization and the sweeps, in polls of a progress level
 * (polls = -1 restores the default, about a second; 0 gives up at the first poll that finds
 * the level not yet reached).  A wait past its bound stops waiting, so the kernel still
 * ends, and the call reports error HIP: fsi_pc_setup, fsi_pc_apply, fsi_pc_tune,
 * fsi_gmres and fsi_newton_solve.  For tests of that error path; the default is never reached by a
 * correct schedule.  Drops captured graphs. */
fsi_status fsi_set_wait_limit(fsi_solver *s, int32_t polls);

/* ---- introspection (host copies; for tests and diagnostics) ---- */
/* vkind[nverts]: 0 fluid, 1 interface, 2 wall; rowkind[n]: 0 element, 1 Dirichlet,
 * 2 kinematic, 3 dummy; interface triangles from Algorithm 1 as [n_iface][3]. */
fsi_status fsi_topology_get(const fsi_solver *s, int8_t *vkind, uint8_t *rowkind,
                            int32_t *n_iface, int32_t *iface_faces);
fsi_status fsi_pc_sizes(const fsi_solver *s, int32_t *nsub, int64_t *nloc_rows,
                        int64_t *nloc_blocks, int64_t *nlevels_total);
/* Partition, RCM-ordered subdomain vertex lists, local block patterns, and (after
 * fsi_pc_setup) the factors: strict L blocks (unit diagonal implied), strict U blocks,
 * inverted diagonal blocks in the diagonal positions, and the U diagonal blocks before
 * inversion (udiag).  With FP32 or BF16 sweeps the factors returned are the rounded ones the
 * sweeps use, widened to FP64 (the FP64 factors are overwritten by their rounding); with an
 * FP32 factorization, its FP32 factors and udiag, widened. */
fsi_status fsi_pc_get(const fsi_solver *s, int32_t *part, int32_t *sub_ptr, int32_t *sub_verts,
                      int32_t *sub_nowned, int64_t *blk_ptr, int32_t *lrowptr, int32_t *lcolind,
                      double *factors, double *udiag);

/* ---- kernel timing (HIP events on the solver's stream) ----
 * fsi_prof_enable(s, 1) starts recording an event pair around every launch of the timed
 * kernels; fsi_prof_get returns the summed duration (ms) and launch count for a kernel
 * name: "ilu_fwd", "ilu_bwd", "ilu_factor", "spmv", "elem_jac_fluid", "elem_jac_solid",
 * "jac_init", "elem_res_fluid", "elem_res_solid", "res_gather", "mdot", "vupdate". */
fsi_status fsi_prof_enable(fsi_solver *s, int32_t on);
fsi_status fsi_prof_get(fsi_solver *s, const char *kernel, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif
