/* FP64 CPU oracle of the monolithic Newton-Krylov-Schwarz FSI step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, sequential, deliberately slow
 * restatement of the method of Kong, Kheyfets, Finol and Cai (arXiv 1810.04289),
 * written from the paper.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Every entry point works on HOST pointers, returns 0 on success or one of the
 * status codes below, and never aborts.  Arrays are vertex-major with 7 unknowns per
 * vertex [u_x u_y u_z p d_x d_y d_z] (n = 7V), 0-based int32 indices.
 *
 * Parity status: every function is pinned by tests against the paper's definitions,
 * closed forms, invariants, textbook special cases or brute force, except where a
 * header comment below says "parity unpinned".
 */
#ifndef FSIO_H
#define FSIO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { FSIO_OK = 0, FSIO_ERR_ARG = 1, FSIO_ERR_MESH = 2, FSIO_ERR_OOM = 3, FSIO_ERR_HIP = 4,
       FSIO_ERR_INVERTED = 5, FSIO_ERR_ZERO_PIVOT = 6, FSIO_ERR_DIVERGED = 7 };

typedef struct {
  int32_t nverts, ntets, nbfaces;
  const double *X;            /* [nverts][3] reference coordinates */
  const int32_t *tets;        /* [ntets][4] positive orientation */
  const int8_t *tet_domain;   /* [ntets] 0 fluid, 1 solid */
  const int32_t *bfaces;      /* [nbfaces][3] */
  const int8_t *bface_tag;    /* 1 inlet, 2 outlet, 3 ring in, 4 ring out, 5 outer wall, 0 none */
} fsio_mesh;

typedef struct { double rho_f, mu_f, rho_s, E_s, nu_s, eta_s, C_I; } fsio_physics;

typedef struct {
  int32_t nsub, overlap, ilu_level, ordering;
  const int32_t *part;        /* [nverts] or NULL = recursive coordinate bisection */
  int32_t gmres_restart, gmres_maxit;
  double gmres_rtol;
  double newton_rtol, newton_atol;
  int32_t newton_maxit, jac_lag;
  double ls_c;
  int32_t ls_max_halvings;
  int32_t precision;
} fsio_opts;

typedef struct {
  int32_t iters, restarts, converged, pad;
  double rnorm0, rnorm_est, rnorm_true;
} fsio_lin_stats;

#define FSIO_MAX_NEWTON 64
typedef struct {
  int32_t newton_iters, linear_iters, line_search_cuts, converged;
  double fnorm0, fnorm;
  double t_funceval, t_jaceval, t_pcsetup, t_pcapply, t_kspsolve, t_kspsetup;
  double fnorm_hist[FSIO_MAX_NEWTON];
  double alpha_hist[FSIO_MAX_NEWTON];
  int32_t lin_hist[FSIO_MAX_NEWTON];
} fsio_step_stats;

typedef struct fsio_solver fsio_solver;

int fsio_create(const fsio_mesh *mesh, const fsio_physics *phys, const fsio_opts *opts,
                fsio_solver **out);
int fsio_destroy(fsio_solver *s);
int fsio_sizes(const fsio_solver *s, int64_t *n, int64_t *nnzb);
const char *fsio_last_error(const fsio_solver *s);

/* Step data: old state y_{n-1}, Dirichlet values g, nodal body force f [V][3] or NULL,
 * extra Dirichlet mask [n] (1 = Dirichlet with value g) or NULL. */
int fsio_set_step(fsio_solver *s, double t_n, double dt, const double *y_old, const double *g,
                  const double *body_force, const uint8_t *extra_mask);
int fsio_impose_dirichlet(fsio_solver *s, double *y);
int fsio_residual(fsio_solver *s, const double *y, double *F);
/* complex-step variant: y = y_re + i*y_im, F likewise (for derivative checks) */
int fsio_residual_complex(fsio_solver *s, const double *y_re, const double *y_im, double *F_re,
                          double *F_im);
int fsio_jacobian(fsio_solver *s, const double *y);
int fsio_jacobian_get(const fsio_solver *s, int32_t *rowptr, int32_t *colind, double *vals);
/* replace the Jacobian's values (same pattern as fsio_jacobian_get reports) */
int fsio_jacobian_set(fsio_solver *s, const double *vals);
int fsio_spmv(fsio_solver *s, const double *x, double *y);
int fsio_pc_setup(fsio_solver *s);
int fsio_pc_apply(fsio_solver *s, const double *v, double *z);
int fsio_gmres(fsio_solver *s, const double *rhs, double *x, fsio_lin_stats *st);
int fsio_newton_solve(fsio_solver *s, double *y, fsio_step_stats *st);

/* introspection (tests) */
int fsio_topology_get(const fsio_solver *s, int8_t *vkind, uint8_t *rowkind, int32_t *n_iface,
                      int32_t *iface_faces);
int fsio_pc_sizes(const fsio_solver *s, int32_t *nsub, int64_t *nloc_rows, int64_t *nloc_blocks,
                  int64_t *nlevels_total);
int fsio_pc_get(const fsio_solver *s, int32_t *part, int32_t *sub_ptr, int32_t *sub_verts,
                int32_t *sub_nowned, int64_t *blk_ptr, int32_t *lrowptr, int32_t *lcolind,
                double *factors, double *udiag);
/* element-level access for pins: element residual (28) and dual-number Jacobian (28x28) */
int fsio_element(fsio_solver *s, const double *y, int32_t e, double *Re, double *Je);
/* operation counts of element e's residual at y (measurement): value_ops, the operations of
 * one evaluation (its algorithmic flops); tangent_ops, the operations one forward-mode
 * derivative direction adds; the exact element Jacobian by forward mode costs
 * value_ops + 28 tangent_ops */
int fsio_element_ops(fsio_solver *s, const double *y, int32_t e, int64_t *value_ops, int64_t *tangent_ops);

#ifdef __cplusplus
}
#endif
#endif
