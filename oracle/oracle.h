/*
 * Oracle: a plain, slow, FP64 CPU implementation of the block-based AMR
 * explicit discontinuous Galerkin method for the compressible Euler
 * equations (Liu et al., "An unstructured block-based adaptive mesh
 * refinement approach for explicit discontinuous Galerkin method").
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; the two agree only through the
 * documented data layout and leaf order.
 *
 * Every routine follows the paper's definitions written out directly:
 *   - conservation law and Euler fluxes           (Sec. 2, Eq. 1-2; EOS Eq. 23)
 *   - Galerkin weak form and M dK/dt = R          (Sec. 2, Eq. 3-4)
 *   - Lax-Friedrichs (Rusanov) numerical flux     (Sec. 2, Eq. 5, dissipative sign)
 *   - SSP Runge-Kutta, third order                (Sec. 2 and Sec. 5.1)
 *   - forest of block trees, roots at level 1     (Sec. 3.1)
 *   - N^d cells per block, one guard layer        (Sec. 3.3)
 *   - L2 inheritance parent<->children            (Sec. 3.4, Eq. 11-14)
 *   - guard-cell fill: copy / split / combine     (Sec. 3.5, Eq. 15-17)
 *   - per-step procedure                          (Sec. 4.3)
 *
 * Data layout shared with the GPU library (by contract, not by code):
 *   state  U[leaf][var][mode][cell]     cell = i + N*(j + N*k), x fastest
 *   guard  G[leaf][face][var][mode][t]  face = 2*axis + (side>0), t runs over
 *                                       the face's N^(d-1) cells with the
 *                                       lower remaining axis fastest
 *   modes  graded by total degree s = 0..p; within s, m_x from s down to 0,
 *          then m_y from s-m_x down to 0, m_z the rest
 *   leaves trees row-major (x fastest), then Morton order inside a tree
 *   keys   (tree, level, i, j, k) per leaf, roots at level 1
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* non-periodic faces: outflow (Euler, Sec. 5.3.1) or, for the diffusion
 * equation, Dirichlet data from the exact solution (Sec. 5.2) */
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_DIRICHLET = 2 };
enum { ORC_HANG_PAPER = 0, ORC_HANG_CONSERVATIVE = 1 };
enum { ORC_IC_VORTEX = 0, ORC_IC_SEDOV = 1, ORC_IC_UNIFORM = 2, ORC_IC_XWAVE = 3, ORC_IC_COSINE = 4, ORC_IC_EXP = 5 };
/* equation solved: the Euler equations (Sec. 2), the linear scalar
 * convection equation of Sec. 5.1 or the diffusion equation of Sec. 5.2 */
enum { ORC_EQ_EULER = 0, ORC_EQ_ADVECTION = 1, ORC_EQ_DIFFUSION = 2 };

typedef struct orc_forest orc_forest;

/* ---- basis / quadrature pieces (exported for the pins) ---- */
double orc_legendre(int n, double x);
double orc_legendre_deriv(int n, double x);
void orc_gauss_legendre(int q, double *x, double *w);
int orc_num_modes(int dim, int p);
void orc_mode_exponents(int dim, int p, int *exps /* nb x 3 */);
/* L2 split (Eq. 11-12) and combine (Eq. 13-14) operators between a parent
 * cell and its child `child` (bit a of child = upper half along axis a),
 * both nb x nb, row = output mode. */
void orc_split_matrix(int dim, int p, int child, double *S);
void orc_combine_matrix(int dim, int p, int child, double *C);
/* Euler flux along `axis` and the Rusanov flux for outward normal
 * sign*e_axis (Eq. 2, 5, 23). */
void orc_euler_flux(int dim, double gamma, const double *u, int axis, double *f);
void orc_rusanov(int dim, double gamma, const double *um, const double *up,
                 int axis, int sign, double *fhat);

/* ---- forest ---- */
orc_forest *orc_create(int dim, int p, int n_cell, const int *roots,
                       const double *lo, const double *hi, const int *bc,
                       int max_level, double gamma, int hanging);
/* Switch a freshly created forest (before any other call) to the scalar
 * convection equation u_t + vel . grad u = 0 (one variable). */
void orc_set_advection(orc_forest *f, const double *vel);
/* Upwind (Rusanov with alpha = |vel . n|) flux of the scalar convection
 * equation for the outward normal sign*e_axis. */
double orc_upwind(const double *vel, double um, double up, int axis, int sign);
/* Switch a freshly created forest to the diffusion equation
 * u_t = nu div grad u (Sec. 5.2, one variable) discretised with the
 * symmetric interior-penalty DG method; every non-periodic face takes
 * Dirichlet data from the exact solution exp(a . x + nu |a|^2 t)
 * (a = avec[0..2]). */
void orc_set_diffusion(orc_forest *f, double nu, const double *avec);
/* Frames of the root blocks (Sec. 3.1: neighbouring roots may be rotated
 * against each other): codes[tree] is the rotation of the root's local axes,
 * global vector = Q local vector; 2-D: code k = k quarter turns
 * counter-clockwise; 3-D: code k = the k-th signed permutation matrix with
 * determinant +1 (permutations of the local axes in lexicographic order,
 * then the sign patterns of the local axes, bit l = axis l negative).  The
 * leaf keys, cells, modes and momentum of a root are in its local frame.
 * The convection velocity is taken along each root's local axes.
 * Requires equal root edges and the paper hanging mode; returns 0, or -1
 * (nothing changed).  Call before refining. */
int orc_set_frames(orc_forest *f, const int *codes);
/* time of the state (Dirichlet data of the diffusion equation); orc_step
 * advances it by dt */
/* Sec. 3.3, Eq. 6: bilinear (3-D: trilinear) root blocks from the root
 * grid nodes xy ((roots_x + 1) x (roots_y + 1) [x (roots_z + 1)] points of d
 * coordinates, x fastest).  With rotated frames (either call first) a
 * root's local axes follow the node grid's axes as its frame turns them,
 * and the momentum is stored along the global axes.  -1 if not allowed
 * (conservative mode, diffusion), if a root has a non-positive Jacobian at
 * a corner, or if periodic node copies do not match. */
int orc_set_nodes(orc_forest *f, const double *xy);
void orc_set_time(orc_forest *f, double t);
double orc_get_time(const orc_forest *f);
void orc_destroy(orc_forest *f);
int orc_num_leaves(const orc_forest *f);
void orc_leaf_keys(const orc_forest *f, int *keys /* n x 5 */);
long orc_state_len(const orc_forest *f);
long orc_guard_len(const orc_forest *f);
/* refinement: flags per leaf (+1 refine, -1 coarsen, 0 keep); level limits,
 * sibling completeness and 2:1 face balance are enforced (refinement wins).
 * Returns the new leaf count; orc_apply_adapt then switches the forest and
 * projects u_old (old layout) into u_new (new layout) by L2 inheritance. */
int orc_plan_adapt(orc_forest *f, const signed char *flags);
void orc_apply_adapt(orc_forest *f, const double *u_old, double *u_new);

/* ---- solver pieces ---- */
void orc_project_ic(const orc_forest *f, int kind, const double *params,
                    double t, double *u);
void orc_fill_guards(const orc_forest *f, const double *u, double *g);
void orc_residual(const orc_forest *f, const double *u, const double *g,
                  double *r);
void orc_rk_combine(long n, int stage, double dt, const double *un,
                    const double *us, const double *r, double *unext);
double orc_max_rate(const orc_forest *f, const double *u);
double orc_dt(const orc_forest *f, const double *u, double cfl);
void orc_totals(const orc_forest *f, const double *u, double *totals);
void orc_limit_positivity(const orc_forest *f, double *u);
void orc_indicator(const orc_forest *f, const double *u, double *eta);
/* One SSP-RK3 step (Sec. 4.3): guard fill and residual before each stage,
 * optional positivity limiter after each stage.  dt_fixed > 0 overrides the
 * CFL time step.  Returns the dt used. */
double orc_step(const orc_forest *f, double cfl, double dt_fixed,
                int limiter, double *u);
/* L1/L2 error against an analytic solution (quadrature with p+3 points). */
void orc_errors(const orc_forest *f, const double *u, int kind,
                const double *params, double t, double *l1, double *l2);
int orc_threads(void);
/* OpenMP threads of the oracle's parallel loops (n > 0) */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
