/*
 * dgamr - block-based AMR explicit discontinuous Galerkin residual for the
 * compressible Euler equations on one MI355X (gfx950) GPU.
 *
 * Method: Liu et al., "An unstructured block-based adaptive mesh refinement
 * approach for explicit discontinuous Galerkin method".  A forest of
 * equal-size quad/hex blocks (Sec. 3.1), N^d cells per block with one layer
 * of guard cells (Sec. 3.3), guard cells filled by copy / split / combine
 * (Sec. 3.5, Eq. 15-17, operators of Sec. 3.4, Eq. 11-14), the Galerkin weak
 * form M dK/dt = R (Sec. 2, Eq. 3-4) with the Lax-Friedrichs (Rusanov)
 * numerical flux (Eq. 5) and SSP Runge-Kutta time marching (Sec. 2), all per
 * the procedure of Sec. 4.3.
 *
 * Conventions
 *  - Every call returns 0 (DGAMR_OK) or a negative DGAMR_E* code; the text
 *    of the last error of the calling thread is dgamr_last_error().  No C++
 *    exception crosses this interface.
 *  - Ownership: the library owns the forest topology, the neighbour and
 *    guard-fill tables and the basis tables (host and device copies).  The
 *    caller owns every state, guard, residual and work buffer: device memory
 *    passed as plain pointers, sized by dgamr_state_bytes().  Device calls
 *    are asynchronous on the caller's stream; host calls are synchronous.
 *    A forest handle must not be used by two threads at once.
 *  - Layouts (all FP64 unless stated):
 *      state    U[leaf][var][mode][cell]      cell = i + N*(j + N*k), x fastest
 *      guard    G[leaf][face][var][mode][t]   face = 2*axis + (side > 0);
 *               t indexes the N^(d-1) cells of the face, the lower of the
 *               remaining axes fastest
 *      residual R like U, FP64; FP32 when the forest precision is
 *               DGAMR_FP32
 *      vars     (rho, rho u, rho v[, rho w], E), E = total energy per volume
 *      modes    total-degree Legendre products P_mx P_my [P_mz], |m| <= p,
 *               graded by |m|; inside one degree m_x descending, then m_y
 *               descending.  Mode 0 is the cell mean.
 *      leaves   trees row-major (x fastest), then Morton order inside a
 *               tree; key = (tree, level, i, j, k), roots at level 1.
 */
#ifndef DGAMR_H
#define DGAMR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DGAMR_OK = 0,
    DGAMR_EINVAL = -1,       /* bad argument or descriptor */
    DGAMR_EUNSUPPORTED = -2, /* valid but not built (e.g. degree or size limits) */
    DGAMR_EBALANCE = -3,     /* topology violates 2:1 face balance */
    DGAMR_EHIP = -4,         /* a HIP runtime call failed */
    DGAMR_ENONPHYSICAL = -5, /* non-finite or non-positive density/pressure found */
    DGAMR_ESTATE = -6,       /* call out of order (e.g. apply before set) */
    DGAMR_EFULL = -7         /* a pool has no free slot range or member id */
};

/* Non-periodic faces: outflow (Euler, Sec. 5.3.1) or Dirichlet data from the
 * exact solution (diffusion only, Sec. 5.2). */
enum { DGAMR_BC_PERIODIC = 0, DGAMR_BC_OUTFLOW = 1, DGAMR_BC_DIRICHLET = 2 };
/* Residual arithmetic: FP64, or FP32 (FP32 inputs and accumulation for the
 * volume, face and lifting contractions; the state and the stage update stay
 * FP64). */
enum { DGAMR_FP64 = 0, DGAMR_FP32 = 1 };
enum { DGAMR_HANG_PAPER = 0, DGAMR_HANG_CONSERVATIVE = 1 };
enum { DGAMR_LIMITER_NONE = 0, DGAMR_LIMITER_POSITIVITY = 1 };
enum { DGAMR_IC_VORTEX = 0, DGAMR_IC_SEDOV = 1, DGAMR_IC_UNIFORM = 2, DGAMR_IC_XWAVE = 3, DGAMR_IC_COSINE = 4,
       DGAMR_IC_EXP = 5 };
/* Equation: the Euler equations (Sec. 2, Eq. 1-5, 23; d+2 variables), the
 * linear scalar convection equation u_t + vel . grad u = 0 of Sec. 5.1 (one
 * variable; Rusanov flux with alpha = |vel . n|, i.e. upwind), or the
 * diffusion equation u_t = nu div grad u of Sec. 5.2 (one variable;
 * symmetric interior-penalty DG with penalty 2 (p+1)^2 / h, Dirichlet data on
 * non-periodic faces from the exact solution exp(a . x + nu |a|^2 t)). */
enum { DGAMR_EQ_EULER = 0, DGAMR_EQ_ADVECTION = 1, DGAMR_EQ_DIFFUSION = 2 };

typedef struct {
    int dim;          /* 2 or 3 */
    int degree;       /* polynomial degree p, 0..3 */
    int n_cell;       /* N cells per block side: even, 2..16 (2-D) or 2..8 (3-D) */
    int roots[3];     /* root blocks per axis (unused axes: 1) */
    double lo[3];     /* domain box */
    double hi[3];
    int bc[3];        /* DGAMR_BC_* per axis */
    int max_level;    /* >= 1; roots are level 1 */
    double gamma;     /* ideal-gas ratio (Eq. 23) */
    int precision;    /* DGAMR_FP64 or DGAMR_FP32 (residual contractions) */
    int hanging;      /* DGAMR_HANG_PAPER (guard-cell fluxes, Sec. 3.5) or
                         DGAMR_HANG_CONSERVATIVE (coarse side lifts the fine-side flux) */
    int limiter;      /* DGAMR_LIMITER_* applied after each stage by dgamr_step */
    int equation;     /* DGAMR_EQ_*; scalar convection and diffusion require FP64
                         and no limiter; diffusion degree >= 1, bc periodic or
                         Dirichlet, paper hanging mode */
    double velocity[3]; /* convection velocity (DGAMR_EQ_ADVECTION) */
    double diffusivity; /* nu (DGAMR_EQ_DIFFUSION), > 0 */
    double exact_a[3];  /* a of the exact solution exp(a . x + nu |a|^2 t) that
                           gives the Dirichlet data (DGAMR_EQ_DIFFUSION) */
} dgamr_forest_desc;

typedef struct dgamr_forest dgamr_forest;
/* A captured HIP graph of solver steps (dgamr_run_capture, dgamr_pools_capture). */
typedef struct dgamr_graph dgamr_graph;

/* Sec. 3.1: a forest of root blocks at level 1 with periodic or outflow
 * links (Sec. 5.1, 5.3.1).  Builds the host topology, the device neighbour
 * tables and uploads them to the current device.  EINVAL on a bad
 * descriptor, EUNSUPPORTED outside the built limits. */
int dgamr_create_forest(const dgamr_forest_desc *desc, dgamr_forest **out);

/* Sec. 3.1, 3.5: root blocks whose local frames are rotated against each
 * other.  codes[tree] (one per root, trees row-major) is the rotation of the
 * root's local axes, global vector = Q local vector: 2-D, code k = k quarter
 * turns counter-clockwise (0..3); 3-D, code k = the k-th signed permutation
 * matrix of determinant +1 when the permutations of the local axes are
 * taken in lexicographic order and then the sign patterns (bit l: local
 * axis l negative), 0..23.  The leaf keys, cells, modes and momentum of a
 * root are in its local frame.  A guard cell across roots of different
 * frames is the copy, split or combine of the neighbour's cells in the
 * neighbour's frame, then turned into the own frame (K_d = R^n S^i K_s,
 * Eq. 15-17): a signed permutation of the modes (exact: total-degree
 * Legendre spaces are closed under signed permutations of the axes) and of
 * the momentum components.  Each stage of such a forest runs the fill into
 * the guard buffer, then the stage kernel reading the far side of block
 * faces from it, fused with the stage update and the limiter.  With
 * bilinear / trilinear roots (dgamr_set_root_nodes, before or after this
 * call) a root's local axes follow the node grid's axes as its frame turns
 * them, the momentum is stored along the global axes, and the fill turns
 * the modes only.  Scalar convection takes the velocity along each root's
 * local axes.  Requires equal root edges, the unrefined forest (ESTATE
 * otherwise) and the paper hanging mode (EUNSUPPORTED); pools do not admit
 * such forests. */
int dgamr_set_root_frames(dgamr_forest *f, const int32_t *codes);

/* Sec. 3.3, Eq. 6: root blocks as bilinear (3-D: trilinear) images of the
 * reference square (cube).  xy (host, (roots[0] + 1) * (roots[1] + 1)
 * [* (roots[2] + 1)] points of dim coordinates, x fastest) are the root
 * grid nodes: root (rx, ry[, rz]) has the corner nodes (rx + bx, ry + by[,
 * rz + bz]), b in {0,1}^dim.  On a periodic axis the last node layer must
 * be the first one moved by the period.  Every root must have a positive
 * Jacobian at its corners.  A leaf's cells are the images of equal squares
 * (cubes) of its root's reference box; the residual carries the map's
 * Jacobian at every quadrature point (the contravariant volume flux, face
 * normals and areas from the adjugate of the Jacobian) and the cell's full
 * mass matrix.  The guard cells and the inheritance on regrid stay the
 * reference-space operators of Eq. 11-17.  The steps of such a forest run
 * the fill and the residual fused with the stage update as separate
 * launches; the CFL rate takes the cell means over the physical cells and,
 * per reference axis, the face normal and width 2 det(J) / |row of adj(J)|
 * at the cell centre; the totals integrate over the physical cells; the
 * indicator keeps the reference cell means (mode 0); the positivity
 * limiter scales about the mean over the physical cell, int U |J| / int |J|,
 * and so also moves mode 0.  Root frames (dgamr_set_root_frames) may be set
 * as well.  EUNSUPPORTED for 3-D degree 3, the conservative mode, the
 * diffusion equation or FP32;
 * EINVAL for nodes that are not finite, a root
 * with a non-positive corner Jacobian, or unmatched periodic nodes.  Pools
 * do not admit such forests. */
int dgamr_set_root_nodes(dgamr_forest *f, const double *xy);
int dgamr_destroy_forest(dgamr_forest *f);

/* Host queries.  keys: n_leaves x 5 int32 (tree, level, i, j, k). */
int dgamr_num_leaves(const dgamr_forest *f, int64_t *n);
int dgamr_leaf_keys(const dgamr_forest *f, int32_t *keys);
/* Bytes of one state array, of the guard buffer, of the residual buffer and
 * of the work buffer dgamr_step and the reductions need. */
int dgamr_state_bytes(const dgamr_forest *f, size_t *u_bytes, size_t *guard_bytes,
                      size_t *residual_bytes, size_t *work_bytes);

/* Sec. 4.3 step 3, Sec. 3.1, Sec. 3.4: plan refinement from host flags
 * (n_leaves int8: +1 refine, -1 coarsen, 0 keep).  Rules: flags count
 * only inside [1, max_level]; refinement is closed under 2:1 face balance
 * (refinement wins); a family of 2^d sibling leaves coarsens only if all
 * are flagged -1, none refines, and no outside face neighbour ends finer
 * than the family.  Writes the new leaf count.  Host only; the forest is
 * unchanged until dgamr_apply_refinement. */
int dgamr_set_refinement(dgamr_forest *f, const int8_t *flags, int64_t *n_new);
/* Eq. 11-14: switch to the planned forest and write u_new (new layout,
 * caller-allocated) from u_old (old layout) by L2 inheritance: refined
 * children get the split of their parent cells, coarsened parents the
 * combine of their children, other leaves are copied.  Synchronises the
 * stream.  ESTATE if no plan is pending. */
int dgamr_apply_refinement(dgamr_forest *f, const double *u_old, double *u_new, hipStream_t stream);

/* Sec. 3.5, Eq. 15-17: fill every guard cell from the stage input u
 * (read-only): copy (same level), split of the coarser neighbour cell,
 * combine of the finer neighbour cells; outflow faces mirror the own cell. */
int dgamr_fill_guardcells(dgamr_forest *f, const double *u, double *guard, hipStream_t stream);

/* Sec. 2, Eq. 3-5: R = M^-1 [ volume flux integral - surface integral of the
 * Rusanov flux ], neighbour traces from the block interior or the guard
 * buffer.  r is FP64, or FP32 for DGAMR_FP32 forests. */
int dgamr_dg_residual(dgamr_forest *f, const double *u, const double *guard, void *r,
                      hipStream_t stream);

/* Sec. 2 (SSP-RK3): u_next = a_s u_n + b_s (u_s + dt r), with
 * (a,b) = (0,1), (3/4,1/4), (1/3,2/3) for stage 0,1,2.  dt is read from
 * device memory.  u_next may alias u_s. */
int dgamr_rk_stage(dgamr_forest *f, int stage, const double *dt_dev, const double *u_n,
                   const double *u_s, const void *r, double *u_next, hipStream_t stream);

/* Sec. 4.3 step 2(a): dt = cfl / max over cells of sum_a (|u_a| + c)/h_a
 * from the cell means, written to device memory.  Scalar convection: the
 * same with |vel_a| for |u_a| + c; diffusion: dt = cfl / max over cells of
 * nu sum_a 1/h_a^2 (a diffusive CFL number; explicit SSP-RK3 with the
 * penalty above is stable for cfl up to about 0.04 / 0.01 / 0.004 at
 * p = 1 / 2 / 3). */
int dgamr_compute_dt(dgamr_forest *f, double cfl, const double *u, double *dt_dev, void *work,
                     hipStream_t stream);

/* Time of the state of a diffusion forest (the Dirichlet data of a stage is
 * the exact solution at the stage's time: t, t + dt, t + dt/2).  dgamr_step
 * and dgamr_run advance it by each step's dt; dgamr_dg_residual uses it.
 * Host calls; other equations keep but do not use it. */
int dgamr_set_time(dgamr_forest *f, double t);
int dgamr_get_time(const dgamr_forest *f, double *t);

/* Sec. 4.3 step 2: one SSP-RK3 time step, in place on u: dt from the CFL
 * condition (cfl > 0) or taken from dt_dev (cfl <= 0), then per stage the
 * guard fill, the residual and the stage update (and the positivity limiter
 * when the forest asks for it).  The far side of every block face is
 * computed inside the stage kernel straight from the neighbours' cells (same
 * values as dgamr_fill_guardcells), except where a fill kernel writes into
 * the work buffer before each stage: guard traces for the 3-D
 * lane-per-(cell, variable) kernel, and guard coefficients on forests with
 * rotated root frames or bilinear / trilinear roots.  Asynchronous;
 * captures into a HIP graph.  Diffusion
 * forests (cfl > 0 required; dt computed on the host from the forest's
 * finest cells and written to dt_dev): per stage the guard fill of
 * coefficients into the work buffer, then the interior-penalty residual and
 * stage update with the Dirichlet data at the stage time; the forest's time
 * advances by dt (so a graph replay would repeat the times: not captured). */
int dgamr_step(dgamr_forest *f, double cfl, double *u, void *work, double *dt_dev,
               hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dgamr_step without the caller's work buffer.  The work area is a static
 * device array of DGAMR_STATIC_WORK_BYTES (256 MiB) that the library holds
 * on every GPU it runs on until the process ends; nothing is allocated or
 * freed here, and no events are recorded.  Same launches and results as
 * dgamr_step (cfl > 0: CFL time step; cfl <= 0: dt from dt_dev).  A forest
 * whose work area (dgamr_state_bytes) exceeds the array fails with
 * DGAMR_EUNSUPPORTED before anything is launched.  Every call on one GPU
 * shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (two streams, or two threads) race.  The forest's
 * device must be current. */
#define DGAMR_STATIC_WORK_BYTES (256u << 20)
int dgamr_step_static(dgamr_forest *f, double cfl, double *u, double *dt_dev, hipStream_t stream);

/* Sec. 4.3 step 2 repeated: nsteps SSP-RK3 steps in place on u, three
 * kernel launches per step.  With cfl > 0 the CFL time step of each step
 * after the first is folded into the previous step's last stage (its
 * new-state wave speeds are max-reduced on the device), so the results
 * equal nsteps calls of dgamr_step; dt_dev holds the last step's dt.  With
 * cfl <= 0 every step uses the dt already in dt_dev. */
int dgamr_run(dgamr_forest *f, double cfl, int nsteps, double *u, void *work, double *dt_dev,
              hipStream_t stream);

/* The same nsteps steps as dgamr_run (cfl > 0), captured once into a HIP
 * graph and replayed with dgamr_graph_launch: each launch advances u by
 * nsteps steps from its current contents, with the CFL time step of the
 * first step computed inside the graph and every later one folded into the
 * previous step's last stage; results equal dgamr_run's.  The graph holds
 * the pointers u, work and dt_dev.  The profiling hook is not recorded into
 * the graph.  Launching after a refinement of f fails with DGAMR_ESTATE. */
int dgamr_run_capture(dgamr_forest *f, double cfl, int nsteps, double *u, void *work, double *dt_dev,
                      dgamr_graph **out);

/* Conserved totals T_v = sum over cells |cell| * mean_v (FP64), written to
 * totals_dev[n_var]; a fixed-order reduction. */
int dgamr_conserved_totals(dgamr_forest *f, const double *u, double *totals_dev, void *work,
                           hipStream_t stream);

/* Positivity-preserving scaling limiter (Zhang-Shu, named in Sec. 5.3.2)
 * applied in place: each cell scaled about its mean (on bilinear /
 * trilinear roots, the mean over the physical cell).  EINVAL for scalar
 * equations. */
int dgamr_limit_positivity(dgamr_forest *f, double *u, hipStream_t stream);

/* Block indicator per leaf (FP64, device): Euler, max/min density cell mean
 * over the block's cells and face-guard cells; scalar convection, the
 * largest cell mean there (Sec. 5.1 refines on the cell average). */
int dgamr_indicator(dgamr_forest *f, const double *u, double *eta_dev, void *work,
                    hipStream_t stream);

/* L2 projection of an analytic state (DGAMR_IC_*, parameters as the test
 * workloads define them) with p+3 Gauss points per axis.  DGAMR_IC_COSINE
 * (scalar convection only): params k, L_x, L_y, L_z; the state is
 * prod_a [cos(2 pi k (x_a - vel_a t)/L_a) - 1] with the forest's velocity. */
int dgamr_project_ic(dgamr_forest *f, int kind, const double *params /* 8 */, double t,
                     double *u, hipStream_t stream);

/* Non-physical state check: sets *bad (host) to the number of cells with a
 * non-finite value or a non-positive mean density or pressure.  Synchronous. */
int dgamr_check_state(dgamr_forest *f, const double *u, int64_t *bad, void *work, hipStream_t stream);

/* Kernel tuning (for the autotuner and measurements; results do not
 * depend on it beyond floating-point rounding):
 *   DGAMR_TUNE_STAGE_VARIANT: stage kernel, -1 automatic (default),
 *     0 one lane per (cell, variable), 1 one thread per cell.  2-D: variant
 *     0 in row slabs for latency-bound small forests, 1 for throughput on
 *     large forests.  3-D (fused FP64 stage without the limiter or mortar
 *     faces; other forests always run variant 1): variant 0 in slabs of
 *     layers, automatic at degree 3;
 *   DGAMR_TUNE_VAR_SPLIT_MAX_CELLS: the automatic 2-D choice uses variant 0
 *     up to this many cells (default 131072);
 *   DGAMR_TUNE_SLAB_ROWS: layers of the block's last axis per stage
 *     workgroup (0 automatic, else a divisor of n_cell within the kernel's
 *     thread budget; a launch that does not fit fails with DGAMR_EHIP);
 *   DGAMR_TUNE_MFMA: FP32 residual (DGAMR_FP32 forests): 1 contracts the
 *     volume integral on the matrix cores (v_mfma_f32_16x16x4f32, FP32
 *     accumulation: 16 cells x 16 quadrature points or modes per tile) at
 *     degree 2 and 3 (3-D: degree 2) when a stage workgroup is whole waves
 *     of cells; 0 (default) on the vector unit.  The traces, face fluxes and
 *     lifting run on the vector unit either way.  With a few modes per cell
 *     the tiles are mostly padding, and the matrix cores' FP32 rate is twice
 *     the vector unit's (without packed FP32 instructions), so the vector
 *     unit, which also skips the basis tables' structural zeros, is as fast
 *     or faster on every measured forest. */
enum { DGAMR_TUNE_STAGE_VARIANT = 0, DGAMR_TUNE_VAR_SPLIT_MAX_CELLS = 1, DGAMR_TUNE_SLAB_ROWS = 2,
       DGAMR_TUNE_MFMA = 3 };
int dgamr_set_tuning(dgamr_forest *f, int knob, long value);

/* Measurement hook: while enabled, every launch of the fused stage kernel
 * inside dgamr_step is bracketed by two HIP events on the caller's stream
 * (not usable under HIP graph capture); on forests with rotated frames or
 * non-affine roots, whose stages are several launches, each stage's
 * launches (fill, residual, update, limiter) are bracketed together.  dgamr_profile_read waits for the
 * recorded events, returns the summed kernel time in milliseconds and the
 * number of launches, and clears the record. */
int dgamr_profile_enable(dgamr_forest *f, int enable);
int dgamr_profile_read(dgamr_forest *f, double *stage_ms, int64_t *stage_launches);

/* ---------------------------------------------------------------------
 * Pools: many forests stepped together (batched and served solves).
 *
 * Not a construct of the paper: it applies the same per-stage residual and
 * SSP-RK3 update (Sec. 2-3) to many independent forests in each launch.  A
 * pool is a device-resident arena of leaf slots for forests of one class:
 * dim, degree, n_cell, gamma, precision, hanging and limiter of the class
 * descriptor (its roots, lo, hi, bc and max_level are ignored).  Admitting
 * a forest copies its topology into a contiguous range of free slots; the
 * member's state lives in the caller's state arena at that range, in the
 * layout of the forest's own state buffer (dgamr_state_bytes), and the
 * caller writes it (e.g. dgamr_project_ic of the forest into the arena at
 * slot_first).  A pool step advances every member by one SSP-RK3 step with
 * its own CFL time step; a member's arithmetic does not depend on the other
 * members, so its result is the same alone and in any mix.
 *
 * Ownership: the pool owns its topology tables (device and pinned host);
 * the caller owns the state arena and the work buffer (sizes from
 * dgamr_pool_bytes for the capacity).  Admit and release enqueue table
 * uploads on the given stream; steps on the same stream see them in order.
 * A released member's slots keep their contents until the next admission.
 * Pools are not thread-safe.  The stage kernel is chosen as for a single
 * forest of the class (3-D degree 3: one lane per (cell, variable); else
 * one thread per cell) until dgamr_pool_set_shape, dgamr_pool_set_lanes or
 * dgamr_pool_autotune changes it.
 * --------------------------------------------------------------------- */
typedef struct dgamr_pool dgamr_pool;

int dgamr_pool_create(const dgamr_forest_desc *cls, int64_t capacity_leaves, int32_t max_members,
                      dgamr_pool **out);
int dgamr_pool_destroy(dgamr_pool *p);
/* bytes of the state arena (capacity leaves) and of the work buffer */
int dgamr_pool_bytes(const dgamr_pool *p, size_t *state_bytes, size_t *work_bytes);
/* Admit forest f (same class) with CFL number cfl: on success *member is its
 * id (0 <= id < max_members) and *slot_first the first of its n_leaves
 * consecutive slots.  DGAMR_EFULL when no free range or id is left. */
int dgamr_pool_admit(dgamr_pool *p, const dgamr_forest *f, double cfl, int32_t *member, int64_t *slot_first,
                     hipStream_t stream);
int dgamr_pool_release(dgamr_pool *p, int32_t member, hipStream_t stream);
/* One SSP-RK3 step of every member: per-member dt from the CFL condition,
 * then three fused stage launches over the listed leaves of all members. */
int dgamr_pool_step(dgamr_pool *p, double *u_arena, void *work, hipStream_t stream);
/* Device address of the per-member dt of the last step (max_members
 * doubles inside work). */
int dgamr_pool_dt(const dgamr_pool *p, void *work, double **dt_dev);
/* Leaves in use and active members (host). */
int dgamr_pool_stats(const dgamr_pool *p, int64_t *leaves_used, int32_t *members);
/* Launch shape of the pool's stage kernel (the thread-per-cell kernel):
 * rows = layers of the block's last axis per workgroup (0 = largest
 * allowed), grid = workgroups of a persistent launch (0 = one per work
 * item). */
int dgamr_pool_set_shape(dgamr_pool *p, int32_t rows, int32_t grid);
/* Launch shape of the pool's stage kernel (the lane-per-(cell, variable)
 * kernel, for FP64 classes without the limiter and, in 3-D, without mortar
 * faces): rows = rows of cells (2-D, 4 rows N <= 512) or whole layers (3-D,
 * at least two unless the whole block, at most 144 cells) per workgroup,
 * 0 = the kernel's own choice.  DGAMR_EINVAL for other classes or rows. */
int dgamr_pool_set_lanes(dgamr_pool *p, int32_t rows);
/* Autotuner: times the stage kernel on the pool's current members for every
 * allowed (rows, grid) pair of the thread-per-cell kernel and, for the
 * classes dgamr_pool_set_lanes accepts, every slab height of the
 * lane-per-(cell, variable) kernel, and keeps the fastest; writes the choice (variant 1
 * thread per cell, 0 lane per variable; rows; grid) and its average launch
 * time in microseconds (any output pointer may be null).  Synchronous; the state
 * arena is read, the work buffer overwritten. */
int dgamr_pool_autotune(dgamr_pool *p, double *u_arena, void *work, hipStream_t stream, int32_t *variant,
                        int32_t *rows, int32_t *grid, double *best_us);

/* HIP graph of nsteps steps of several pools, captured once and replayed
 * with dgamr_graph_launch: one branch per pool holding its nsteps steps in
 * order, the branches independent (pools share no memory), so the device
 * runs the pools' launches concurrently.  A graph holds the
 * pools' work-list lengths at capture: launching it after an admit or
 * release on any of its pools fails with DGAMR_ESTATE. */
int dgamr_pools_capture(dgamr_pool *const *pools, double *const *u_arenas, void *const *works, int32_t npools,
                        int32_t nsteps, dgamr_graph **out);
int dgamr_graph_launch(dgamr_graph *g, hipStream_t stream);
int dgamr_graph_destroy(dgamr_graph *g);

/* Accuracy check of the device arithmetic the stage kernels use for the
 * density reciprocal and the wave-speed square root (Newton-Raphson and
 * Goldschmidt iterations from the hardware estimates): y[i] = 1/x[i]
 * (fn 0) or sqrt(x[i]) (fn 1, 0 for x <= 0), n doubles in device memory,
 * asynchronous on the stream. */
int dgamr_math_probe(int fn, const double *x, double *y, int64_t n, hipStream_t stream);

const char *dgamr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
