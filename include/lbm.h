/*
 * lbm.h -- C-ABI of the MI355X refined-grid lattice Boltzmann library
 * (liblbm.so).  The operations follow the problem statement of Coreixas &
 * Latt, arXiv 2504.04465: a static cell-centred quad/octree given by level
 * masks (Secs. 4.3-4.4), populations started at equilibrium from macroscopic
 * fields (App. A.3), an asynchronous multi-level time loop (Sec. 4.5) with
 * Rohde coalescence / uniform explosion at interfaces (Sec. 3.2, Eqs.
 * coalescence and explosion_uniform), and macroscopic output.
 *
 * Conventions for every entry point:
 *   - Levels are numbered 0 = coarsest; level l takes 2^l substeps per coarse
 *     step (the paper numbers them the other way).
 *   - Host pointers are owned by the caller and only accessed during the call.
 *   - Device memory is owned by the library.  It is obtained through the
 *     allocator given to lbm_create (or hipMalloc when none is given) and
 *     released by lbm_destroy.
 *   - Every call returns an lbm_status; no exception crosses the ABI.  The
 *     text of the last error is available from lbm_last_error.
 *   - Numerical failures inside lbm_step (NaN / Inf populations, Newton
 *     iterations exhausted) are latched on the device and reported as
 *     LBM_E_NUMERIC by the next synchronous call (lbm_sync, lbm_moments,
 *     lbm_stats).  The latch stays set until lbm_init.
 *   - Cells are in canonical order: level-major, Morton (Z-order) order inside
 *     a level with x in the lowest key bit, then y, then z.
 *   - Dense arrays are indexed with x fastest, then y, then z.
 *   - One context per host thread; calls on a context are not re-entrant.
 *     All device work of a context is enqueued on its stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_ARG = -1,         /* invalid argument                                  */
  LBM_E_MASK = -2,        /* inconsistent level / solid masks or faces         */
  LBM_E_NOMEM = -3,       /* allocation failed                                 */
  LBM_E_DEVICE = -4,      /* HIP runtime error                                 */
  LBM_E_STATE = -5,       /* call out of order (no grid, not initialised, ...) */
  LBM_E_NUMERIC = -6,     /* NaN / Inf or Newton failure latched on device     */
  LBM_E_UNSUPPORTED = -7  /* valid but unsupported combination                 */
} lbm_status;

/* lattices of App. A.1 (D3Q27 = D1Q3 x D1Q3 x D1Q3) */
enum { LBM_D2Q9 = 0, LBM_D3Q27 = 1, LBM_D2Q21 = 2, LBM_D2Q37 = 3, LBM_D2Q13 = 4 };

/* collision models of App. A.2:
 *   BGK            Eq. CollisionStep with the polynomial equilibrium Eq. GenEq
 *   RR             recursive regularisation, Eq. GenRegCollision
 *                  (BGK and RR: D2Q9 and D3Q27 on the product basis, D2Q13
 *                  and D2Q21 on the full third-order basis; all storages)
 *   DDF_POLY       double distribution, fourth-order thermal polynomial
 *                  equilibrium, g_eq of Eq. gEq, BGK on f and g (D2Q37)
 *   DDF_NEWTON     double distribution, numerical equilibrium Eq. exponential
 *                  solved by Newton on the eight constraints (D2Q21, D2Q13,
 *                  D2Q37)
 *   DDF_MLP        as DDF_NEWTON, multipliers predicted by the MLP only
 *   DDF_MLP_NEWTON MLP prediction + one Newton step, full Newton wherever the
 *                  constraint residual still exceeds fallback_tol            */
enum { LBM_BGK = 0, LBM_RR = 1, LBM_DDF_POLY = 2, LBM_DDF_NEWTON = 3,
       LBM_DDF_MLP = 4, LBM_DDF_MLP_NEWTON = 5 };

/* population storage; collisions run in FP64 for LBM_FP64 and in FP32
 * otherwise (Newton always in FP64) */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_SHIFTED = 2 /* stores f_i - w_i */ };

/* face boundary conditions (App. A.3) */
enum { LBM_BC_PERIODIC = 0,    /* faces 2a and 2a+1 must both be periodic     */
       LBM_BC_WALL = 1,        /* staircase bounce-back                        */
       LBM_BC_MOVING_WALL = 2, /* Ladd velocity bounce-back, wall density 1   */
       LBM_BC_NEUMANN = 3,     /* copy of the nearest fluid cell, B layers     */
       LBM_BC_EQUILIBRIUM = 4  /* equilibrium Dirichlet, B layers              */ };

/* node flags reported by lbm_grid_export */
enum { LBM_F_COARSE_GHOST = 1, LBM_F_FINE_GHOST = 2, LBM_F_BC_NEUMANN = 4,
       LBM_F_BC_EQ = 8, LBM_F_SPONGE = 16 };

/* neighbour-list sentinels reported by lbm_grid_export */
enum { LBM_NBR_NONE = -1, LBM_NBR_SOLID = -2 /* moving wall on face k: -3-k */ };

typedef struct {
  int lattice;             /* LBM_D2Q9 ...                                   */
  int collision;           /* LBM_BGK ...                                    */
  int storage;             /* LBM_FP64 ...                                   */
  double nu_finest;        /* viscosity, lattice units of the finest level;
                              <= 0: inviscid, tau = 1/2 on every level       */
  double T0;               /* reference temperature (DDF), tau = nu/T0 + 1/2 */
  double gamma;            /* specific heat ratio (DDF), Cv = 1/(gamma-1)    */
  double sensor_A;         /* alpha on [0.1, 1) of Eq. shock_function        */
  int sensor_on;           /* kinetic sensor, Eqs. DeltaAvg / shock_function */
  int trace_equilibration; /* RR: bulk relaxation time one on the trace      */
  double newton_tol;       /* stop when max_a |G_a| / rho <= newton_tol      */
  double fallback_tol;     /* MLP_NEWTON: full Newton above this residual    */
  int newton_max_it;       /* Newton iteration cap (failure latches NUMERIC) */
  int lambda_warm_start;   /* 1: start Newton from the stored multipliers    */
  int host_only;           /* 1: build the grid on the host only; no device
                              call is made and init/step return LBM_E_STATE  */
  int in_place;            /* 1: stream in place on one population buffer
                              (AA pattern: even steps read and write the
                              cell's own rows, the opposite row for the
                              result; odd steps pull from and push to the
                              neighbours), half the population memory.  One
                              level only, periodic / wall / moving-wall
                              faces, no sponge, no surrogate; otherwise
                              lbm_grid_build returns LBM_E_UNSUPPORTED.
                              Results are identical to two buffers.      */
} lbm_params;

typedef struct {
  int kind;                /* LBM_BC_*                                        */
  double rho, u[3], T;     /* moving-wall velocity, or equilibrium state     */
  int extrapolate_rho;     /* equilibrium: take rho from the source cell     */
  double sponge_sigma_max; /* pressure sponge strength at this face (Eq.
                              relaxation_pressure, linear ramp)              */
  double sponge_width;     /* ramp width in coarse cells                     */
} lbm_face_bc;

/* A mask restricted to a box [lo, lo + n) of one level's cell coordinates;
 * values outside the box are 0.  data holds n[0]*n[1]*n[2] bytes, x fastest. */
typedef struct {
  const uint8_t *data;
  int32_t lo[3];
  int32_t n[3];
} lbm_mask;

typedef void *(*lbm_dev_alloc_fn)(size_t bytes, void *alloc_ctx);
typedef void (*lbm_dev_free_fn)(void *ptr, void *alloc_ctx);

/* Create a context.  dev_alloc / dev_free may be NULL (hipMalloc / hipFree are
 * then used); hip_stream may be NULL (the null stream).  Errors: LBM_E_ARG
 * for an unknown lattice / collision / storage or an unsupported combination
 * (LBM_E_UNSUPPORTED), LBM_E_NOMEM. */
lbm_status lbm_create(const lbm_params *params, lbm_dev_alloc_fn dev_alloc,
                      lbm_dev_free_fn dev_free, void *alloc_ctx,
                      void *hip_stream, lbm_ctx **out);

/* Build the static tree and every derived table (Secs. 4.3-4.4): cells per
 * level in canonical order, flags, the pull neighbour list (source x - xi_i
 * on the same level), the coarse-ghost list with its child table and unknown
 * populations, boundary layers, sponge strength.  refine[l-1] (l = 1 ..
 * n_levels-1) has level l-1 resolution and marks the cells refined to level
 * >= l; solid[l] (may be NULL, or have NULL data) marks level-l cells whose
 * centre is inside a body.  faces: x-, x+, y-, y+, z-, z+ (z faces ignored in
 * 2-D).  The grid is uploaded to the device unless host_only.  Errors:
 * LBM_E_ARG (bad sizes), LBM_E_MASK (refinement not nested, interfaces closer
 * than B cells of the coarser level, a solid body cutting an interface, a
 * boundary layer overlapping an interface, unpaired periodic faces),
 * LBM_E_NOMEM, LBM_E_DEVICE.  Replaces any previous grid and state. */
lbm_status lbm_grid_build(lbm_ctx *ctx, int dim, const int32_t ext_coarse[3],
                          int n_levels, const lbm_mask *refine,
                          const lbm_mask *solid, const lbm_face_bc faces[6]);

/* Where lbm_grid_build and lbm_remesh construct the tree and its brick
 * layout (Secs. 4.3-4.4; Sec. 8 names the host-side tree construction as
 * the cost of remeshing): on = 1 (the default) builds them on the GPU,
 * every rule of the construction applied per cell in parallel (Z order by
 * a radix sort of Morton keys, lists by prefix sums), and copies the result
 * into the context's host copy; on = 0 builds them on the host.  Both give
 * the same grid value for value and the same errors.  Host-only contexts
 * always build on the host.  Takes effect at the next build.  Errors:
 * LBM_E_ARG (null context). */
lbm_status lbm_set_device_build(lbm_ctx *ctx, int on);

/* Cell counts; n_per_level has n_levels entries.  eq_fine_cells is
 * sum_l n_l / 2^(L-1-l) (Sec. 7.5, "equivalent fine cells").  Any output
 * pointer may be NULL. */
lbm_status lbm_grid_info(lbm_ctx *ctx, int64_t *n_cells, int64_t *n_per_level,
                         int64_t *n_coarse_ghosts, double *eq_fine_cells);

/* Device placement of the grid (Sec. 4.4 gives the paper's own layout; this
 * one differs): the cells of each level sit in bricks of 64 slots (4x4x4 in
 * 3-D, 8x8 in 2-D) in Z order, one brick per wavefront.  A cell whose pull
 * sources all follow from its brick's neighbour bricks reads no neighbour
 * list; every other cell (ghosts, boundary layers, cells next to walls or
 * bodies) has an explicit row of pull sources.  n_slots counts the slots of
 * all levels including the unused ones of partly filled bricks;
 * n_exception_rows the cells with an explicit row; slots_per_level and
 * rows_per_level have n_levels entries.  Any output pointer may be NULL. */
lbm_status lbm_layout_info(lbm_ctx *ctx, int64_t *n_slots, int64_t *n_exception_rows,
                           int64_t *slots_per_level, int64_t *rows_per_level);

/* The brick layout of the grid (Sec. 4.4 data layout, as placed for the
 * device), for inspection and tests: slot_of [n_cells] the slot of each
 * canonical cell; xrow_of [n_cells] its exception row or -1; nbrick
 * [n_slots / 64][nbp] the neighbour brick ids (nbp = 16 in 2-D, 32 in 3-D;
 * -1 where there is none); xmask [n_slots / 64] the lanes with exception
 * rows; xnbr [Q-1][n_rows] the pull sources of the exception rows (slot,
 * coalesced slot >= n_slots, -1 bounce-back, -2 - k moving wall of face k).
 * Sizes from lbm_layout_info; any pointer may be NULL.  Errors: LBM_E_ARG,
 * LBM_E_STATE (no grid). */
lbm_status lbm_layout_export(lbm_ctx *ctx, int32_t *slot_of, int32_t *xrow_of, int32_t *nbrick, uint64_t *xmask,
                             int32_t *xnbr);

/* Export the tables in canonical form (any pointer may be NULL):
 * coords [n][3], level [n], flags [n], nbr [n][Q-1] (sentinels above),
 * child [n_coarse_ghosts][2^D] (octant o = cx | cy<<1 | cz<<2, -1 missing),
 * bc_src [n] (-1 for non-boundary cells). */
lbm_status lbm_grid_export(lbm_ctx *ctx, int32_t *coords, int8_t *level,
                           uint8_t *flags, int32_t *nbr, int32_t *child,
                           int32_t *bc_src);

/* Start every cell (ghosts included) at equilibrium (App. A.3): moments is a
 * host array [n_mom][n_cells], n_mom = 1 + D (+1 temperature for DDF):
 * rho, u_x, u_y, (u_z), (T).  D2Q21 multipliers come from a cold Newton.
 * Clears the numeric latch and the counters.  Synchronous. */
lbm_status lbm_init(lbm_ctx *ctx, const double *moments);

/* Enqueue n coarse steps: per coarse step 2^(L-1) finest substeps; at each
 * substep the active levels run coarsest first (coupling then collide-and-
 * stream, Sec. 4.5).  Does not synchronise. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n_coarse_steps);

/* Replace the values of a face (same kind), e.g. an inlet Mach ramp; takes
 * effect for work enqueued afterwards. */
lbm_status lbm_set_face_bc(lbm_ctx *ctx, int face, const lbm_face_bc *bc);

/* Replay pairs of coarse steps from a HIP graph (on: 1) instead of launching
 * every kernel (the scheduler of Sec. 4.5 issues ~10 launches per level per
 * coarse step, which dominates on small grids).  Two coarse steps return
 * every level's buffer parity to its start, so one captured graph serves
 * every later pair while the parities, face values and grid are unchanged;
 * it is re-captured otherwise.  lbm_step then advances pairs from the graph
 * and single steps by launches; results are identical.  Off by default; not
 * used while profiling.  The context's stream must not be the null stream
 * (capture is refused there and lbm_step launches as usual). */
lbm_status lbm_set_graphs(lbm_ctx *ctx, int on);

/* Concurrent levels (Sec. 4.5; the paper's remedy for small levels that
 * leave most of the GPU idle): with on != 0 (the default) every substep
 * at which two or more levels are active runs their collide-and-stream
 * updates as one launch whose blocks span all those levels, after the
 * substep's coalescences and before its boundary fills and explosions;
 * results are identical to per-level launches.  Used where the model has
 * it (BGK, RR and the polynomial double distribution; the Newton and
 * surrogate models keep per-level launches), with two buffers, and not
 * while kernel timing is enabled (timing is per level).  Errors: LBM_E_ARG
 * for a null context. */
lbm_status lbm_set_level_fusion(lbm_ctx *ctx, int on);

/* Inflow noise (the seeded perturbation of the cylinder's inflow): du, a
 * host array [3][n_cells] in canonical cell order, is added per cell to the
 * face velocity in Ladd's moving-wall term (App. A.3) of every moving-wall
 * link of the cell; other cells ignore their entries.  The values are
 * caller-owned and copied; NULL removes the perturbation.  A new grid
 * (lbm_grid_build, lbm_remesh) starts without it.  Synchronous.  Errors:
 * LBM_E_STATE without a grid on the device, LBM_E_ARG for non-finite
 * values, LBM_E_UNSUPPORTED with in-place streaming or the Newton /
 * surrogate equilibria, LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_set_inflow_noise(lbm_ctx *ctx, const double *du);

/* Macroscopic fields of the state at the synchronisation point (pre-
 * collision populations, coarse ghosts with coalesced unknowns; fine ghosts
 * are NaN), written to the host array out [n_mom][n_cells].  Synchronous. */
lbm_status lbm_moments(lbm_ctx *ctx, double *out);

/* As lbm_moments but into device memory out_dev [n_mom][n_cells]; enqueued
 * on the context stream, no synchronisation. */
lbm_status lbm_moments_device(lbm_ctx *ctx, double *out_dev);

typedef struct {
  double mass, momentum[3], energy; /* sum over non-fine-ghost cells of
                                       2^(-D l) sum_i (1, xi, |xi|^2/2) f_i
                                       (+ g/2 for DDF), FP64              */
  double kinetic_energy;            /* sum over the same cells of
                                       2^(-D l) rho |u|^2 / 2 (the monitor
                                       of the convergence test, Sec. 5.2) */
  int64_t updates[8];               /* cell updates per level             */
  int64_t newton_calls, newton_iterations, newton_failures;
  int64_t mlp_fallbacks, nonfinite_cells;
  int64_t coarse_steps;
  int64_t newton_hist[16];          /* Newton solves of the collisions by
                                       steps taken: bin k < 15 counts solves
                                       of k steps, bin 15 longer ones and
                                       failures (per-cell iteration counts
                                       as a stability monitor, Sec. 4.4)  */
} lbm_stats;

/* Conservation sums and counters; synchronous. */
lbm_status lbm_stats_get(lbm_ctx *ctx, lbm_stats *out);

/* Allocation-free variant of the conservation sums of lbm_stats_get, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Writes
 * out_dev[6] = {mass, momentum x, y, z, total energy, kinetic energy}, the
 * same values lbm_stats_get reports, bit for bit, into caller-owned device
 * memory; enqueued on the context stream, no synchronisation, no device or
 * host allocation.  The block partials live in a static device array of
 * 8 x 1024 x 6 + 6 doubles (384 KiB) that each GPU holds until the process
 * ends; every context on a GPU shares it, so calls that overlap on one GPU
 * (two streams, or two threads) race and must be serialised by the caller.
 * Limit: grids of at most 8 levels (any number of cells); more -> LBM_E_ARG.
 * Errors: LBM_E_STATE before lbm_init, LBM_E_ARG for a null out_dev,
 * LBM_E_DEVICE if the array's device address could not be obtained when
 * the context was created, or a launch failed. */
lbm_status lbm_sums_device(lbm_ctx *ctx, double *out_dev);

/* Wait for all enqueued work; reports a latched numeric failure. */
lbm_status lbm_sync(lbm_ctx *ctx);

/* Kernel timing: when enabled, every collide-and-stream launch is bracketed
 * by HIP events on the context stream.  lbm_profile_read synchronises and
 * returns, for level l, the number of timed launches, their summed duration
 * in milliseconds, and the algorithmic bytes one update of that level moves
 * (read + write of the populations, neighbour indices and multipliers). */
lbm_status lbm_profile_enable(lbm_ctx *ctx, int on);
lbm_status lbm_profile_read(lbm_ctx *ctx, int level, int64_t *launches,
                            double *total_ms, double *bytes_per_update);

/* Checkpoint: raw state in canonical cell order, FP64 on the host:
 * f [Q][n_cells] (pre-collision, as at the synchronisation point),
 * g [Q][n_cells] (DDF only, else may be NULL), lambda [8][n_cells] (D2Q21
 * only, else may be NULL).  lbm_set_state restores such a state. */
lbm_status lbm_get_state(lbm_ctx *ctx, double *f, double *g, double *lambda);

/* Kinetic sensor of every cell at the synchronisation point (Eq.
 * DeltaAvg): eps = mean over i of |f_i - f_eq,i| / |f_eq,i|, with f_eq the
 * collision model's equilibrium at the cell's own moments (Newton
 * warm-started from the stored multipliers, which are not changed), on f
 * only; NaN for fine ghosts.  eps: host array [n_cells], canonical order.
 * The paper refines where eps exceeds 0.2 (Sec. 8).  Errors: LBM_E_STATE
 * without a state. */
lbm_status lbm_sensor(lbm_ctx *ctx, double *eps);

/* Mesh adaptation (Sec. 8, methodology of the adaptive runs): replaces the
 * grid by the one the new refinement masks (and solid masks, as in
 * lbm_grid_build; extent, level count and faces unchanged) describe, and
 * moves the state across at the synchronisation point.  Every new cell,
 * ghosts included, takes the pre-collision populations (and multipliers)
 * of the old grid's cells other than fine ghosts (coarse ghosts with their
 * unknown populations coalesced; these cells tile the domain): copied
 * from the old cell at the same place and level, or from the old cell that
 * contains it where the old grid is coarser (uniform explosion), or
 * averaged over the old cells inside it, weighted by volume, where the old
 * grid is finer (coalescence).  The move runs on the device; the new tree
 * is built on the host.  Cell numbering, layout and all device buffers are
 * replaced (re-read lbm_grid_info / lbm_grid_export); step and update
 * counts carry over, Newton / surrogate counters restart, surrogate
 * weights are kept.  Errors: LBM_E_STATE without a state; LBM_E_MASK for
 * inconsistent masks (the context then has neither grid nor state) or for
 * a new fluid cell over old solid cells (then it has the new grid and no
 * state); LBM_E_NOMEM.  The old state is lost on any error. */
lbm_status lbm_remesh(lbm_ctx *ctx, const lbm_mask *refine, const lbm_mask *solid);
lbm_status lbm_set_state(lbm_ctx *ctx, const double *f, const double *g,
                         const double *lambda);

/* The state of the listed cells only (same content as lbm_get_state, at the
 * synchronisation point of Sec. 4.5): cells [n] canonical indices; f [Q][n],
 * g [Q][n] (DDF), lambda [8][n] (Newton family, may be NULL), host arrays
 * owned by the caller, entry k for cells[k].  Lets a caller sample a large
 * grid without copying all of it.  Errors: LBM_E_ARG (index out of range),
 * LBM_E_STATE, LBM_E_DEVICE. */
lbm_status lbm_get_cells(lbm_ctx *ctx, const int64_t *cells, int64_t n, double *f, double *g,
                         double *lambda);

/* ---- multiplier surrogate (D2Q21 contexts) ----------------------------
 * A small network replaces the per-cell Newton solve of the numerical
 * equilibrium (App. A.2, Eq. exponential, constraints G(0)..G(3)): it maps
 * (rho, u_x, u_y, T) to the eight multipliers.  Network 4 -> 64 -> 64 -> 64
 * -> 8, SiLU hidden layers, evaluated and trained on BF16 matrix cores with
 * FP32 accumulation and FP32 master weights (Adam).  Packed parameters, 9176
 * floats: W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[8][64]
 * b4[8] mu[8] sigma[8]; inputs are normalised as ((rho-2.6)/2.4, u_x/2.5,
 * u_y/2.5, (T-1.75)/1.25), outputs as lambda = mu + sigma * y.  The network
 * is evaluated on the canonical state u_x >= u_y >= 0; the multipliers of
 * any state follow from the lattice's reflection symmetry (x / y swap and sign
 * flips of the odd multipliers), so predictions are exactly symmetric.  Host arrays
 * are row-major per sample.  LBM_E_ARG when the context is not D2Q21, or a
 * size is not a multiple of 32 where one is required. */
enum { LBM_MLP_PARAMS = 9176 };

lbm_status lbm_mlp_set_weights(lbm_ctx *ctx, const float *w, int64_t n);
lbm_status lbm_mlp_get_weights(lbm_ctx *ctx, float *w, int64_t n);

/* Newton labels (FP64, cold start lambda = 0, the context's newton_tol and
 * newton_max_it): x [n][4] = (rho, u_x, u_y, T) -> lambda [n][8];
 * ok[i] = 1 when converged (unrealisable moments do not converge);
 * iterations[i] = Newton iterations (-1 when not converged). */
lbm_status lbm_mlp_label(lbm_ctx *ctx, const double *x, int64_t n, double *lambda, uint8_t *ok,
                         int32_t *iterations);

/* Surrogate prediction: x [n][4] -> lambda [n][8]. */
lbm_status lbm_mlp_predict(lbm_ctx *ctx, const double *x, int64_t n, double *lambda);

/* Loss (mean Huber loss, delta 0.5, on normalised outputs) and its gradient with
 * respect to the packed parameters (9160 trainable entries) for one batch of
 * normalised inputs xh [n][4] and targets th [n][8]; n a multiple of 32. */
lbm_status lbm_mlp_grad(lbm_ctx *ctx, const float *xh, const float *th, int64_t n, double *loss,
                        float *grad);

/* Train on samples x [n][4] with Newton labels lambda [n][8]: mu / sigma are
 * taken from the labels, weights start from the ones set (or a seeded
 * initialisation), `epochs` passes in seeded random order, mini-batches of
 * `batch` (multiple of 32), Adam with a cosine-decayed learning rate.
 * epoch_loss [epochs] receives the mean training loss of every pass. */
lbm_status lbm_mlp_train(lbm_ctx *ctx, const double *x, const double *lambda, int64_t n, int epochs,
                         int batch, double lr, uint64_t seed, double *epoch_loss);

const char *lbm_last_error(const lbm_ctx *ctx);
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
