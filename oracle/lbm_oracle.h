/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the refined-grid lattice Boltzmann
 * update (Coreixas & Latt, arXiv 2504.04465).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product library
 * never links or calls it, and the two share no code.
 *
 * Conventions (readings of the paper are listed in the design notes):
 *   - levels are numbered 0 = coarsest; level l takes 2^l substeps per coarse
 *     step (the paper numbers them the other way, Sec. 4.5);
 *   - populations are pre-collision values, stored cell-major (AoS);
 *   - every array is indexed with x fastest, then y, then z.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OL_D2Q9 = 0, OL_D3Q27 = 1, OL_D2Q21 = 2, OL_D2Q37 = 3, OL_D2Q13 = 4 };
enum { OL_BGK = 0, OL_RR = 1, OL_DDF_POLY = 2, OL_DDF_NEWTON = 3 };
enum { OL_BC_PERIODIC = 0, OL_BC_WALL = 1, OL_BC_MOVING_WALL = 2,
       OL_BC_NEUMANN = 3, OL_BC_EQUILIBRIUM = 4 };
enum { OL_NONE = -1, OL_SOLID = -2 }; /* moving wall on face k: -3-k */
enum { OL_F_COARSE_GHOST = 1, OL_F_FINE_GHOST = 2, OL_F_BC_NEUMANN = 4,
       OL_F_BC_EQ = 8, OL_F_SPONGE = 16 };

typedef struct {
  int kind;
  double rho, u[3], T;
  int extrapolate_rho;
  double sponge_sigma_max, sponge_width; /* width in coarse cells */
} ol_face;

typedef struct {
  int lattice, collision;
  double nu_finest;      /* <= 0: inviscid, tau = 1/2 on every level */
  double T0, gamma, sensor_A;
  int sensor_on, trace_eq;
  double newton_tol;
  int newton_max_it, warm_start;
} ol_params;

typedef struct ol_sim ol_sim;

ol_sim *ol_create(const ol_params *p);
void ol_destroy(ol_sim *s);
const char *ol_error(const ol_sim *s);

/* lattice description: c[Q*3], w[Q], opp[Q] */
int ol_lattice(const ol_sim *s, int *D, int *Q, int *B, int *c, double *w,
               double *cs2, int *opp);

/* grid (Sec. 3-4): refine[l-1] (l=1..L-1) has level l-1 resolution;
 * solid[l] (may be NULL) has level l resolution. */
int ol_grid(ol_sim *s, int dim, const int32_t ext[3], int n_levels,
            const uint8_t *const *refine, const uint8_t *const *solid,
            const ol_face faces[6]);
int64_t ol_n_cells(const ol_sim *s);
int ol_level_counts(const ol_sim *s, int64_t *n_per_level);
int64_t ol_n_ghosts(const ol_sim *s);
int ol_export(const ol_sim *s, int32_t *coords, int8_t *level, uint8_t *flags,
              int32_t *nbr, int32_t *child, int32_t *bc_src);

int ol_init(ol_sim *s, const double *moments);
int ol_step(ol_sim *s, int64_t n_coarse_steps);
int ol_moments(ol_sim *s, double *out);
int ol_sums(ol_sim *s, double *out); /* mass, momentum[D], energy (DDF) */
/* sum of 2^(-D l) rho |u|^2 / 2 over the cells that are not fine ghosts */
int ol_kinetic_energy(ol_sim *s, double *out);
int ol_set_face(ol_sim *s, int face, const ol_face *f);
/* per-cell perturbation of the moving-wall velocity ("inflow noise"):
 * du SoA [3][n] in canonical cell order, added to the face velocity in the
 * Ladd term of every moving-wall link of the cell; NULL removes it */
int ol_set_inflow_noise(ol_sim *s, const double *du);
int ol_counters(const ol_sim *s, int64_t *updates_per_level,
                int64_t *newton_iters, int64_t *newton_calls);
int ol_get_state(const ol_sim *s, double *f, double *g, double *lam);
/* the synchronisation-point state: as ol_get_state, with the unknown
 * populations of every coarse ghost coalesced from its children */
int ol_get_sync_state(ol_sim *s, double *f, double *g, double *lam);
/* kinetic sensor (Eq. DeltaAvg) of every cell at the synchronisation
 * point against the equilibrium at its own moments; NaN for fine ghosts */
int ol_sensor(ol_sim *s, double *eps);
/* replaces the state of every cell by the given pre-collision populations
 * (and multipliers); [n][Q] / [n][8] like ol_get_state */
int ol_set_state(ol_sim *s, const double *f, const double *g, const double *lam);

/* single-cell routines (tau given, no sponge) */
int ol_feq(ol_sim *s, double rho, const double *u, double T, double *feq,
           double *geq, double *lam);
int ol_collide(ol_sim *s, double tau, const double *f, const double *g,
               double *fs, double *gs, double *lam, double *eps_out);
int ol_newton(ol_sim *s, const double *u, double T, double *lam, double tol,
              int max_it);
double ol_tau(const ol_sim *s, int level);

#ifdef __cplusplus
}
#endif
#endif
