/*
 * lbm_oracle.c -- plain, slow, FP64 CPU oracle of the refined-grid lattice
 * Boltzmann update of Coreixas & Latt (arXiv 2504.04465).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code, header or table with
 * the HIP library.
 *
 * The oracle follows the paper's steps in its notation and order:
 *   - lattices and weights: Table "lattices_structure" (App. A.1), the D2Q37
 *     weights re-solved from the eighth-order isotropy conditions;
 *   - Hermite tensors and equilibria: App. A.2, Eqs. GenEq and
 *     RecursivityEquilibrium; recursive regularisation: Eq. GenRegCollision and
 *     the non-equilibrium recursion that follows it;
 *   - numerical equilibrium: Eqs. exponential, Hfunction, constraints and the
 *     eight moment constraints G(0)..G(3) that follow; DDF closure: Eqs. gEq
 *     and polyTemp; kinetic sensor: Eqs. DeltaAvg and shock_function;
 *   - Rohde coupling: Eqs. coalescence and explosion_uniform (Sec. 3.2);
 *     level scheduler: Sec. 4.5; grid layout: Secs. 4.3-4.4;
 *   - boundary conditions: App. A.3; pressure sponge: Eq. relaxation_pressure.
 *
 * Storage is cell-major (AoS) pre-collision populations, double buffered.
 * Loops over the cells of one level-substep are order-independent, so the
 * optional OpenMP pragmas do not change any result.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 37
#define MAXM 32
#define NLAM 8
#define MAXL 8

struct ol_sim {
  ol_params p;
  char err[256];
  /* lattice */
  int D, Q, B;
  int c[MAXQ][3];
  double w[MAXQ];
  double cs2;
  int opp[MAXQ];
  int nm;
  int m[MAXM][3];
  double H[MAXQ][MAXM];
  double Cv;
  double mom[MAXQ][NLAM]; /* numerical-equilibrium moment vectors */
  /* grid */
  int have_grid, dim, L;
  int32_t ext[3];
  ol_face face[6];
  int64_t n, off[MAXL + 1];
  int32_t *xyz;
  int8_t *lev;
  uint8_t *flag;
  int32_t *nbr;
  int64_t ng, goff[MAXL + 1];
  int32_t *ghost, *child;
  int32_t *bcsrc;
  int8_t *bcface;
  double *sigma, *rho_inf;
  double *wall_du; /* [n][3] inflow noise on moving-wall links, or NULL */
  double tau[MAXL];
  /* state */
  int have_state;
  double *f, *fs, *g, *gs, *lam;
  uint8_t *collided;
  int64_t upd[MAXL], newton_it, newton_calls;
  int numeric_error;
};

static int fail(ol_sim *s, int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(s->err, sizeof s->err, fmt, ap);
  va_end(ap);
  return code;
}

/* ------------------------------------------------------------------------ */
/* Lattices (App. A.1, Table lattices_structure; D3Q27 = D1Q3^3)             */
/* ------------------------------------------------------------------------ */

static int iabs_(int a) { return a < 0 ? -a : a; }

/* group weight of velocity (a,b,cz); returns 0 if not in the lattice */
static int group_of(int lat, const int *v, int *grp) {
  int a = iabs_(v[0]), b = iabs_(v[1]), cz = iabs_(v[2]);
  int hi = a > b ? a : b, lo = a > b ? b : a;
  if (lat == OL_D3Q27) {
    if (a > 1 || b > 1 || cz > 1) return 0;
    *grp = (a != 0) + (b != 0) + (cz != 0);
    return 1;
  }
  if (cz != 0) return 0;
  static const int q9[][2] = {{0, 0}, {1, 0}, {1, 1}};
  static const int q13[][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}};
  static const int q21[][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 2}, {3, 0}};
  static const int q37[][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0},
                               {2, 1}, {2, 2}, {3, 0}, {3, 1}};
  const int(*tab)[2];
  int nt;
  if (lat == OL_D2Q9) { tab = q9; nt = 3; }
  else if (lat == OL_D2Q13) { tab = q13; nt = 4; }
  else if (lat == OL_D2Q21) { tab = q21; nt = 6; }
  else { tab = q37; nt = 8; }
  for (int k = 0; k < nt; ++k)
    if (tab[k][0] == hi && tab[k][1] == lo) { *grp = k; return 1; }
  return 0;
}

/* Solve the nine isotropy conditions of D2Q37 (moments of a Gaussian of
 * variance cs2 up to order eight) for the eight group weights and cs2, by
 * Newton's method in long double, starting from the tabulated values. */
static void solve_d2q37(long double wg[8], long double *cs2) {
  static const double start[9] = {0.233150669132352, 0.107306091542219,
                                  0.057667859888794, 0.014208216158450,
                                  0.005353049000513, 0.001011937592673,
                                  0.000245301027757, 0.000283414252994,
                                  0.697953322019683};
  /* equations: sum_i w_i xi_x^a xi_y^b = coef * c^k */
  static const int ea[9] = {0, 2, 4, 2, 6, 4, 8, 6, 4};
  static const int eb[9] = {0, 0, 0, 2, 0, 2, 0, 2, 4};
  static const int ek[9] = {0, 1, 2, 2, 3, 3, 4, 4, 4};
  static const long double ec[9] = {1, 1, 3, 1, 15, 3, 105, 15, 9};
  long double S[9][8];
  memset(S, 0, sizeof S);
  for (int y = -3; y <= 3; ++y)
    for (int x = -3; x <= 3; ++x) {
      int v[3] = {x, y, 0}, g;
      if (!group_of(OL_D2Q37, v, &g)) continue;
      for (int e = 0; e < 9; ++e) {
        long double t = 1;
        for (int k = 0; k < ea[e]; ++k) t *= x;
        for (int k = 0; k < eb[e]; ++k) t *= y;
        S[e][g] += t;
      }
    }
  long double z[9];
  for (int k = 0; k < 9; ++k) z[k] = start[k];
  for (int it = 0; it < 60; ++it) {
    long double J[9][10];
    for (int e = 0; e < 9; ++e) {
      long double F = 0;
      for (int g = 0; g < 8; ++g) { F += S[e][g] * z[g]; J[e][g] = S[e][g]; }
      long double ck = 1, dck = 0;
      for (int k = 0; k < ek[e]; ++k) ck *= z[8];
      if (ek[e] > 0) {
        dck = ek[e];
        for (int k = 0; k < ek[e] - 1; ++k) dck *= z[8];
      }
      F -= ec[e] * ck;
      J[e][8] = -ec[e] * dck;
      J[e][9] = -F;
    }
    /* Gaussian elimination with partial pivoting */
    for (int col = 0; col < 9; ++col) {
      int piv = col;
      for (int r = col + 1; r < 9; ++r)
        if (fabsl(J[r][col]) > fabsl(J[piv][col])) piv = r;
      for (int k = 0; k < 10; ++k) {
        long double t = J[col][k]; J[col][k] = J[piv][k]; J[piv][k] = t;
      }
      for (int r = col + 1; r < 9; ++r) {
        long double fct = J[r][col] / J[col][col];
        for (int k = col; k < 10; ++k) J[r][k] -= fct * J[col][k];
      }
    }
    long double d[9];
    for (int r = 8; r >= 0; --r) {
      long double acc = J[r][9];
      for (int k = r + 1; k < 9; ++k) acc -= J[r][k] * d[k];
      d[r] = acc / J[r][r];
    }
    long double nd = 0;
    for (int k = 0; k < 9; ++k) { z[k] += d[k]; nd += fabsl(d[k]); }
    if (nd < 1e-30L) break;
  }
  for (int g = 0; g < 8; ++g) wg[g] = z[g];
  *cs2 = z[8];
}

static double h1d(int n, double xi, double cs2) {
  /* one-dimensional factors of the Hermite tensors listed in App. A.2 */
  switch (n) {
  case 0: return 1.0;
  case 1: return xi;
  case 2: return xi * xi - cs2;
  case 3: return (xi * xi - 3.0 * cs2) * xi;
  default: return xi * xi * xi * xi - 6.0 * cs2 * xi * xi + 3.0 * cs2 * cs2;
  }
}

static int cmp_vel(const void *pa, const void *pb) {
  const int *a = (const int *)pa, *b = (const int *)pb;
  int na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
  int nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  if (na != nb) return na < nb ? -1 : 1;
  for (int k = 0; k < 3; ++k)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}

static int setup_lattice(ol_sim *s) {
  int lat = s->p.lattice;
  if (lat < 0 || lat > 4) return fail(s, -1, "unknown lattice %d", lat);
  s->D = (lat == OL_D3Q27) ? 3 : 2;
  int R = (lat == OL_D2Q21 || lat == OL_D2Q37) ? 3 : lat == OL_D2Q13 ? 2 : 1;
  int vel[MAXQ][3], nq = 0;
  for (int z = (s->D == 3 ? -R : 0); z <= (s->D == 3 ? R : 0); ++z)
    for (int y = -R; y <= R; ++y)
      for (int x = -R; x <= R; ++x) {
        int v[3] = {x, y, z}, g;
        if (!group_of(lat, v, &g)) continue;
        vel[nq][0] = x; vel[nq][1] = y; vel[nq][2] = z;
        ++nq;
      }
  qsort(vel, nq, sizeof vel[0], cmp_vel);
  s->Q = nq;
  long double wg37[8], cs37 = 0;
  if (lat == OL_D2Q37) solve_d2q37(wg37, &cs37);
  s->B = 0;
  for (int i = 0; i < nq; ++i) {
    int g;
    for (int k = 0; k < 3; ++k) {
      s->c[i][k] = vel[i][k];
      if (iabs_(vel[i][k]) > s->B) s->B = iabs_(vel[i][k]);
    }
    group_of(lat, vel[i], &g);
    switch (lat) {
    case OL_D2Q9: {
      static const double w9[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
      s->w[i] = w9[g];
      break;
    }
    case OL_D2Q13: {
      static const double w13[4] = {36.0 / 96.0, 8.0 / 96.0, 6.0 / 96.0, 1.0 / 96.0};
      s->w[i] = w13[g];
      break;
    }
    case OL_D2Q21: {
      static const double w21[6] = {91.0 / 324.0, 1.0 / 12.0, 2.0 / 27.0,
                                    7.0 / 360.0, 1.0 / 432.0, 1.0 / 1620.0};
      s->w[i] = w21[g];
      break;
    }
    case OL_D3Q27: {
      static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0,
                                    1.0 / 216.0};
      s->w[i] = w27[g];
      break;
    }
    default: s->w[i] = (double)wg37[g];
    }
  }
  s->cs2 = lat == OL_D2Q9 || lat == OL_D3Q27 ? 1.0 / 3.0
           : lat == OL_D2Q21                  ? 2.0 / 3.0
           : lat == OL_D2Q13                  ? 0.5
                                              : (double)cs37;
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < nq; ++j)
      if (s->c[j][0] == -s->c[i][0] && s->c[j][1] == -s->c[i][1] &&
          s->c[j][2] == -s->c[i][2])
        s->opp[i] = j;
  /* kept Hermite multi-indices (Table lattices_hermite; product basis for
   * D3Q27; full third order for D2Q13 and D2Q21, App. A.2; full fourth
   * order for the D2Q37 thermal equilibrium) */
  s->nm = 0;
  for (int mz = 0; mz <= 4; ++mz)
    for (int my = 0; my <= 4; ++my)
      for (int mx = 0; mx <= 4; ++mx) {
        int keep;
        if (lat == OL_D2Q9) keep = mz == 0 && mx <= 2 && my <= 2;
        else if (lat == OL_D3Q27) keep = mx <= 2 && my <= 2 && mz <= 2;
        else if (lat == OL_D2Q37) keep = mz == 0 && mx + my <= 4;
        else keep = mz == 0 && mx + my <= 3; /* D2Q13, D2Q21 */
        if (!keep) continue;
        s->m[s->nm][0] = mx; s->m[s->nm][1] = my; s->m[s->nm][2] = mz;
        s->nm++;
      }
  for (int i = 0; i < nq; ++i)
    for (int k = 0; k < s->nm; ++k) {
      double h = 1.0;
      for (int d = 0; d < 3; ++d) h *= h1d(s->m[k][d], s->c[i][d], s->cs2);
      s->H[i][k] = h;
    }
  /* moments constrained by the numerical equilibrium (App. A.2):
   * 1, xi_x, xi_y, xi_x^2, xi_x xi_y, xi_y^2, xi_x|xi|^2, xi_y|xi|^2 */
  for (int i = 0; i < nq; ++i) {
    double x = s->c[i][0], y = s->c[i][1], n2 = x * x + y * y;
    double v[NLAM] = {1.0, x, y, x * x, x * y, y * y, x * n2, y * n2};
    memcpy(s->mom[i], v, sizeof v);
  }
  s->Cv = 1.0 / (s->p.gamma - 1.0);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibria (App. A.2)                                                    */
/* ------------------------------------------------------------------------ */

static double factm(const int *m) {
  double f = 1.0;
  for (int d = 0; d < 3; ++d)
    for (int k = 2; k <= m[d]; ++k) f *= k;
  return f;
}

/* isothermal equilibrium Hermite moment, by the recursion
 * a^(n)_{a1..an} = u_{an} a^(n-1)_{a1..a(n-1)}, a^(0) = rho */
static double aeq_iso(const int *m, double rho, const double *u) {
  int k = -1;
  for (int d = 2; d >= 0; --d)
    if (m[d] > 0) { k = d; break; }
  if (k < 0) return rho;
  int mm[3] = {m[0], m[1], m[2]};
  mm[k] -= 1;
  return u[k] * aeq_iso(mm, rho, u);
}

/* raw moments of a 1-D Gaussian of mean u and variance T */
static double gauss_raw(int n, double u, double T) {
  double mu0 = 1.0, mu1 = u;
  if (n == 0) return mu0;
  for (int k = 1; k < n; ++k) {
    double mu2 = u * mu1 + k * T * mu0;
    mu0 = mu1;
    mu1 = mu2;
  }
  return mu1;
}

/* Hermite coefficient of a Maxwellian of temperature T: the expectation of
 * the Hermite tensor (reference cs2) under the Gaussian, factor by factor */
static double aeq_thermal(const int *m, double rho, const double *u, double T,
                          double cs2) {
  double a = rho;
  for (int d = 0; d < 3; ++d) {
    double mu0 = 1.0, mu1 = gauss_raw(1, u[d], T), mu2 = gauss_raw(2, u[d], T);
    double mu3 = gauss_raw(3, u[d], T), mu4 = gauss_raw(4, u[d], T);
    double e;
    switch (m[d]) {
    case 0: e = mu0; break;
    case 1: e = mu1; break;
    case 2: e = mu2 - cs2 * mu0; break;
    case 3: e = mu3 - 3.0 * cs2 * mu1; break;
    default: e = mu4 - 6.0 * cs2 * mu2 + 3.0 * cs2 * cs2 * mu0;
    }
    a *= e;
  }
  return a;
}

/* polynomial equilibrium, Eq. GenEq:
 * f_eq_i = w_i sum_n 1/(n! cs^2n) H^(n)_i : a^(n)_eq, written over symmetric
 * multi-indices m (the Frobenius product counts each of the n!/m! orderings) */
static void feq_poly(const ol_sim *s, double rho, const double *u, double T,
                     int thermal, double *feq) {
  double a[MAXM];
  for (int k = 0; k < s->nm; ++k) {
    a[k] = thermal ? aeq_thermal(s->m[k], rho, u, T, s->cs2)
                   : aeq_iso(s->m[k], rho, u);
    int n = s->m[k][0] + s->m[k][1] + s->m[k][2];
    a[k] /= factm(s->m[k]) * pow(s->cs2, n);
  }
  for (int i = 0; i < s->Q; ++i) {
    double acc = 0.0;
    for (int k = 0; k < s->nm; ++k) acc += s->H[i][k] * a[k];
    feq[i] = s->w[i] * acc;
  }
}

/* ------------------------------------------------------------------------ */
/* Numerical equilibrium (App. A.2, Eqs. exponential / constraints)          */
/* ------------------------------------------------------------------------ */

static void expo_feq(const ol_sim *s, const double *lam, double *feq) {
  for (int i = 0; i < s->Q; ++i) {
    double e = 1.0;
    for (int a = 0; a < NLAM; ++a) e += lam[a] * s->mom[i][a];
    feq[i] = exp(-e);
  }
}

static void constraint_targets(const double *u, double T, double *M) {
  double uu = u[0] * u[0] + u[1] * u[1];
  /* per unit density: 2(E+T) = |u|^2 + (D+2) T with 2E = |u|^2 + D T */
  M[0] = 1.0; M[1] = u[0]; M[2] = u[1];
  M[3] = u[0] * u[0] + T; M[4] = u[0] * u[1]; M[5] = u[1] * u[1] + T;
  M[6] = u[0] * (uu + 4.0 * T); M[7] = u[1] * (uu + 4.0 * T);
}

static void residual(const ol_sim *s, const double *lam, const double *M,
                     double *G, double *feq) {
  expo_feq(s, lam, feq);
  for (int a = 0; a < NLAM; ++a) {
    double acc = 0.0;
    for (int i = 0; i < s->Q; ++i) acc += feq[i] * s->mom[i][a];
    G[a] = acc - M[a];
  }
}

static double norm2(const double *G) {
  double acc = 0.0;
  for (int a = 0; a < NLAM; ++a) acc += G[a] * G[a];
  return sqrt(acc);
}

/* largest |G_a|; a NaN residual propagates, so it never passes the tolerance */
static double normmax(const double *G) {
  double mx = 0.0;
  for (int a = 0; a < NLAM; ++a)
    if (!(fabs(G[a]) <= mx)) mx = fabs(G[a]);
  return mx;
}

/* Newton-Raphson with backtracking line search on the eight constraints,
 * solved per unit density (the multipliers do not depend on rho).
 * Returns the number of iterations, or -1 when not converged. */
static int newton_solve(const ol_sim *s, const double *u, double T,
                        double *lam, double tol, int max_it) {
  double M[NLAM], G[NLAM], feq[MAXQ];
  constraint_targets(u, T, M);
  residual(s, lam, M, G, feq);
  for (int it = 0; it <= max_it; ++it) {
    if (normmax(G) <= tol) return it;
    if (it == max_it) break;
    /* Jacobian of G is -sum_i f_i m_i m_i^T; the step solves
     * (sum_i f_i m_i m_i^T) delta = G */
    double A[NLAM][NLAM + 1];
    for (int a = 0; a < NLAM; ++a) {
      for (int b = 0; b < NLAM; ++b) {
        double acc = 0.0;
        for (int i = 0; i < s->Q; ++i)
          acc += feq[i] * s->mom[i][a] * s->mom[i][b];
        A[a][b] = acc;
      }
      A[a][NLAM] = G[a];
    }
    for (int col = 0; col < NLAM; ++col) {
      int piv = col;
      for (int r = col + 1; r < NLAM; ++r)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      for (int k = 0; k <= NLAM; ++k) {
        double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t;
      }
      for (int r = col + 1; r < NLAM; ++r) {
        double fct = A[r][col] / A[col][col];
        for (int k = col; k <= NLAM; ++k) A[r][k] -= fct * A[col][k];
      }
    }
    double d[NLAM];
    for (int r = NLAM - 1; r >= 0; --r) {
      double acc = A[r][NLAM];
      for (int k = r + 1; k < NLAM; ++k) acc -= A[r][k] * d[k];
      d[r] = acc / A[r][r];
    }
    double n0 = norm2(G), alpha = 1.0, trial[NLAM], Gt[NLAM], ft[MAXQ];
    for (int h = 0; h <= 30; ++h) {
      for (int a = 0; a < NLAM; ++a) trial[a] = lam[a] + alpha * d[a];
      residual(s, trial, M, Gt, ft);
      if (norm2(Gt) < n0 || h == 30) break;
      alpha *= 0.5;
    }
    memcpy(lam, trial, sizeof trial);
    memcpy(G, Gt, sizeof Gt);
    memcpy(feq, ft, sizeof ft);
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Collision at one cell                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  double rho, u[3], T;
} moments_t;

static moments_t cell_moments(const ol_sim *s, const double *f,
                              const double *g) {
  moments_t r = {0.0, {0.0, 0.0, 0.0}, 0.0};
  double j[3] = {0.0, 0.0, 0.0}, e = 0.0;
  for (int i = 0; i < s->Q; ++i) {
    r.rho += f[i];
    for (int d = 0; d < s->D; ++d) j[d] += f[i] * s->c[i][d];
  }
  for (int d = 0; d < s->D; ++d) r.u[d] = j[d] / r.rho;
  if (g) {
    /* Eq. polyTemp */
    double uu = 0.0;
    for (int i = 0; i < s->Q; ++i) {
      double c2 = 0.0;
      for (int d = 0; d < s->D; ++d) c2 += (double)s->c[i][d] * s->c[i][d];
      e += c2 * f[i] + g[i];
    }
    for (int d = 0; d < s->D; ++d) uu += r.u[d] * r.u[d];
    r.T = (e - r.rho * uu) / (2.0 * r.rho * s->Cv);
  }
  return r;
}

static int is_ddf(const ol_sim *s) {
  return s->p.collision == OL_DDF_POLY || s->p.collision == OL_DDF_NEWTON;
}

/* equilibrium f (and g, for DDF) at given macroscopic state */
static int equilibrium(ol_sim *s, double rho, const double *u, double T,
                       double *feq, double *geq, double *lam) {
  if (s->p.collision == OL_DDF_NEWTON) {
    double l0[NLAM];
    if (!s->p.warm_start || !lam) memset(l0, 0, sizeof l0);
    else memcpy(l0, lam, sizeof l0);
    int it = newton_solve(s, u, T, l0, s->p.newton_tol, s->p.newton_max_it);
#pragma omp atomic
    s->newton_calls += 1;
    if (it < 0) return -1;
#pragma omp atomic
    s->newton_it += it;
    if (lam) memcpy(lam, l0, sizeof l0);
    double e[MAXQ];
    expo_feq(s, l0, e);
    for (int i = 0; i < s->Q; ++i) feq[i] = rho * e[i];
  } else {
    feq_poly(s, rho, u, T, s->p.collision == OL_DDF_POLY, feq);
  }
  if (geq) /* Eq. gEq */
    for (int i = 0; i < s->Q; ++i)
      geq[i] = (2.0 * s->Cv - s->D) * T * feq[i];
  return 0;
}

/* kinetic sensor, Eqs. DeltaAvg and shock_function */
static double sensor_alpha(const ol_sim *s, const double *f, const double *feq,
                           double tau, double *eps_out) {
  double eps = 0.0;
  for (int i = 0; i < s->Q; ++i) {
    double den = fabs(feq[i]);
    if (den < 1e-300) den = 1e-300;
    eps += fabs(f[i] - feq[i]) / den;
  }
  eps /= s->Q;
  if (eps_out) *eps_out = eps;
  if (eps < 0.01) return 1.0;
  if (eps < 0.10) return 1.05;
  if (eps < 1.00) return s->p.sensor_A;
  return 1.0 / tau;
}

/* non-equilibrium Hermite moment of a tuple of coordinate indexes, by the
 * recursion a_neq^(n)_{a1..an} = u_an a_neq^(n-1)_{a1..a(n-1)}
 *                 + (1/rho) sum_{i<n} a_eq^(n-2)_{beta_i} a_neq^(2)_{ai an},
 * with a_neq^(0) = a_neq^(1) = 0 and (1/rho) a_eq^(n-2) = product of u. */
static double aneq_tuple(int n, const int *al, const double *u,
                         double a2[3][3]) {
  if (n < 2) return 0.0;
  if (n == 2) return a2[al[0]][al[1]];
  double r = u[al[n - 1]] * aneq_tuple(n - 1, al, u, a2);
  for (int i = 0; i < n - 1; ++i) {
    double pu = 1.0;
    for (int k = 0; k < n - 1; ++k)
      if (k != i) pu *= u[al[k]];
    r += pu * a2[al[i]][al[n - 1]];
  }
  return r;
}

/* collision of one cell; tau_eff may be changed by the sensor */
static int collide_cell(ol_sim *s, double tau, double sigma, double rho_inf,
                        const double *f, const double *g, double *fs,
                        double *gs, double *lam, double *eps_out) {
  moments_t mo = cell_moments(s, f, is_ddf(s) ? g : NULL);
  /* pressure sponge applied before collision, Eq. relaxation_pressure */
  double rho_c = mo.rho * (1.0 - sigma) + sigma * rho_inf;
  double feq[MAXQ], geq[MAXQ];
  int coll = s->p.collision;
  if (coll == OL_BGK) {
    feq_poly(s, rho_c, mo.u, 0.0, 0, feq);
    for (int i = 0; i < s->Q; ++i) fs[i] = f[i] - (f[i] - feq[i]) / tau;
    return 0;
  }
  if (coll == OL_RR) {
    /* Eq. GenRegCollision with a_neq^(2) = sum_i H^(2)_i (f_i - f_i^eq) */
    double fe0[MAXQ];
    feq_poly(s, mo.rho, mo.u, 0.0, 0, fe0);
    double a2[3][3] = {{0}};
    for (int al = 0; al < s->D; ++al)
      for (int be = 0; be < s->D; ++be) {
        double acc = 0.0;
        for (int i = 0; i < s->Q; ++i) {
          double h = s->c[i][al] * s->c[i][be] - (al == be ? s->cs2 : 0.0);
          acc += h * (f[i] - fe0[i]);
        }
        a2[al][be] = acc;
      }
    if (s->p.trace_eq) { /* bulk relaxation time set to one */
      double tr = 0.0;
      for (int al = 0; al < s->D; ++al) tr += a2[al][al];
      for (int al = 0; al < s->D; ++al) a2[al][al] -= tr / s->D;
    }
    double as[MAXM];
    for (int k = 0; k < s->nm; ++k) {
      int tup[12], n = 0;
      for (int d = 0; d < 3; ++d)
        for (int r = 0; r < s->m[k][d]; ++r) tup[n++] = d;
      double ae = aeq_iso(s->m[k], rho_c, mo.u);
      double an = aneq_tuple(n, tup, mo.u, a2);
      as[k] = (ae + (1.0 - 1.0 / tau) * an) / (factm(s->m[k]) * pow(s->cs2, n));
    }
    for (int i = 0; i < s->Q; ++i) {
      double acc = 0.0;
      for (int k = 0; k < s->nm; ++k) acc += s->H[i][k] * as[k];
      fs[i] = s->w[i] * acc;
    }
    return 0;
  }
  /* double distribution (DDF_POLY / DDF_NEWTON) */
  if (equilibrium(s, rho_c, mo.u, mo.T, feq, geq, lam) != 0) return -1;
  double te = tau;
  if (s->p.sensor_on) te = tau * sensor_alpha(s, f, feq, tau, eps_out);
  for (int i = 0; i < s->Q; ++i) {
    fs[i] = f[i] - (f[i] - feq[i]) / te;
    gs[i] = g[i] - (g[i] - geq[i]) / te;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Creation                                                                  */
/* ------------------------------------------------------------------------ */

ol_sim *ol_create(const ol_params *p) {
  ol_sim *s = (ol_sim *)calloc(1, sizeof(ol_sim));
  if (!s) return NULL;
  s->p = *p;
  if (setup_lattice(s) != 0) { free(s); return NULL; }
  int lat = p->lattice, coll = p->collision;
  int ok = (lat != OL_D2Q37 && (coll == OL_BGK || coll == OL_RR)) ||
           (lat == OL_D2Q37 && coll == OL_DDF_POLY) ||
           ((lat == OL_D2Q21 || lat == OL_D2Q13 || lat == OL_D2Q37) && coll == OL_DDF_NEWTON);
  if (!ok) { free(s); return NULL; }
  return s;
}

static void free_grid(ol_sim *s) {
  free(s->xyz); free(s->lev); free(s->flag); free(s->nbr); free(s->ghost);
  free(s->child); free(s->bcsrc); free(s->bcface); free(s->sigma);
  free(s->rho_inf); free(s->wall_du);
  free(s->f); free(s->fs); free(s->g); free(s->gs); free(s->lam);
  free(s->collided);
  s->xyz = NULL; s->lev = NULL; s->flag = NULL; s->nbr = NULL;
  s->ghost = NULL; s->child = NULL; s->bcsrc = NULL; s->bcface = NULL;
  s->sigma = NULL; s->rho_inf = NULL; s->wall_du = NULL; s->f = NULL; s->fs = NULL;
  s->g = NULL; s->gs = NULL; s->lam = NULL; s->collided = NULL;
  s->have_grid = 0; s->have_state = 0;
}

void ol_destroy(ol_sim *s) {
  if (!s) return;
  free_grid(s);
  free(s);
}

const char *ol_error(const ol_sim *s) { return s ? s->err : "null"; }

int ol_lattice(const ol_sim *s, int *D, int *Q, int *B, int *c, double *w,
               double *cs2, int *opp) {
  *D = s->D; *Q = s->Q; *B = s->B; *cs2 = s->cs2;
  for (int i = 0; i < s->Q; ++i) {
    for (int k = 0; k < 3; ++k) c[3 * i + k] = s->c[i][k];
    w[i] = s->w[i];
    opp[i] = s->opp[i];
  }
  return 0;
}

double ol_tau(const ol_sim *s, int level) { return s->tau[level]; }

/* ------------------------------------------------------------------------ */
/* Grid: masks -> level-grouped Morton-ordered cells (Secs. 3.2, 4.3, 4.4)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t key;
  int32_t x, y, z;
} cellkey;

static int cmp_key(const void *a, const void *b) {
  uint64_t ka = ((const cellkey *)a)->key, kb = ((const cellkey *)b)->key;
  return ka < kb ? -1 : ka > kb ? 1 : 0;
}

static uint64_t morton(int D, int32_t x, int32_t y, int32_t z) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b) {
    k |= (uint64_t)((x >> b) & 1) << (D * b);
    k |= (uint64_t)((y >> b) & 1) << (D * b + 1);
    if (D == 3) k |= (uint64_t)((z >> b) & 1) << (D * b + 2);
  }
  return k;
}

typedef struct {
  int32_t E[3];
  int64_t N;
  uint8_t *inR, *strip, *exists, *pre; /* pre: exists before solid removal */
  const uint8_t *refined;              /* next-level mask at this resolution */
  const uint8_t *solid;
  int32_t *idx;
} lvl_t;

static int64_t lin(const lvl_t *v, int32_t x, int32_t y, int32_t z) {
  return (int64_t)x + (int64_t)v->E[0] * ((int64_t)y + (int64_t)v->E[1] * z);
}

static int periodic_axis(const ol_sim *s, int a) {
  return s->face[2 * a].kind == OL_BC_PERIODIC;
}

int ol_grid(ol_sim *s, int dim, const int32_t ext[3], int L,
            const uint8_t *const *refine, const uint8_t *const *solid,
            const ol_face faces[6]) {
  free_grid(s);
  if (dim != s->D) return fail(s, -1, "dimension %d does not match lattice", dim);
  if (L < 1 || L > MAXL) return fail(s, -1, "bad level count %d", L);
  for (int a = 0; a < 3; ++a) {
    int32_t e = a < dim ? ext[a] : 1;
    if (e < 1) return fail(s, -1, "bad extent");
    s->ext[a] = e;
  }
  for (int k = 0; k < 6; ++k) s->face[k] = faces[k];
  for (int a = 0; a < dim; ++a) {
    int p0 = faces[2 * a].kind == OL_BC_PERIODIC, p1 = faces[2 * a + 1].kind == OL_BC_PERIODIC;
    if (p0 != p1) return fail(s, -2, "periodic faces must come in pairs");
  }
  s->dim = dim;
  s->L = L;
  int B = s->B, D = s->D;
  lvl_t lv[MAXL];
  memset(lv, 0, sizeof lv);
  int rc = 0;
  for (int l = 0; l < L; ++l) {
    lv[l].N = 1;
    for (int a = 0; a < 3; ++a) {
      lv[l].E[a] = a < dim ? (s->ext[a] << l) : 1;
      lv[l].N *= lv[l].E[a];
    }
    lv[l].inR = (uint8_t *)calloc(lv[l].N, 1);
    lv[l].strip = (uint8_t *)calloc(lv[l].N, 1);
    lv[l].exists = (uint8_t *)calloc(lv[l].N, 1);
    lv[l].pre = (uint8_t *)calloc(lv[l].N, 1);
    lv[l].idx = (int32_t *)malloc(lv[l].N * sizeof(int32_t));
    lv[l].refined = l < L - 1 ? refine[l] : NULL;
    lv[l].solid = solid ? solid[l] : NULL;
  }
  /* membership of R_l */
  for (int l = 0; l < L; ++l)
    for (int32_t z = 0; z < lv[l].E[2]; ++z)
      for (int32_t y = 0; y < lv[l].E[1]; ++y)
        for (int32_t x = 0; x < lv[l].E[0]; ++x) {
          int64_t id = lin(&lv[l], x, y, z);
          if (l == 0) { lv[l].inR[id] = 1; continue; }
          int32_t pz = dim == 3 ? z / 2 : 0;
          int64_t pid = lin(&lv[l - 1], x / 2, y / 2, pz);
          lv[l].inR[id] = lv[l - 1].refined[pid] && lv[l - 1].inR[pid];
        }
  /* nesting: a refined cell must belong to its own level */
  for (int l = 0; l < L - 1; ++l)
    for (int64_t id = 0; id < lv[l].N; ++id)
      if (lv[l].refined[id] && !lv[l].inR[id]) {
        rc = fail(s, -2, "refine mask %d is not nested in level %d", l + 1, l);
        goto done;
      }
  /* coarse-ghost strips: refined cells within Chebyshev distance B of an
   * unrefined in-domain cell (periodic faces wrap) */
  for (int l = 0; l < L - 1; ++l) {
    lvl_t *v = &lv[l];
    for (int32_t z = 0; z < v->E[2]; ++z)
      for (int32_t y = 0; y < v->E[1]; ++y)
        for (int32_t x = 0; x < v->E[0]; ++x) {
          int64_t id = lin(v, x, y, z);
          if (!v->refined[id]) continue;
          int hit = 0;
          int R2 = dim == 3 ? B : 0;
          for (int dz = -R2; dz <= R2 && !hit; ++dz)
            for (int dy = -B; dy <= B && !hit; ++dy)
              for (int dx = -B; dx <= B && !hit; ++dx) {
                int32_t q[3] = {x + dx, y + dy, z + dz};
                int out = 0;
                for (int a = 0; a < dim; ++a) {
                  if (q[a] < 0 || q[a] >= v->E[a]) {
                    if (periodic_axis(s, a)) q[a] = ((q[a] % v->E[a]) + v->E[a]) % v->E[a];
                    else out = 1;
                  }
                }
                if (out) continue;
                if (!v->refined[lin(v, q[0], q[1], q[2])]) hit = 1;
              }
          v->strip[id] = (uint8_t)hit;
        }
  }
  /* separation of successive interfaces */
  for (int l = 1; l < L - 1; ++l)
    for (int32_t z = 0; z < lv[l].E[2]; ++z)
      for (int32_t y = 0; y < lv[l].E[1]; ++y)
        for (int32_t x = 0; x < lv[l].E[0]; ++x) {
          if (!lv[l].refined[lin(&lv[l], x, y, z)]) continue;
          int32_t pz = dim == 3 ? z / 2 : 0;
          if (lv[l - 1].strip[lin(&lv[l - 1], x / 2, y / 2, pz)]) {
            rc = fail(s, -2, "refinement interfaces %d and %d are too close", l - 1, l);
            goto done;
          }
        }
  /* existence */
  for (int l = 0; l < L; ++l) {
    lvl_t *v = &lv[l];
    for (int64_t id = 0; id < v->N; ++id) {
      int ref = v->refined ? v->refined[id] : 0;
      v->pre[id] = v->inR[id] && (!ref || v->strip[id]);
      v->exists[id] = v->pre[id] && !(v->solid && v->solid[id]);
    }
  }
  /* solid cells on interfaces */
  for (int l = 0; l < L - 1; ++l) {
    lvl_t *v = &lv[l];
    for (int32_t z = 0; z < v->E[2]; ++z)
      for (int32_t y = 0; y < v->E[1]; ++y)
        for (int32_t x = 0; x < v->E[0]; ++x) {
          int64_t id = lin(v, x, y, z);
          if (!v->strip[id]) continue;
          int nf = 0, nc = 0;
          for (int o = 0; o < (1 << D); ++o) {
            int32_t cx = 2 * x + (o & 1), cy = 2 * y + ((o >> 1) & 1);
            int32_t cz = D == 3 ? 2 * z + ((o >> 2) & 1) : 0;
            nc++;
            if (lv[l + 1].exists[lin(&lv[l + 1], cx, cy, cz)]) nf++;
          }
          if (v->exists[id] ? nf == 0 : nf != 0) {
            rc = fail(s, -2, "solid body cuts a refinement interface badly");
            goto done;
          }
          (void)nc;
        }
  }
  /* ordering: level-major, Morton within level */
  s->n = 0;
  for (int l = 0; l < L; ++l) {
    int64_t cnt = 0;
    for (int64_t id = 0; id < lv[l].N; ++id) cnt += lv[l].exists[id];
    s->off[l] = s->n;
    s->n += cnt;
  }
  s->off[L] = s->n;
  int64_t n = s->n;
  int Qm = s->Q - 1;
  s->xyz = (int32_t *)malloc(n * 3 * sizeof(int32_t));
  s->lev = (int8_t *)malloc(n);
  s->flag = (uint8_t *)calloc(n, 1);
  s->nbr = (int32_t *)malloc(n * Qm * sizeof(int32_t));
  s->bcsrc = (int32_t *)malloc(n * sizeof(int32_t));
  s->bcface = (int8_t *)malloc(n);
  s->sigma = (double *)calloc(n, sizeof(double));
  s->rho_inf = (double *)calloc(n, sizeof(double));
  for (int l = 0; l < L; ++l) {
    lvl_t *v = &lv[l];
    int64_t cnt = s->off[l + 1] - s->off[l], k = 0;
    cellkey *ck = (cellkey *)malloc((cnt > 0 ? cnt : 1) * sizeof(cellkey));
    for (int32_t z = 0; z < v->E[2]; ++z)
      for (int32_t y = 0; y < v->E[1]; ++y)
        for (int32_t x = 0; x < v->E[0]; ++x)
          if (v->exists[lin(v, x, y, z)]) {
            ck[k].key = morton(D, x, y, z);
            ck[k].x = x; ck[k].y = y; ck[k].z = z;
            ++k;
          }
    qsort(ck, cnt, sizeof(cellkey), cmp_key);
    for (int64_t id = 0; id < v->N; ++id) v->idx[id] = -1;
    for (k = 0; k < cnt; ++k) {
      int64_t c = s->off[l] + k;
      s->xyz[3 * c] = ck[k].x; s->xyz[3 * c + 1] = ck[k].y; s->xyz[3 * c + 2] = ck[k].z;
      s->lev[c] = (int8_t)l;
      v->idx[lin(v, ck[k].x, ck[k].y, ck[k].z)] = (int32_t)c;
    }
    free(ck);
  }
  /* flags */
  for (int64_t c = 0; c < n; ++c) {
    int l = s->lev[c];
    int32_t x = s->xyz[3 * c], y = s->xyz[3 * c + 1], z = s->xyz[3 * c + 2];
    if (l < L - 1 && lv[l].strip[lin(&lv[l], x, y, z)]) s->flag[c] |= OL_F_COARSE_GHOST;
    if (l > 0 && lv[l - 1].strip[lin(&lv[l - 1], x / 2, y / 2, D == 3 ? z / 2 : 0)])
      s->flag[c] |= OL_F_FINE_GHOST;
    if ((s->flag[c] & 3) == 3) {
      rc = fail(s, -2, "cell is both coarse and fine ghost");
      goto done;
    }
  }
  /* neighbour list: pull source x - xi_i at the same level */
  for (int64_t c = 0; c < n; ++c) {
    int l = s->lev[c];
    lvl_t *v = &lv[l];
    for (int i = 1; i < s->Q; ++i) {
      int32_t q[3];
      int outface[3], nout = 0;
      for (int a = 0; a < 3; ++a) {
        q[a] = s->xyz[3 * c + a] - s->c[i][a];
        if (a >= dim) continue;
        if (q[a] < 0 || q[a] >= v->E[a]) {
          if (periodic_axis(s, a)) q[a] = ((q[a] % v->E[a]) + v->E[a]) % v->E[a];
          else outface[nout++] = 2 * a + (q[a] >= v->E[a]);
        }
      }
      int32_t val;
      if (nout > 0) {
        int any_wall = 0, mov = -1;
        for (int k = 0; k < nout; ++k) {
          int kind = s->face[outface[k]].kind;
          if (kind == OL_BC_WALL) any_wall = 1;
          if (kind == OL_BC_MOVING_WALL && mov < 0) mov = outface[k];
        }
        if (any_wall) val = OL_SOLID;
        else if (mov >= 0) val = -3 - mov;
        else val = OL_NONE;
      } else {
        int64_t id = lin(v, q[0], q[1], q[2]);
        if (v->exists[id]) val = v->idx[id];
        else if (v->pre[id]) val = OL_SOLID;
        else val = OL_NONE;
      }
      s->nbr[c * Qm + i - 1] = val;
    }
  }
  /* boundary-condition layers, B cells deep on Neumann / equilibrium faces */
  for (int64_t c = 0; c < n; ++c) {
    int l = s->lev[c];
    int32_t src[3] = {s->xyz[3 * c], s->xyz[3 * c + 1], s->xyz[3 * c + 2]};
    int eqf = -1, nef = -1;
    for (int fc = 0; fc < 2 * dim; ++fc) {
      int kind = s->face[fc].kind, a = fc / 2;
      if (kind != OL_BC_NEUMANN && kind != OL_BC_EQUILIBRIUM) continue;
      int32_t E = lv[l].E[a], x = s->xyz[3 * c + a];
      int in = (fc & 1) ? x >= E - B : x < B;
      if (!in) continue;
      src[a] = (fc & 1) ? E - 1 - B : B;
      if (kind == OL_BC_EQUILIBRIUM && eqf < 0) eqf = fc;
      if (kind == OL_BC_NEUMANN && nef < 0) nef = fc;
    }
    s->bcsrc[c] = -1;
    s->bcface[c] = -1;
    if (eqf < 0 && nef < 0) continue;
    if (s->flag[c] & 3) { rc = fail(s, -2, "boundary layer overlaps a refinement interface"); goto done; }
    int32_t sid = -1;
    int inside = 1;
    for (int a = 0; a < dim; ++a)
      if (src[a] < 0 || src[a] >= lv[l].E[a]) inside = 0;
    if (inside) sid = lv[l].idx[lin(&lv[l], src[0], src[1], src[2])];
    if (sid < 0) { rc = fail(s, -2, "boundary cell has no fluid source"); goto done; }
    s->bcsrc[c] = sid;
    s->bcface[c] = (int8_t)(eqf >= 0 ? eqf : nef);
    s->flag[c] |= eqf >= 0 ? OL_F_BC_EQ : OL_F_BC_NEUMANN;
  }
  for (int64_t c = 0; c < n; ++c) {
    int32_t sid = s->bcsrc[c];
    if (sid >= 0 && (s->flag[sid] & (OL_F_BC_EQ | OL_F_BC_NEUMANN))) {
      rc = fail(s, -2, "boundary source lies in a boundary layer");
      goto done;
    }
  }
  /* every non-ghost, non-boundary cell needs a source for each population */
  for (int64_t c = 0; c < n; ++c) {
    if (s->flag[c] & (OL_F_COARSE_GHOST | OL_F_FINE_GHOST | OL_F_BC_EQ | OL_F_BC_NEUMANN)) continue;
    for (int i = 1; i < s->Q; ++i)
      if (s->nbr[c * Qm + i - 1] == OL_NONE) {
        rc = fail(s, -2, "bulk cell without a streaming source");
        goto done;
      }
  }
  /* pressure sponge strength (rectangular stand-in of the radial ramp) */
  for (int64_t c = 0; c < n; ++c) {
    int l = s->lev[c];
    double best = 0.0, rinf = 1.0;
    for (int fc = 0; fc < 2 * dim; ++fc) {
      const ol_face *F = &s->face[fc];
      if (F->kind == OL_BC_PERIODIC || F->sponge_sigma_max <= 0.0 || F->sponge_width <= 0.0) continue;
      int a = fc / 2;
      double ctr = (s->xyz[3 * c + a] + 0.5) / (double)(1 << l);
      double d = (fc & 1) ? s->ext[a] - ctr : ctr;
      double r = 1.0 - d / F->sponge_width;
      if (r < 0.0) r = 0.0;
      if (r > 1.0) r = 1.0;
      double sg = F->sponge_sigma_max * r;
      if (sg > best) { best = sg; rinf = F->rho; }
    }
    s->sigma[c] = best;
    s->rho_inf[c] = rinf;
    if (best > 0.0) s->flag[c] |= OL_F_SPONGE;
  }
  /* coarse-ghost list and child table */
  s->ng = 0;
  for (int64_t c = 0; c < n; ++c) s->ng += (s->flag[c] & OL_F_COARSE_GHOST) != 0;
  s->ghost = (int32_t *)malloc((s->ng > 0 ? s->ng : 1) * sizeof(int32_t));
  s->child = (int32_t *)malloc((s->ng > 0 ? s->ng : 1) * (1 << D) * sizeof(int32_t));
  {
    int64_t k = 0;
    for (int l = 0; l < L; ++l) {
      s->goff[l] = k;
      for (int64_t c = s->off[l]; c < s->off[l + 1]; ++c) {
        if (!(s->flag[c] & OL_F_COARSE_GHOST)) continue;
        s->ghost[k] = (int32_t)c;
        for (int o = 0; o < (1 << D); ++o) {
          int32_t cx = 2 * s->xyz[3 * c] + (o & 1), cy = 2 * s->xyz[3 * c + 1] + ((o >> 1) & 1);
          int32_t cz = D == 3 ? 2 * s->xyz[3 * c + 2] + ((o >> 2) & 1) : 0;
          s->child[k * (1 << D) + o] = lv[l + 1].idx[lin(&lv[l + 1], cx, cy, cz)];
        }
        ++k;
      }
    }
    s->goff[L] = k;
  }
  /* relaxation times per level, Eq. tau_fine_to_coarse applied recursively */
  {
    double cs2e = is_ddf(s) ? s->p.T0 : s->cs2;
    for (int l = 0; l < L; ++l) {
      if (s->p.nu_finest <= 0.0) s->tau[l] = 0.5;
      else s->tau[l] = s->p.nu_finest / (double)(1 << (L - 1 - l)) / cs2e + 0.5;
    }
  }
  s->have_grid = 1;
done:
  for (int l = 0; l < L; ++l) {
    free(lv[l].inR); free(lv[l].strip); free(lv[l].exists); free(lv[l].pre);
    free(lv[l].idx);
  }
  if (rc != 0) free_grid(s);
  return rc;
}

int64_t ol_n_cells(const ol_sim *s) { return s->have_grid ? s->n : -1; }
int64_t ol_n_ghosts(const ol_sim *s) { return s->have_grid ? s->ng : -1; }

int ol_level_counts(const ol_sim *s, int64_t *npl) {
  if (!s->have_grid) return -5;
  for (int l = 0; l < s->L; ++l) npl[l] = s->off[l + 1] - s->off[l];
  return 0;
}

int ol_export(const ol_sim *s, int32_t *coords, int8_t *level, uint8_t *flags,
              int32_t *nbr, int32_t *child, int32_t *bc_src) {
  if (!s->have_grid) return -5;
  int64_t n = s->n;
  if (coords) memcpy(coords, s->xyz, n * 3 * sizeof(int32_t));
  if (level) memcpy(level, s->lev, n);
  if (flags) memcpy(flags, s->flag, n);
  if (nbr) memcpy(nbr, s->nbr, n * (s->Q - 1) * sizeof(int32_t));
  if (child) memcpy(child, s->child, s->ng * (1 << s->D) * sizeof(int32_t));
  if (bc_src) memcpy(bc_src, s->bcsrc, n * sizeof(int32_t));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Initialisation (App. A.3: populations start at equilibrium)               */
/* ------------------------------------------------------------------------ */

int ol_init(ol_sim *s, const double *mom) {
  if (!s->have_grid) return fail(s, -5, "no grid");
  int64_t n = s->n;
  int Q = s->Q, D = s->D, ddf = is_ddf(s);
  free(s->f); free(s->fs); free(s->g); free(s->gs); free(s->lam); free(s->collided);
  s->f = (double *)calloc(n * Q, sizeof(double));
  s->fs = (double *)calloc(n * Q, sizeof(double));
  s->g = ddf ? (double *)calloc(n * Q, sizeof(double)) : NULL;
  s->gs = ddf ? (double *)calloc(n * Q, sizeof(double)) : NULL;
  s->lam = (double *)calloc(n * NLAM, sizeof(double));
  s->collided = (uint8_t *)calloc(n, 1);
  int bad = 0;
  int save_warm = s->p.warm_start;
  s->p.warm_start = 0; /* cold start from lambda = 0 */
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = 0; c < n; ++c) {
    double rho = mom[c], u[3] = {0.0, 0.0, 0.0}, T = 0.0;
    for (int d = 0; d < D; ++d) u[d] = mom[(1 + d) * n + c];
    if (ddf) T = mom[(1 + D) * n + c];
    if (equilibrium(s, rho, u, T, s->f + c * Q, ddf ? s->g + c * Q : NULL,
                    s->lam + c * NLAM) != 0)
      bad = 1;
  }
  s->p.warm_start = save_warm;
  memset(s->upd, 0, sizeof s->upd);
  s->newton_it = 0;
  s->newton_calls = 0;
  s->numeric_error = 0;
  if (bad) return fail(s, -6, "Newton did not converge at initialisation");
  s->have_state = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Time stepping                                                             */
/* ------------------------------------------------------------------------ */

/* population i of coarse ghost G is coalesced from the children unless the
 * coarse level itself supplies it: its pull source at G's level is a cell
 * outside the refined region (a boundary sentinel counts as supplied); a
 * source that is missing or is another coarse ghost lies in the overlap,
 * where the fine level carries the flow */
static int coalesced_pop(const ol_sim *s, int64_t G, int i) {
  int32_t v = s->nbr[G * (s->Q - 1) + i - 1];
  if (v == OL_NONE) return 1;
  return v >= 0 && (s->flag[v] & OL_F_COARSE_GHOST);
}

/* Rohde coupling between level l (coarse) and l+1 (fine): coalescence of the
 * unknown coarse-ghost populations, collision of the coarse ghost, uniform
 * explosion of its post-collision state into all of its children. */
static void coupling(ol_sim *s, int l) {
  int Q = s->Q, Qm = Q - 1, nch = 1 << s->D, ddf = is_ddf(s);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t k = s->goff[l]; k < s->goff[l + 1]; ++k) {
    int64_t G = s->ghost[k];
    const int32_t *ch = s->child + k * nch;
    int nf = 0;
    for (int o = 0; o < nch; ++o) nf += ch[o] >= 0;
    for (int i = 1; i < Q; ++i) {
      if (!coalesced_pop(s, G, i)) continue;
      double af = 0.0, ag = 0.0;
      for (int o = 0; o < nch; ++o) {
        if (ch[o] < 0) continue;
        af += s->f[(int64_t)ch[o] * Q + i];
        if (ddf) ag += s->g[(int64_t)ch[o] * Q + i];
      }
      s->f[G * Q + i] = af / nf;
      if (ddf) s->g[G * Q + i] = ag / nf;
    }
    if (s->p.collision == OL_DDF_NEWTON) {
      for (int a = 0; a < NLAM; ++a) {
        double al = 0.0;
        for (int o = 0; o < nch; ++o)
          if (ch[o] >= 0) al += s->lam[(int64_t)ch[o] * NLAM + a];
        s->lam[G * NLAM + a] = al / nf;
      }
    }
    if (collide_cell(s, s->tau[l], s->sigma[G], s->rho_inf[G], s->f + G * Q,
                     ddf ? s->g + G * Q : NULL, s->fs + G * Q,
                     ddf ? s->gs + G * Q : NULL, s->lam + G * NLAM, NULL) != 0)
      bad = 1;
    s->collided[G] = 1;
    for (int o = 0; o < nch; ++o) {
      if (ch[o] < 0) continue;
      int64_t K = ch[o];
      memcpy(s->f + K * Q, s->fs + G * Q, Q * sizeof(double));
      if (ddf) memcpy(s->g + K * Q, s->gs + G * Q, Q * sizeof(double));
      memcpy(s->lam + K * NLAM, s->lam + G * NLAM, NLAM * sizeof(double));
    }
  }
  if (bad) s->numeric_error = 1;
}

static void boundary_fill(ol_sim *s, int l) {
  int Q = s->Q, ddf = is_ddf(s);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = s->off[l]; c < s->off[l + 1]; ++c) {
    if (!(s->flag[c] & (OL_F_BC_EQ | OL_F_BC_NEUMANN))) continue;
    int64_t src = s->bcsrc[c];
    if (s->flag[c] & OL_F_BC_NEUMANN) {
      /* copy all populations of the nearest fluid cell */
      memcpy(s->fs + c * Q, s->fs + src * Q, Q * sizeof(double));
      if (ddf) memcpy(s->gs + c * Q, s->gs + src * Q, Q * sizeof(double));
      memcpy(s->lam + c * NLAM, s->lam + src * NLAM, NLAM * sizeof(double));
    } else {
      const ol_face *F = &s->face[(int)s->bcface[c]];
      double rho = F->rho;
      if (F->extrapolate_rho) {
        rho = 0.0;
        for (int i = 0; i < Q; ++i) rho += s->fs[src * Q + i];
      }
      double u[3] = {F->u[0], F->u[1], F->u[2]};
      if (equilibrium(s, rho, u, F->T, s->fs + c * Q, ddf ? s->gs + c * Q : NULL,
                      s->lam + c * NLAM) != 0)
        bad = 1;
    }
  }
  if (bad) s->numeric_error = 1;
}

static void collide_and_stream(ol_sim *s, int l) {
  int Q = s->Q, Qm = Q - 1, ddf = is_ddf(s);
  int bad = 0;
  const double cs2w = ddf ? s->p.T0 : s->cs2;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = s->off[l]; c < s->off[l + 1]; ++c) {
    uint8_t fl = s->flag[c];
    if (fl & (OL_F_FINE_GHOST | OL_F_BC_EQ | OL_F_BC_NEUMANN)) {
      /* fine ghosts never collide; boundary cells are refilled below */
      memcpy(s->fs + c * Q, s->f + c * Q, Q * sizeof(double));
      if (ddf) memcpy(s->gs + c * Q, s->g + c * Q, Q * sizeof(double));
    } else if (fl & OL_F_COARSE_GHOST) {
      /* already collided during the coupling step of this substep */
      s->collided[c] = 0;
    } else {
      if (collide_cell(s, s->tau[l], s->sigma[c], s->rho_inf[c], s->f + c * Q,
                       ddf ? s->g + c * Q : NULL, s->fs + c * Q,
                       ddf ? s->gs + c * Q : NULL, s->lam + c * NLAM, NULL) != 0)
        bad = 1;
    }
  }
  if (bad) s->numeric_error = 1;
  boundary_fill(s, l);
  /* pull streaming from the post-collision populations */
#pragma omp parallel for schedule(static)
  for (int64_t c = s->off[l]; c < s->off[l + 1]; ++c) {
    s->f[c * Q] = s->fs[c * Q];
    if (ddf) s->g[c * Q] = s->gs[c * Q];
    for (int i = 1; i < Q; ++i) {
      int32_t v = s->nbr[c * Qm + i - 1];
      double fv, gv = 0.0;
      if (v >= 0) {
        fv = s->fs[(int64_t)v * Q + i];
        if (ddf) gv = s->gs[(int64_t)v * Q + i];
      } else if (v == OL_NONE) {
        fv = s->fs[c * Q + i];
        if (ddf) gv = s->gs[c * Q + i];
      } else {
        int io = s->opp[i];
        fv = s->fs[c * Q + io];
        if (ddf) gv = s->gs[c * Q + io];
        if (v <= -3) { /* Ladd's moving wall, wall density 1; the wall
                          velocity seen by this cell carries its inflow noise */
          const ol_face *F = &s->face[-3 - v];
          double cu = 0.0;
          for (int d = 0; d < s->D; ++d)
            cu += s->c[i][d] * (F->u[d] + (s->wall_du ? s->wall_du[3 * c + d] : 0.0));
          fv += 2.0 * s->w[i] * cu / cs2w;
        }
      }
      s->f[c * Q + i] = fv;
      if (ddf) s->g[c * Q + i] = gv;
    }
  }
  s->upd[l] += s->off[l + 1] - s->off[l];
}

int ol_step(ol_sim *s, int64_t nsteps) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  int L = s->L;
  for (int64_t st = 0; st < nsteps; ++st) {
    for (int t = 0; t < (1 << (L - 1)); ++t)
      for (int l = 0; l < L; ++l) {
        if (t % (1 << (L - 1 - l)) != 0) continue;
        if (l < L - 1) coupling(s, l);
        collide_and_stream(s, l);
      }
  }
  if (s->numeric_error) return fail(s, -6, "numerical failure (Newton did not converge)");
  return 0;
}

int ol_set_face(ol_sim *s, int face, const ol_face *f) {
  if (face < 0 || face > 5) return fail(s, -1, "bad face");
  if (f->kind != s->face[face].kind) return fail(s, -1, "face kind cannot change");
  s->face[face] = *f;
  return 0;
}

/* state at the synchronisation point: pre-collision populations with the
 * unknown coarse-ghost populations coalesced from the children */
static void sync_state(const ol_sim *s, double *f, double *g) {
  int Q = s->Q, Qm = Q - 1, nch = 1 << s->D, ddf = is_ddf(s);
  memcpy(f, s->f, s->n * Q * sizeof(double));
  if (ddf) memcpy(g, s->g, s->n * Q * sizeof(double));
  for (int64_t k = 0; k < s->ng; ++k) {
    int64_t G = s->ghost[k];
    const int32_t *ch = s->child + k * nch;
    int nf = 0;
    for (int o = 0; o < nch; ++o) nf += ch[o] >= 0;
    for (int i = 1; i < Q; ++i) {
      if (!coalesced_pop(s, G, i)) continue;
      double af = 0.0, ag = 0.0;
      for (int o = 0; o < nch; ++o) {
        if (ch[o] < 0) continue;
        af += s->f[(int64_t)ch[o] * Q + i];
        if (ddf) ag += s->g[(int64_t)ch[o] * Q + i];
      }
      f[G * Q + i] = af / nf;
      if (ddf) g[G * Q + i] = ag / nf;
    }
  }
}

int ol_moments(ol_sim *s, double *out) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  int Q = s->Q, D = s->D, ddf = is_ddf(s);
  int64_t n = s->n;
  double *f = (double *)malloc(n * Q * sizeof(double));
  double *g = ddf ? (double *)malloc(n * Q * sizeof(double)) : NULL;
  sync_state(s, f, g);
  for (int64_t c = 0; c < n; ++c) {
    if (s->flag[c] & OL_F_FINE_GHOST) {
      for (int k = 0; k < 1 + D + ddf; ++k) out[k * n + c] = NAN;
      continue;
    }
    moments_t mo = cell_moments(s, f + c * Q, ddf ? g + c * Q : NULL);
    out[c] = mo.rho;
    for (int d = 0; d < D; ++d) out[(1 + d) * n + c] = mo.u[d];
    if (ddf) out[(1 + D) * n + c] = mo.T;
  }
  free(f);
  free(g);
  return 0;
}

/* conserved sums over the O9 state: fine ghosts excluded, cells weighted by
 * their volume 2^(-D l) */
/* compensated (Neumaier) summation: the sums below run over ~1e6 terms
 * whose partial sums are thousands of times larger than the terms, where a
 * plain running sum drifts by ~1e-12 of the result; the compensated sum
 * stays within a few ulps of the exact one */
typedef struct {
  double s, c;
} ksum;

static void ksum_add(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}

static double ksum_get(const ksum *k) { return k->s + k->c; }

int ol_sums(ol_sim *s, double *out) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  int Q = s->Q, D = s->D, ddf = is_ddf(s);
  int64_t n = s->n;
  double *f = (double *)malloc(n * Q * sizeof(double));
  double *g = ddf ? (double *)malloc(n * Q * sizeof(double)) : NULL;
  sync_state(s, f, g);
  ksum M = {0.0, 0.0}, P[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}}, E = {0.0, 0.0};
  for (int64_t c = 0; c < n; ++c) {
    if (s->flag[c] & OL_F_FINE_GHOST) continue;
    double vol = ldexp(1.0, -D * s->lev[c]);
    for (int i = 0; i < Q; ++i) {
      double fi = f[c * Q + i], c2 = 0.0;
      ksum_add(&M, vol * fi);
      for (int d = 0; d < D; ++d) {
        ksum_add(&P[d], vol * fi * s->c[i][d]);
        c2 += (double)s->c[i][d] * s->c[i][d];
      }
      ksum_add(&E, vol * 0.5 * (c2 * fi + (ddf ? g[c * Q + i] : 0.0)));
    }
  }
  out[0] = ksum_get(&M);
  for (int d = 0; d < D; ++d) out[1 + d] = ksum_get(&P[d]);
  out[1 + D] = ksum_get(&E);
  free(f);
  free(g);
  return 0;
}

/* kinetic energy of the synchronisation-point state (the monitor of the
 * paper's convergence test, Sec. 5.2): sum over the cells that are not fine
 * ghosts of 2^(-D l) rho |u|^2 / 2, with rho and u the moments of the cell */
int ol_kinetic_energy(ol_sim *s, double *out) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  int Q = s->Q, D = s->D, ddf = is_ddf(s);
  int64_t n = s->n;
  double *f = (double *)malloc(n * Q * sizeof(double));
  double *g = ddf ? (double *)malloc(n * Q * sizeof(double)) : NULL;
  sync_state(s, f, g);
  ksum K = {0.0, 0.0};
  for (int64_t c = 0; c < n; ++c) {
    if (s->flag[c] & OL_F_FINE_GHOST) continue;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
      rho += f[c * Q + i];
      for (int d = 0; d < D; ++d) j[d] += f[c * Q + i] * s->c[i][d];
    }
    double j2 = 0.0;
    for (int d = 0; d < D; ++d) j2 += j[d] * j[d];
    ksum_add(&K, ldexp(1.0, -D * s->lev[c]) * 0.5 * j2 / rho);
  }
  *out = ksum_get(&K);
  free(f);
  free(g);
  return 0;
}

int ol_set_inflow_noise(ol_sim *s, const double *du) {
  if (!s->have_grid) return fail(s, -5, "no grid");
  free(s->wall_du);
  s->wall_du = NULL;
  if (!du) return 0;
  s->wall_du = (double *)malloc(s->n * 3 * sizeof(double));
  if (!s->wall_du) return fail(s, -3, "out of memory");
  for (int64_t c = 0; c < s->n; ++c)
    for (int d = 0; d < 3; ++d) s->wall_du[3 * c + d] = du[d * s->n + c];
  return 0;
}

int ol_counters(const ol_sim *s, int64_t *upd, int64_t *nit, int64_t *ncalls) {
  if (upd)
    for (int l = 0; l < s->L; ++l) upd[l] = s->upd[l];
  if (nit) *nit = s->newton_it;
  if (ncalls) *ncalls = s->newton_calls;
  return 0;
}

int ol_get_state(const ol_sim *s, double *f, double *g, double *lam) {
  if (!s->have_state) return -5;
  if (f) memcpy(f, s->f, s->n * s->Q * sizeof(double));
  if (g && s->g) memcpy(g, s->g, s->n * s->Q * sizeof(double));
  if (lam) memcpy(lam, s->lam, s->n * NLAM * sizeof(double));
  return 0;
}

int ol_get_sync_state(ol_sim *s, double *f, double *g, double *lam) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  if (!f || (is_ddf(s) && !g)) return fail(s, -1, "null output");
  sync_state(s, f, is_ddf(s) ? g : NULL);
  if (lam) memcpy(lam, s->lam, s->n * NLAM * sizeof(double));
  return 0;
}

int ol_sensor(ol_sim *s, double *eps) {
  if (!s->have_state) return fail(s, -5, "not initialised");
  int Q = s->Q, ddf = is_ddf(s);
  int64_t n = s->n;
  double *f = (double *)malloc(n * Q * sizeof(double));
  double *g = ddf ? (double *)malloc(n * Q * sizeof(double)) : NULL;
  sync_state(s, f, g);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = 0; c < n; ++c) {
    if (s->flag[c] & OL_F_FINE_GHOST) {
      eps[c] = NAN;
      continue;
    }
    moments_t mo = cell_moments(s, f + c * Q, ddf ? g + c * Q : NULL);
    double feq[MAXQ], geq[MAXQ], lam[NLAM];
    memcpy(lam, s->lam + c * NLAM, sizeof lam);
    if (equilibrium(s, mo.rho, mo.u, mo.T, feq, ddf ? geq : NULL, lam) != 0) bad = 1;
    sensor_alpha(s, f + c * Q, feq, 1.0, &eps[c]);
  }
  free(f);
  free(g);
  if (bad) return fail(s, -6, "Newton did not converge in the sensor");
  return 0;
}

int ol_set_state(ol_sim *s, const double *f, const double *g, const double *lam) {
  if (!s->have_grid) return fail(s, -5, "no grid");
  if (!f || (is_ddf(s) && !g)) return fail(s, -1, "null populations");
  int64_t n = s->n;
  int Q = s->Q, ddf = is_ddf(s);
  free(s->f); free(s->fs); free(s->g); free(s->gs); free(s->lam); free(s->collided);
  s->f = (double *)malloc(n * Q * sizeof(double));
  s->fs = (double *)calloc(n * Q, sizeof(double));
  s->g = ddf ? (double *)malloc(n * Q * sizeof(double)) : NULL;
  s->gs = ddf ? (double *)calloc(n * Q, sizeof(double)) : NULL;
  s->lam = (double *)calloc(n * NLAM, sizeof(double));
  s->collided = (uint8_t *)calloc(n, 1);
  memcpy(s->f, f, n * Q * sizeof(double));
  if (ddf) memcpy(s->g, g, n * Q * sizeof(double));
  if (lam) memcpy(s->lam, lam, n * NLAM * sizeof(double));
  s->numeric_error = 0;
  s->have_state = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-cell entry points used by the tests                                */
/* ------------------------------------------------------------------------ */

int ol_feq(ol_sim *s, double rho, const double *u, double T, double *feq,
           double *geq, double *lam) {
  double l0[NLAM] = {0};
  if (lam) memcpy(l0, lam, sizeof l0);
  int r = equilibrium(s, rho, u, T, feq, is_ddf(s) ? geq : NULL, l0);
  if (lam) memcpy(lam, l0, sizeof l0);
  return r;
}

int ol_collide(ol_sim *s, double tau, const double *f, const double *g,
               double *fs, double *gs, double *lam, double *eps_out) {
  double l0[NLAM] = {0};
  if (lam) memcpy(l0, lam, sizeof l0);
  int r = collide_cell(s, tau, 0.0, 1.0, f, g, fs, gs, l0, eps_out);
  if (lam) memcpy(lam, l0, sizeof l0);
  return r;
}

int ol_newton(ol_sim *s, const double *u, double T, double *lam, double tol,
              int max_it) {
  return newton_solve(s, u, T, lam, tol, max_it);
}
