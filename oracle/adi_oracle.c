/*
 * adi_oracle.c -- plain CPU FP64 reference ("oracle") for the axisymmetric ADI
 * heat solver of Ayriyan & Busa, "Parallel Algorithm for Numerical Solution of
 * Heat Equation in Complex Cylindrical Domain" (arXiv 1912.03744).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Everything is double precision, written as plain loops in the order of the
 * paper's definitions and meant to be compiled with -O2 -ffp-contract=off.
 * The reference path (or_step) is single-threaded; or_step_omp runs the same
 * line solves on several cores, the paper's parallelisation, for timing.  It is slow on purpose: every cell carries its own
 * operator coefficients, assembled straight from the finite-volume form, and
 * every line is solved by the Thomas algorithm without pivoting (Sec. 3, the
 * closing sentence on the solution of the line systems).
 *
 * Model (Sec. 2, eq. 1, in its linear, piecewise-constant special case):
 *   C dT/dt = (1/r) d/dr (r k dT/dr) + d/dz (k dT/dz) + Q,   C = rho c_V,
 * on the L-shaped assembly of Fig. 1: cooler (region 0) r < r0 for z < zmax;
 * insulator (1) r0 <= r < r1, heater (2) r1 <= r < r2, outer insulator (3)
 * r2 <= r < rmax, all for z < z0; terminal slab (4) zmax <= z < ztop over the
 * whole radius.  Cells with r >= r0 and z0 <= z < zmax lie outside the domain
 * ("masked", id 255).
 *
 * Readings taken where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *  - Grid (eq. 7, Fig. 3): cell-centred; uniform grids use the exact
 *    expressions r_face[i] = rmax*i/nr and r_c[i] = (i+0.5)*rmax/nr (same in
 *    z with ztop), so that any other implementation can reproduce the region
 *    map bit for bit.  Optional face arrays give non-uniform grids; centres are
 *    then face midpoints.
 *  - Regions: the material of a cell is that of its centre, first rule wins:
 *    z_c >= zmax -> 4; r_c < r0 -> 0; z_c >= z0 -> masked; r_c < r1 -> 1;
 *    r_c < r2 -> 2; else 3.
 *  - Operators (eq. 10-11) in balance (finite-volume) form; identical to the
 *    printed formulas on uniform grids.  The conductivity on a face between
 *    two cells is the harmonic (series) value 1/(d_a/(2k_a) + d_b/(2k_b)),
 *    the paper's half-node conductivity text being garbled.
 *  - Boundary conditions (eq. 6) generalised to one Robin family per face
 *    class: class 0 = bottom face z = 0, class 1 = outer face r = rmax,
 *    class 2 = top face z = ztop, class 3 = any face against a masked cell.
 *    The flux through a boundary face of cell c is -g (T_c - T_inf) with the
 *    series conductance g = 1/(d_c/(2k_c) + 1/h): h = 0 gives Neumann (g = 0),
 *    h = infinity gives Dirichlet at the face (g = 2k_c/d_c).  The axis r = 0
 *    carries no flux (face radius 0).
 *  - Time stepping: Peaceman-Rachford (eq. 8-9), tau_a = tau/2, source in both
 *    half steps; or the locally one-dimensional backward-Euler splitting
 *    ("LOD-BE", tau_a = tau, source in the r half step only).
 *  - Masked cells are identity rows holding 0; they never change.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MASKED 255

/* Status codes returned by every entry point. */
#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

/* A fully assembled problem: geometry, region per cell, and per-cell operator
 * coefficients.  Row-major, r fastest: cell (i, j) is at j*nr + i. */
typedef struct {
  int nr, nz;
  double r0, r1, r2, rmax, z0, zmax, ztop;
  double h[4], tinf[4];
  double k[5], rhoc[5], q[5];
  double *rf, *zf;      /* faces: nr+1, nz+1 */
  double *rc, *zc;      /* centres */
  double *dr, *dz;      /* widths */
  uint8_t *region;      /* nz*nr */
  /* A_r T = Lr_w T_{i-1} + Lr_c T_i + Lr_e T_{i+1} + br */
  double *Lr_w, *Lr_c, *Lr_e, *br;
  /* A_z T = Lz_s T_{j-1} + Lz_c T_j + Lz_n T_{j+1} + bz */
  double *Lz_s, *Lz_c, *Lz_n, *bz;
  /* boundary loss weights: B_r(T) = sum Bw_r * T - Bt_r, likewise z */
  double *Bw_r, *Bt_r, *Bw_z, *Bt_z;
  double *C, *Q;        /* rho c and source per cell (0 when masked) */
  double *V;            /* control volume r_c dr dz (2 pi dropped) */
  /* Temperature-dependent material laws of the nonlinear path (Sec. 2,
   * eq. 1-2): per region, cubic polynomials c0 + c1 T + c2 T^2 + c3 T^3 of
   * the conductivity lambda, the volumetric heat capacity rho c_V and the
   * source amplitude chi I^2/S_C; set by or_nl_set_laws. */
  double lam[5][4], cap[5][4], src[5][4];
} or_problem;

/* ------------------------------------------------------------------ grid -- */

static int region_of(const or_problem *p, double rc, double zc) {
  if (zc >= p->zmax) return 4;
  if (rc < p->r0) return 0;
  if (zc >= p->z0) return OR_MASKED;
  if (rc < p->r1) return 1;
  if (rc < p->r2) return 2;
  return 3;
}

/* Series conductance of the half cell (width d, conductivity k) in series
 * with a surface film of coefficient h. */
static double series_g(double d, double k, double h) {
  if (h == 0.0) return 0.0;
  if (isinf(h)) return 2.0 * k / d;
  return 1.0 / (d / (2.0 * k) + 1.0 / h);
}

/* Conductance between two active cell centres across their common face. */
static double face_G(double da, double ka, double db, double kb) {
  return 1.0 / (da / (2.0 * ka) + db / (2.0 * kb));
}

void or_free(or_problem *p) {
  if (!p) return;
  double **arrs[] = {&p->rf, &p->zf, &p->rc, &p->zc, &p->dr, &p->dz,
                     &p->Lr_w, &p->Lr_c, &p->Lr_e, &p->br,
                     &p->Lz_s, &p->Lz_c, &p->Lz_n, &p->bz,
                     &p->Bw_r, &p->Bt_r, &p->Bw_z, &p->Bt_z,
                     &p->C, &p->Q, &p->V};
  for (size_t a = 0; a < sizeof(arrs) / sizeof(arrs[0]); ++a) free(*arrs[a]);
  free(p->region);
  free(p);
}

/*
 * Build a problem.
 *   geom[7] = r0, r1, r2, rmax, z0, zmax, ztop
 *   rfaces / zfaces: nr+1 / nz+1 monotone face coordinates, or NULL (uniform)
 *   bc[8]   = h[0..3], t_inf[0..3]
 *   k, rhoc, q: 5 values each, one per region
 * Returns NULL on invalid input or allocation failure.
 */
or_problem *or_create(const double *geom, int nr, int nz, const double *rfaces,
                      const double *zfaces, const double *bc, const double *k,
                      const double *rhoc, const double *q) {
  if (nr < 1 || nz < 1) return NULL;
  or_problem *p = (or_problem *)calloc(1, sizeof(or_problem));
  if (!p) return NULL;
  p->nr = nr;
  p->nz = nz;
  p->r0 = geom[0]; p->r1 = geom[1]; p->r2 = geom[2]; p->rmax = geom[3];
  p->z0 = geom[4]; p->zmax = geom[5]; p->ztop = geom[6];
  for (int c = 0; c < 4; ++c) { p->h[c] = bc[c]; p->tinf[c] = bc[4 + c]; }
  for (int m = 0; m < 5; ++m) { p->k[m] = k[m]; p->rhoc[m] = rhoc[m]; p->q[m] = q[m]; }

  size_t n = (size_t)nr * nz;
  p->rf = malloc(sizeof(double) * (nr + 1));
  p->zf = malloc(sizeof(double) * (nz + 1));
  p->rc = malloc(sizeof(double) * nr);
  p->zc = malloc(sizeof(double) * nz);
  p->dr = malloc(sizeof(double) * nr);
  p->dz = malloc(sizeof(double) * nz);
  p->region = malloc(n);
  double **cell[] = {&p->Lr_w, &p->Lr_c, &p->Lr_e, &p->br, &p->Lz_s, &p->Lz_c,
                     &p->Lz_n, &p->bz, &p->Bw_r, &p->Bt_r, &p->Bw_z, &p->Bt_z,
                     &p->C, &p->Q, &p->V};
  int ok = p->rf && p->zf && p->rc && p->zc && p->dr && p->dz && p->region;
  for (size_t a = 0; a < sizeof(cell) / sizeof(cell[0]); ++a) {
    *cell[a] = calloc(n, sizeof(double));
    ok = ok && *cell[a];
  }
  if (!ok) { or_free(p); return NULL; }

  /* Grid (eq. 7): faces, centres, widths. */
  for (int i = 0; i <= nr; ++i) p->rf[i] = rfaces ? rfaces[i] : p->rmax * i / nr;
  for (int j = 0; j <= nz; ++j) p->zf[j] = zfaces ? zfaces[j] : p->ztop * j / nz;
  for (int i = 0; i < nr; ++i) {
    p->rc[i] = rfaces ? 0.5 * (rfaces[i] + rfaces[i + 1]) : (i + 0.5) * p->rmax / nr;
    p->dr[i] = p->rf[i + 1] - p->rf[i];
  }
  for (int j = 0; j < nz; ++j) {
    p->zc[j] = zfaces ? 0.5 * (zfaces[j] + zfaces[j + 1]) : (j + 0.5) * p->ztop / nz;
    p->dz[j] = p->zf[j + 1] - p->zf[j];
  }
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i)
      p->region[(size_t)j * nr + i] = (uint8_t)region_of(p, p->rc[i], p->zc[j]);

  /* Operators (eq. 10-11), one cell at a time. */
  for (int j = 0; j < nz; ++j) {
    for (int i = 0; i < nr; ++i) {
      size_t c = (size_t)j * nr + i;
      int m = p->region[c];
      if (m == OR_MASKED) continue;
      double kc = p->k[m];
      double vol_r = p->rc[i] * p->dr[i]; /* r-weighted width of the cell */
      p->C[c] = p->rhoc[m];
      p->Q[c] = p->q[m];
      p->V[c] = vol_r * p->dz[j];

      /* West face at rf[i]. */
      if (i == 0) {
        /* axis r = 0: the face radius is zero, no flux */
      } else if (p->region[c - 1] == OR_MASKED) {
        /* Never reached on the layout of Fig. 1: cells outside the domain
         * lie at r >= r0 and every active cell of their rows at r < r0, so
         * a cut-out cell is never west of an active one.  Kept so that the
         * operator stays defined for any region map. */
        double g = series_g(p->dr[i], kc, p->h[3]);
        p->Lr_c[c] -= p->rf[i] * g / vol_r;
        p->br[c] += p->rf[i] * g * p->tinf[3] / vol_r;
        p->Bw_r[c] += p->rf[i] * g * p->dz[j];
        p->Bt_r[c] += p->rf[i] * g * p->tinf[3] * p->dz[j];
      } else {
        double G = face_G(p->dr[i - 1], p->k[p->region[c - 1]], p->dr[i], kc);
        p->Lr_w[c] = p->rf[i] * G / vol_r;
        p->Lr_c[c] -= p->rf[i] * G / vol_r;
      }
      /* East face at rf[i+1]. */
      if (i == nr - 1 || p->region[c + 1] == OR_MASKED) {
        int cls = (i == nr - 1) ? 1 : 3;
        double g = series_g(p->dr[i], kc, p->h[cls]);
        p->Lr_c[c] -= p->rf[i + 1] * g / vol_r;
        p->br[c] += p->rf[i + 1] * g * p->tinf[cls] / vol_r;
        p->Bw_r[c] += p->rf[i + 1] * g * p->dz[j];
        p->Bt_r[c] += p->rf[i + 1] * g * p->tinf[cls] * p->dz[j];
      } else {
        double G = face_G(p->dr[i], kc, p->dr[i + 1], p->k[p->region[c + 1]]);
        p->Lr_e[c] = p->rf[i + 1] * G / vol_r;
        p->Lr_c[c] -= p->rf[i + 1] * G / vol_r;
      }
      /* South face at zf[j]. */
      if (j == 0 || p->region[c - nr] == OR_MASKED) {
        int cls = (j == 0) ? 0 : 3;
        double g = series_g(p->dz[j], kc, p->h[cls]);
        p->Lz_c[c] -= g / p->dz[j];
        p->bz[c] += g * p->tinf[cls] / p->dz[j];
        p->Bw_z[c] += vol_r * g;
        p->Bt_z[c] += vol_r * g * p->tinf[cls];
      } else {
        double G = face_G(p->dz[j - 1], p->k[p->region[c - nr]], p->dz[j], kc);
        p->Lz_s[c] = G / p->dz[j];
        p->Lz_c[c] -= G / p->dz[j];
      }
      /* North face at zf[j+1]. */
      if (j == nz - 1 || p->region[c + nr] == OR_MASKED) {
        int cls = (j == nz - 1) ? 2 : 3;
        double g = series_g(p->dz[j], kc, p->h[cls]);
        p->Lz_c[c] -= g / p->dz[j];
        p->bz[c] += g * p->tinf[cls] / p->dz[j];
        p->Bw_z[c] += vol_r * g;
        p->Bt_z[c] += vol_r * g * p->tinf[cls];
      } else {
        double G = face_G(p->dz[j], kc, p->dz[j + 1], p->k[p->region[c + nr]]);
        p->Lz_n[c] = G / p->dz[j];
        p->Lz_c[c] -= G / p->dz[j];
      }
    }
  }
  return p;
}

int or_nr(const or_problem *p) { return p->nr; }
int or_nz(const or_problem *p) { return p->nz; }

/* Copy out grid arrays (any pointer may be NULL). */
void or_grid(const or_problem *p, double *rf, double *zf, double *rc, double *zc) {
  if (rf) memcpy(rf, p->rf, sizeof(double) * (p->nr + 1));
  if (zf) memcpy(zf, p->zf, sizeof(double) * (p->nz + 1));
  if (rc) memcpy(rc, p->rc, sizeof(double) * p->nr);
  if (zc) memcpy(zc, p->zc, sizeof(double) * p->nz);
}

void or_region_map(const or_problem *p, uint8_t *out) {
  memcpy(out, p->region, (size_t)p->nr * p->nz);
}

/* Per-cell coefficient export, for tests that assemble dense matrices.
 * which: 0 Lr_w 1 Lr_c 2 Lr_e 3 br 4 Lz_s 5 Lz_c 6 Lz_n 7 bz 8 C 9 Q 10 V
 *        11 Bw_r 12 Bt_r 13 Bw_z 14 Bt_z */
int or_coeffs(const or_problem *p, int which, double *out) {
  const double *src[] = {p->Lr_w, p->Lr_c, p->Lr_e, p->br, p->Lz_s, p->Lz_c,
                         p->Lz_n, p->bz, p->C, p->Q, p->V,
                         p->Bw_r, p->Bt_r, p->Bw_z, p->Bt_z};
  if (which < 0 || which > 14) return OR_EINVAL;
  memcpy(out, src[which], sizeof(double) * (size_t)p->nr * p->nz);
  return OR_OK;
}

/* ------------------------------------------------------------ operators -- */

/* (A_r T) and (A_z T) per cell, including the boundary constants.  Masked
 * cells get 0. */
void or_apply(const or_problem *p, const double *T, double *Ar, double *Az) {
  int nr = p->nr, nz = p->nz;
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      size_t c = (size_t)j * nr + i;
      if (p->region[c] == OR_MASKED) {
        if (Ar) Ar[c] = 0.0;
        if (Az) Az[c] = 0.0;
        continue;
      }
      if (Ar) {
        double v = p->Lr_c[c] * T[c] + p->br[c];
        if (i > 0) v += p->Lr_w[c] * T[c - 1];
        if (i < nr - 1) v += p->Lr_e[c] * T[c + 1];
        Ar[c] = v;
      }
      if (Az) {
        double v = p->Lz_c[c] * T[c] + p->bz[c];
        if (j > 0) v += p->Lz_s[c] * T[c - nr];
        if (j < nz - 1) v += p->Lz_n[c] * T[c + nr];
        Az[c] = v;
      }
    }
}

/* ---------------------------------------------------------------- Thomas -- */

/* Solve a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i = 0..n-1 (a_0 and
 * c_{n-1} ignored), by forward elimination and back substitution without
 * pivoting.  cp and dp are caller-provided work arrays of length n. */
void or_thomas(int n, const double *a, const double *b, const double *c,
               const double *d, double *x, double *cp, double *dp) {
  cp[0] = c[0] / b[0];
  dp[0] = d[0] / b[0];
  for (int i = 1; i < n; ++i) {
    double den = b[i] - a[i] * cp[i - 1];
    cp[i] = (i < n - 1) ? c[i] / den : 0.0;
    dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
  }
  x[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* ------------------------------------------------------------- ADI steps -- */

/* Scratch for the line solves. */
typedef struct { double *a, *b, *c, *d, *x, *cp, *dp; } or_lines;

static int lines_alloc(or_lines *w, int n) {
  w->a = malloc(sizeof(double) * n); w->b = malloc(sizeof(double) * n);
  w->c = malloc(sizeof(double) * n); w->d = malloc(sizeof(double) * n);
  w->x = malloc(sizeof(double) * n); w->cp = malloc(sizeof(double) * n);
  w->dp = malloc(sizeof(double) * n);
  return w->a && w->b && w->c && w->d && w->x && w->cp && w->dp;
}
static void lines_free(or_lines *w) {
  free(w->a); free(w->b); free(w->c); free(w->d); free(w->x); free(w->cp); free(w->dp);
}

/*
 * r-implicit half step (eq. 8 for PR, first LOD-BE stage):
 *   (C/ta - L_r) Tout = (C/ta) Tin + theta*(A_z Tin) + Q + b_r
 * one Thomas solve per row j.
 */
static void row_r(const or_problem *p, double ta, double theta,
                  const double *Tin, double *Tout, or_lines *w, int j) {
  int nr = p->nr, nz = p->nz;
  for (int i = 0; i < nr; ++i) {
    size_t c = (size_t)j * nr + i;
    if (p->region[c] == OR_MASKED) {
      w->a[i] = 0.0; w->b[i] = 1.0; w->c[i] = 0.0; w->d[i] = 0.0;
      continue;
    }
    double Cc = p->C[c] / ta;
    w->a[i] = -p->Lr_w[c];
    w->b[i] = Cc - p->Lr_c[c];
    w->c[i] = -p->Lr_e[c];
    double az = p->Lz_c[c] * Tin[c] + p->bz[c];
    if (j > 0) az += p->Lz_s[c] * Tin[c - nr];
    if (j < nz - 1) az += p->Lz_n[c] * Tin[c + nr];
    w->d[i] = Cc * Tin[c] + theta * az + p->Q[c] + p->br[c];
  }
  or_thomas(nr, w->a, w->b, w->c, w->d, w->x, w->cp, w->dp);
  for (int i = 0; i < nr; ++i) Tout[(size_t)j * nr + i] = w->x[i];
}

/*
 * z-implicit half step (eq. 9 for PR, second LOD-BE stage):
 *   (C/ta - L_z) Tout = (C/ta) Tin + theta*(A_r Tin + Q) + b_z
 * one Thomas solve per column i.
 */
static void col_z(const or_problem *p, double ta, double theta,
                  const double *Tin, double *Tout, or_lines *w, int i) {
  int nr = p->nr, nz = p->nz;
  for (int j = 0; j < nz; ++j) {
    size_t c = (size_t)j * nr + i;
    if (p->region[c] == OR_MASKED) {
      w->a[j] = 0.0; w->b[j] = 1.0; w->c[j] = 0.0; w->d[j] = 0.0;
      continue;
    }
    double Cc = p->C[c] / ta;
    w->a[j] = -p->Lz_s[c];
    w->b[j] = Cc - p->Lz_c[c];
    w->c[j] = -p->Lz_n[c];
    double ar = p->Lr_c[c] * Tin[c] + p->br[c];
    if (i > 0) ar += p->Lr_w[c] * Tin[c - 1];
    if (i < nr - 1) ar += p->Lr_e[c] * Tin[c + 1];
    w->d[j] = Cc * Tin[c] + theta * (ar + p->Q[c]) + p->bz[c];
  }
  or_thomas(nz, w->a, w->b, w->c, w->d, w->x, w->cp, w->dp);
  for (int j = 0; j < nz; ++j) Tout[(size_t)j * nr + i] = w->x[j];
}

/*
 * Advance T by nsteps steps of size dt.
 *   scheme 0: Peaceman-Rachford (eq. 8-9): ta = dt/2, theta = 1.
 *   scheme 1: LOD backward Euler: ta = dt, theta = 0.
 * If Tbar is not NULL it receives the intermediate field of the last step.
 */
int or_step(const or_problem *p, int scheme, double dt, long nsteps, double *T,
            double *Tbar) {
  if (!(dt > 0.0) || nsteps < 0 || (scheme != 0 && scheme != 1)) return OR_EINVAL;
  size_t n = (size_t)p->nr * p->nz;
  int L = p->nr > p->nz ? p->nr : p->nz;
  double ta = scheme == 0 ? 0.5 * dt : dt;
  double theta = scheme == 0 ? 1.0 : 0.0;
  or_lines w;
  double *mid = malloc(sizeof(double) * n);
  if (!mid || !lines_alloc(&w, L)) { free(mid); lines_free(&w); return OR_ENOMEM; }
  for (long s = 0; s < nsteps; ++s) {
    for (int j = 0; j < p->nz; ++j) row_r(p, ta, theta, T, mid, &w, j);
    for (int i = 0; i < p->nr; ++i) col_z(p, ta, theta, mid, T, &w, i);
  }
  if (Tbar && nsteps > 0) memcpy(Tbar, mid, sizeof(double) * n);
  free(mid);
  lines_free(&w);
  return OR_OK;
}

/*
 * The same steps with the line solves of each half step shared among
 * nthreads OpenMP threads, the parallelisation of the paper (Sec. 4: the
 * independent line systems of a half step run on the cores of one shared-
 * memory node).  Every line is solved by the same sequence of operations as
 * in or_step, so T comes out bit-identical; only the CPU timing of the method
 * changes.  *used receives the number of threads that ran.
 */
int or_step_omp(const or_problem *p, int scheme, double dt, long nsteps, double *T,
                int nthreads, int *used) {
  if (!(dt > 0.0) || nsteps < 0 || (scheme != 0 && scheme != 1) || nthreads < 1)
    return OR_EINVAL;
  size_t n = (size_t)p->nr * p->nz;
  int L = p->nr > p->nz ? p->nr : p->nz;
  double ta = scheme == 0 ? 0.5 * dt : dt;
  double theta = scheme == 0 ? 1.0 : 0.0;
  double *mid = malloc(sizeof(double) * n);
  or_lines *w = calloc((size_t)nthreads, sizeof(or_lines));
  int ok = mid && w;
  for (int t = 0; ok && t < nthreads; ++t) ok = lines_alloc(&w[t], L);
  if (!ok) {
    for (int t = 0; w && t < nthreads; ++t) lines_free(&w[t]);
    free(w); free(mid);
    return OR_ENOMEM;
  }
  int ran = 1;
#pragma omp parallel num_threads(nthreads)
  {
#ifdef _OPENMP
    or_lines *mine = &w[omp_get_thread_num()];
#pragma omp single
    ran = omp_get_num_threads();
#else
    or_lines *mine = &w[0];
#endif
    for (long s = 0; s < nsteps; ++s) {
#pragma omp for schedule(static)
      for (int j = 0; j < p->nz; ++j) row_r(p, ta, theta, T, mid, mine, j);
#pragma omp for schedule(static)
      for (int i = 0; i < p->nr; ++i) col_z(p, ta, theta, mid, T, mine, i);
    }
  }
  if (used) *used = ran;
  for (int t = 0; t < nthreads; ++t) lines_free(&w[t]);
  free(w);
  free(mid);
  return OR_OK;
}

/* ------------------------------------------------------------ diagnostics -- */

/* out[0] = E = sum C T V, out[1] = B_r(T), out[2] = B_z(T), out[3] = P = sum Q V
 * over active cells.  B_r / B_z are the heat flows out through the r- / z-
 * boundary faces (2 pi dropped). */
void or_energy(const or_problem *p, const double *T, double *out) {
  double E = 0.0, Br = 0.0, Bz = 0.0, P = 0.0;
  size_t n = (size_t)p->nr * p->nz;
  for (size_t c = 0; c < n; ++c) {
    if (p->region[c] == OR_MASKED) continue;
    E += p->C[c] * T[c] * p->V[c];
    Br += p->Bw_r[c] * T[c] - p->Bt_r[c];
    Bz += p->Bw_z[c] * T[c] - p->Bt_z[c];
    P += p->Q[c] * p->V[c];
  }
  out[0] = E; out[1] = Br; out[2] = Bz; out[3] = P;
}

/*
 * Terminal-face profile: the cell values of one row, resampled at
 * r_k = (k + 0.5) * rmax / npts by linear interpolation between cell centres,
 * held constant beyond the first and last centres.
 *   which 0: top row j = nz-1; which 1: first row with z_c >= zmax.
 * Every cell of the row must be active.
 */
int or_profile(const or_problem *p, const double *T, int which, int npts, double *out) {
  int nr = p->nr, j = -1;
  if (npts < 1) return OR_EINVAL;
  if (which == 0) j = p->nz - 1;
  else if (which == 1) {
    for (int jj = 0; jj < p->nz; ++jj)
      if (p->zc[jj] >= p->zmax) { j = jj; break; }
  }
  if (j < 0) return OR_EINVAL;
  for (int i = 0; i < nr; ++i)
    if (p->region[(size_t)j * nr + i] == OR_MASKED) return OR_EINVAL;
  const double *row = T + (size_t)j * nr;
  for (int kk = 0; kk < npts; ++kk) {
    double r = (kk + 0.5) * p->rmax / npts;
    double v;
    if (r <= p->rc[0]) v = row[0];
    else if (r >= p->rc[nr - 1]) v = row[nr - 1];
    else {
      int i = 0;
      while (!(r < p->rc[i + 1])) ++i; /* rc[i] <= r < rc[i+1] */
      v = row[i] + (row[i + 1] - row[i]) * (r - p->rc[i]) / (p->rc[i + 1] - p->rc[i]);
    }
    out[kk] = v;
  }
  return OR_OK;
}

/* ===================================================================== */
/*  Nonlinear path: the simple (Picard) iteration of Sec. 3 (eq. 12-14),  */
/*  the pulsed source of Sec. 2 (eq. 2-4) and the adaptive time step of  */
/*  Sec. 3 and Sec. 4.                                                   */
/* ===================================================================== */
/*
 * Readings (listed with the others in the design notes):
 *  - The material laws are not published; each region carries cubic
 *    polynomials in T for lambda, rho c_V and the source amplitude
 *    chi(T) I^2/S_C (zero outside the heater for the paper's cell).
 *  - Face conductivity (the garbled half-node formula after eq. 11): each
 *    side's lambda is evaluated at the mean of the two cell temperatures
 *    and the two half cells are combined in series.  Inside one material
 *    on a uniform grid this is the paper's lambda_m((T_i + T_{i+1})/2)/h;
 *    with constant laws it is the linear path's harmonic conductance.
 *    A boundary film uses lambda at the cell's own temperature.
 *  - The source of both half steps is X at the half layer: chi at the
 *    iterate (eq. 12) or at T-bar (eq. 14), times p(t + tau/2).
 *  - Iteration: T^0 = T (eq. 12) or T-bar (eq. 14); stop when the max norm
 *    of T^{s+1} - T^s over the cells of the domain is below eps (eq. 13);
 *    a half step that has not stopped after iter_max solves fails.
 *  - Time step (Sec. 4): at the start of every step tau = t_trs/1000 inside
 *    a transition of the source (the first t_trs of a switch-on or a
 *    switch-off) and t_src/100 elsewhere; a step ends no later than the next
 *    switch point, transition end or t_end, so that transitions are always
 *    taken with the short step; a failed step is retried with tau/2.
 *  - Periodic regime (Sec. 4, criterion unstated): at each period start the
 *    field is compared with the one of the previous period start; the run
 *    stops once the max norm of the change is below a given tolerance.
 */

/* c0 + c1 T + c2 T^2 + c3 T^3 */
static double poly3(const double *c, double T) {
  return c[0] + T * (c[1] + T * (c[2] + T * c[3]));
}

/* lam, cap, src: 5 regions x 4 coefficients each, region-major. */
void or_nl_set_laws(or_problem *p, const double *lam, const double *cap, const double *src) {
  for (int m = 0; m < 5; ++m)
    for (int q = 0; q < 4; ++q) {
      p->lam[m][q] = lam[4 * m + q];
      p->cap[m][q] = cap[4 * m + q];
      p->src[m][q] = src[4 * m + q];
    }
}

/*
 * Normalised periodic source p(t) (eq. 2).  kind 0: p = 1; kind 1: the
 * rectangular pulse train u(t) of eq. 3 (Heaviside step taken as 1 at 0);
 * kind 2: the smoothed switching v(t) of eq. 4.  pp = t_per, t_src, t_trs,
 * xi, zeta.  The sum over periods runs over every n from 0 up to the period
 * after the one containing t (later periods contribute exactly nothing for
 * t >= 0 in eq. 3, and at most the far tail of the erf in eq. 4).
 */
double or_pulse(int kind, double t, const double *pp) {
  if (kind == 0) return 1.0;
  const double tper = pp[0], tsrc = pp[1], ttrs = pp[2], xi = pp[3], zeta = pp[4];
  long nmax = (long)floor(t / tper) + 1;
  double s = 0.0;
  for (long n = 0; n <= nmax; ++n) {
    double a = t - n * tper;       /* time since the n-th switch-on */
    double b = t - n * tper - tsrc; /* time since the n-th switch-off */
    if (kind == 1) {
      s += (a >= 0.0 ? 1.0 : 0.0) - (b >= 0.0 ? 1.0 : 0.0);
    } else {
      s += 0.5 * (erf(xi * (zeta * a / ttrs - 1.0)) - erf(xi * (zeta * b / ttrs - 1.0)));
    }
  }
  return s;
}

/* Coefficients of A_r at row j, position i, with the laws evaluated on the
 * field F (eq. 10 in balance form): A_r T = w T[i-1] + c T[i] + e T[i+1] + b. */
static void nl_coef_r(const or_problem *p, const double *F, int j, int i,
                      double *w, double *cc, double *e, double *b) {
  int nr = p->nr;
  size_t c = (size_t)j * nr + i;
  int m = p->region[c];
  double vol_r = p->rc[i] * p->dr[i];
  double kc = poly3(p->lam[m], F[c]);
  *w = 0.0; *cc = 0.0; *e = 0.0; *b = 0.0;
  if (i == 0) {
    /* axis: no flux */
  } else if (p->region[c - 1] == OR_MASKED) {
    double g = series_g(p->dr[i], kc, p->h[3]);
    *cc -= p->rf[i] * g / vol_r;
    *b += p->rf[i] * g * p->tinf[3] / vol_r;
  } else {
    double Tf = 0.5 * (F[c - 1] + F[c]);
    double G = face_G(p->dr[i - 1], poly3(p->lam[p->region[c - 1]], Tf), p->dr[i], poly3(p->lam[m], Tf));
    *w = p->rf[i] * G / vol_r;
    *cc -= p->rf[i] * G / vol_r;
  }
  if (i == nr - 1 || p->region[c + 1] == OR_MASKED) {
    int cls = (i == nr - 1) ? 1 : 3;
    double g = series_g(p->dr[i], kc, p->h[cls]);
    *cc -= p->rf[i + 1] * g / vol_r;
    *b += p->rf[i + 1] * g * p->tinf[cls] / vol_r;
  } else {
    double Tf = 0.5 * (F[c] + F[c + 1]);
    double G = face_G(p->dr[i], poly3(p->lam[m], Tf), p->dr[i + 1], poly3(p->lam[p->region[c + 1]], Tf));
    *e = p->rf[i + 1] * G / vol_r;
    *cc -= p->rf[i + 1] * G / vol_r;
  }
}

/* Coefficients of A_z at row j, position i, laws on F (eq. 11):
 * A_z T = s T[j-1] + c T[j] + n T[j+1] + b. */
static void nl_coef_z(const or_problem *p, const double *F, int j, int i,
                      double *so, double *cc, double *no, double *b) {
  int nr = p->nr, nz = p->nz;
  size_t c = (size_t)j * nr + i;
  int m = p->region[c];
  double kc = poly3(p->lam[m], F[c]);
  *so = 0.0; *cc = 0.0; *no = 0.0; *b = 0.0;
  if (j == 0 || p->region[c - nr] == OR_MASKED) {
    int cls = (j == 0) ? 0 : 3;
    double g = series_g(p->dz[j], kc, p->h[cls]);
    *cc -= g / p->dz[j];
    *b += g * p->tinf[cls] / p->dz[j];
  } else {
    double Tf = 0.5 * (F[c - nr] + F[c]);
    double G = face_G(p->dz[j - 1], poly3(p->lam[p->region[c - nr]], Tf), p->dz[j], poly3(p->lam[m], Tf));
    *so = G / p->dz[j];
    *cc -= G / p->dz[j];
  }
  if (j == nz - 1 || p->region[c + nr] == OR_MASKED) {
    int cls = (j == nz - 1) ? 2 : 3;
    double g = series_g(p->dz[j], kc, p->h[cls]);
    *cc -= g / p->dz[j];
    *b += g * p->tinf[cls] / p->dz[j];
  } else {
    double Tf = 0.5 * (F[c] + F[c + nr]);
    double G = face_G(p->dz[j], poly3(p->lam[m], Tf), p->dz[j + 1], poly3(p->lam[p->region[c + nr]], Tf));
    *no = G / p->dz[j];
    *cc -= G / p->dz[j];
  }
}

/* (A_r T) and (A_z T) with the laws evaluated on the field F, boundary
 * constants included (0 outside the domain). */
void or_nl_apply(const or_problem *p, const double *F, const double *T, double *Ar, double *Az) {
  int nr = p->nr, nz = p->nz;
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      size_t c = (size_t)j * nr + i;
      if (p->region[c] == OR_MASKED) { Ar[c] = 0.0; Az[c] = 0.0; continue; }
      double w, cc, e, b;
      nl_coef_r(p, F, j, i, &w, &cc, &e, &b);
      double v = cc * T[c] + b;
      if (i > 0) v += w * T[c - 1];
      if (i < nr - 1) v += e * T[c + 1];
      Ar[c] = v;
      nl_coef_z(p, F, j, i, &w, &cc, &e, &b);
      v = cc * T[c] + b;
      if (j > 0) v += w * T[c - nr];
      if (j < nz - 1) v += e * T[c + nr];
      Az[c] = v;
    }
}

/* Largest |a - b| over the cells of the domain (the norm of eq. 13). */
static double max_change(const or_problem *p, const double *a, const double *b) {
  double d = 0.0;
  size_t n = (size_t)p->nr * p->nz;
  for (size_t c = 0; c < n; ++c) {
    if (p->region[c] == OR_MASKED) continue;
    double x = fabs(a[c] - b[c]);
    if (x > d) d = x;
  }
  return d;
}

/*
 * First half step by the iteration of eq. 12: implicit in r with the laws
 * at the iterate T^s, explicit Lambda_z at the current layer T (laws at T).
 * Tbar receives the last iterate.  Returns the number of solves if the stop
 * rule of eq. 13 was met within iter_max, else -1 (Tbar then holds the last
 * iterate).  work: 2 fields.  *last_change: the norm that decided.
 */
static int nl_half_r(const or_problem *p, const double *T, double ta, double pval,
                     double eps, int iter_max, double *Tbar, double *work,
                     or_lines *w, double *last_change) {
  int nr = p->nr, nz = p->nz;
  size_t n = (size_t)nr * nz;
  double *Ts = work, *Az = work + n;
  /* the explicit part Lambda_z[T] does not change over the iteration */
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      size_t c = (size_t)j * nr + i;
      if (p->region[c] == OR_MASKED) { Az[c] = 0.0; continue; }
      double so, cc, no, b;
      nl_coef_z(p, T, j, i, &so, &cc, &no, &b);
      double az = cc * T[c] + b;
      if (j > 0) az += so * T[c - nr];
      if (j < nz - 1) az += no * T[c + nr];
      Az[c] = az;
    }
  memcpy(Ts, T, sizeof(double) * n);                       /* T^0 = T */
  for (int s = 0; s < iter_max; ++s) {
    for (int j = 0; j < nz; ++j) {
      for (int i = 0; i < nr; ++i) {
        size_t c = (size_t)j * nr + i;
        int m = p->region[c];
        if (m == OR_MASKED) {
          w->a[i] = 0.0; w->b[i] = 1.0; w->c[i] = 0.0; w->d[i] = 0.0;
          continue;
        }
        double we, cc, ea, b;
        nl_coef_r(p, Ts, j, i, &we, &cc, &ea, &b);
        double Cc = poly3(p->cap[m], Ts[c]) / ta;
        double X = poly3(p->src[m], Ts[c]) * pval;
        w->a[i] = -we;
        w->b[i] = Cc - cc;
        w->c[i] = -ea;
        w->d[i] = Cc * T[c] + Az[c] + X + b;
      }
      or_thomas(nr, w->a, w->b, w->c, w->d, w->x, w->cp, w->dp);
      for (int i = 0; i < nr; ++i) Tbar[(size_t)j * nr + i] = w->x[i];
    }
    double d = max_change(p, Tbar, Ts);
    *last_change = d;
    if (d < eps) return s + 1;
    memcpy(Ts, Tbar, sizeof(double) * n);
  }
  return -1;
}

/*
 * Second half step by the iteration of eq. 14: implicit in z with the laws
 * at the iterate, rho c_V and the source at T-bar, explicit Lambda_r[T-bar]
 * (laws at T-bar).  Same conventions as nl_half_r.
 */
static int nl_half_z(const or_problem *p, const double *Tbar, double ta, double pval,
                     double eps, int iter_max, double *That, double *work,
                     or_lines *w, double *last_change) {
  int nr = p->nr, nz = p->nz;
  size_t n = (size_t)nr * nz;
  double *Ts = work, *Ar = work + n;
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      size_t c = (size_t)j * nr + i;
      int m = p->region[c];
      if (m == OR_MASKED) { Ar[c] = 0.0; continue; }
      double we, cc, ea, b;
      nl_coef_r(p, Tbar, j, i, &we, &cc, &ea, &b);
      double ar = cc * Tbar[c] + b;
      if (i > 0) ar += we * Tbar[c - 1];
      if (i < nr - 1) ar += ea * Tbar[c + 1];
      Ar[c] = ar + poly3(p->src[m], Tbar[c]) * pval;   /* Lambda_r[T-bar] + X-bar */
    }
  memcpy(Ts, Tbar, sizeof(double) * n);                    /* T^0 = T-bar */
  for (int s = 0; s < iter_max; ++s) {
    for (int i = 0; i < nr; ++i) {
      for (int j = 0; j < nz; ++j) {
        size_t c = (size_t)j * nr + i;
        int m = p->region[c];
        if (m == OR_MASKED) {
          w->a[j] = 0.0; w->b[j] = 1.0; w->c[j] = 0.0; w->d[j] = 0.0;
          continue;
        }
        double so, cc, no, b;
        nl_coef_z(p, Ts, j, i, &so, &cc, &no, &b);
        double Cc = poly3(p->cap[m], Tbar[c]) / ta;
        w->a[j] = -so;
        w->b[j] = Cc - cc;
        w->c[j] = -no;
        w->d[j] = Cc * Tbar[c] + Ar[c] + b;
      }
      or_thomas(nz, w->a, w->b, w->c, w->d, w->x, w->cp, w->dp);
      for (int j = 0; j < nz; ++j) That[(size_t)j * nr + i] = w->x[j];
    }
    double d = max_change(p, That, Ts);
    *last_change = d;
    if (d < eps) return s + 1;
    memcpy(Ts, That, sizeof(double) * n);
  }
  return -1;
}

/*
 * One step of size tau from time t by eq. 12 then eq. 14 (Peaceman-
 * Rachford half steps of tau/2, source at t + tau/2).  On success T is
 * replaced by T-hat and 1 is returned; if either iteration fails to stop
 * within iter_max solves, T is left unchanged and 0 is returned.  it[0],
 * it[1] receive the solves of each half step (-1: failed, 0: not run);
 * chg[0], chg[1] the last change norm of each (the value compared with eps).
 */
int or_nl_step(const or_problem *p, double *T, double tau, double t, int kind, const double *pp,
               double eps, int iter_max, int *it, double *chg) {
  size_t n = (size_t)p->nr * p->nz;
  int L = p->nr > p->nz ? p->nr : p->nz;
  double ta = 0.5 * tau;
  double pval = or_pulse(kind, t + 0.5 * tau, pp);
  or_lines w;
  double *buf = malloc(sizeof(double) * 4 * n);
  if (!buf || !lines_alloc(&w, L)) { free(buf); lines_free(&w); return OR_ENOMEM; }
  double *Tbar = buf, *That = buf + n, *work = buf + 2 * n;
  it[0] = it[1] = 0;
  chg[0] = chg[1] = 0.0;
  int ok = 0;
  it[0] = nl_half_r(p, T, ta, pval, eps, iter_max, Tbar, work, &w, &chg[0]);
  if (it[0] > 0) {
    it[1] = nl_half_z(p, Tbar, ta, pval, eps, iter_max, That, work, &w, &chg[1]);
    if (it[1] > 0) {
      memcpy(T, That, sizeof(double) * n);
      ok = 1;
    }
  }
  free(buf);
  lines_free(&w);
  return ok;
}

/* Switch points and transition ends of the source in the period of t and
 * the next one: n t_per, n t_per + t_trs, n t_per + t_src, n t_per + t_src
 * + t_trs.  Returns the first one later than t + guard (or +inf). */
static double next_boundary(double t, const double *pp, double guard) {
  const double tper = pp[0], tsrc = pp[1], ttrs = pp[2];
  double n0 = floor(t / tper);
  double best = INFINITY;
  for (int k = 0; k < 2; ++k) {
    double base = (n0 + k) * tper;
    double cand[4] = {base, base + ttrs, base + tsrc, base + tsrc + ttrs};
    for (int q = 0; q < 4; ++q)
      if (cand[q] > t + guard && cand[q] < best) best = cand[q];
  }
  return best;
}

/* Inside a transition: the first t_trs after a switch-on or a switch-off. */
static int in_transition(double t, const double *pp) {
  const double tper = pp[0], tsrc = pp[1], ttrs = pp[2];
  double ph = t - floor(t / tper) * tper;
  return ph < ttrs || (ph >= tsrc && ph < tsrc + ttrs);
}

/*
 * The adaptive loop of Sec. 4 from time *t up to t_end (or the periodic
 * regime).  kind / pp: the source pulse (pp = t_per, t_src, t_trs, xi,
 * zeta); with kind 0 (constant source) the step is t_src/100 throughout
 * and no boundaries are placed.  ctl = eps, tau_min, periodic_tol (0: no
 * periodic stop), tau_trs_div (1000), tau_src_div (100); iter_max the
 * iteration limit; max_steps a cap on accepted steps.
 * counts[0..4] receive: accepted steps, rejected (halved) attempts, solves
 * of the r iterations, solves of the z iterations, periodic stop flag.
 * If log is not NULL, up to log_cap accepted steps are recorded as
 * (t_before, tau, solves_r, solves_z).  *t is advanced.  Returns OR_OK, or
 * OR_EINVAL when tau fell below tau_min.
 */
int or_nl_run(const or_problem *p, double *T, double *t, double t_end, int kind, const double *pp,
              const double *ctl, int iter_max, long max_steps, long *counts, double *log, long log_cap,
              double *min_margin) {
  const double eps = ctl[0], tau_min = ctl[1], ptol = ctl[2];
  const double div_trs = ctl[3], div_src = ctl[4];
  size_t n = (size_t)p->nr * p->nz;
  double *prev = malloc(sizeof(double) * n);
  if (!prev) return OR_ENOMEM;
  memcpy(prev, T, sizeof(double) * n);
  for (int q = 0; q < 5; ++q) counts[q] = 0;
  double margin = INFINITY;
  int status = OR_OK;
  /* times closer than this to a switch point or transition end count as
   * being on it (t accumulates rounding as it steps) */
  const double guard = 1e-9 * pp[2] / div_trs;
  while (counts[0] < max_steps) {
    if (!(t_end - *t > guard)) break;
    double tau0 = (kind != 0 && in_transition(*t + guard, pp)) ? pp[2] / div_trs : pp[1] / div_src;
    double tau = tau0;
    int ends_period = 0;
    if (kind != 0) {
      double b = next_boundary(*t, pp, guard);
      if (b - *t <= tau) {
        tau = b - *t;
        /* landing on a period start: b is a multiple of t_per */
        double k = floor(b / pp[0] + 0.5);
        ends_period = fabs(b - k * pp[0]) <= guard;
      }
    }
    if (t_end - *t < tau) { tau = t_end - *t; ends_period = 0; }
    int it[2];
    double chg[2];
    for (;;) {
      int ok = or_nl_step(p, T, tau, *t, kind, pp, eps, iter_max, it, chg);
      if (ok < 0) { status = ok; goto done; }
      for (int h = 0; h < 2; ++h)
        if (it[h] != 0) {
          double mg = fabs(chg[h] - eps) / eps;
          if (mg < margin) margin = mg;
        }
      if (ok) break;
      counts[1] += 1;
      tau *= 0.5;
      ends_period = 0;
      if (tau < tau_min) { status = OR_EINVAL; goto done; }
    }
    if (log && counts[0] < log_cap) {
      double *r = log + 4 * counts[0];
      r[0] = *t; r[1] = tau; r[2] = it[0]; r[3] = it[1];
    }
    *t += tau;
    counts[0] += 1;
    counts[2] += it[0];
    counts[3] += it[1];
    if (ends_period && ptol > 0.0) {
      double d = max_change(p, T, prev);
      double mg = fabs(d - ptol) / ptol;
      if (mg < margin) margin = mg;
      memcpy(prev, T, sizeof(double) * n);
      if (d < ptol) { counts[4] = 1; break; }
    }
  }
done:
  if (min_margin) *min_margin = margin;
  free(prev);
  return status;
}
