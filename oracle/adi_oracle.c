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
