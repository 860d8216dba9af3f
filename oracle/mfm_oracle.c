/*
 * mfm_oracle.c -- plain FP64 CPU oracle of the MFV/MFM neighbour loops of
 * arXiv 2211.12243 (Alonso Asensio et al., "Mesh-free hydrodynamics in
 * pkdgrav3").
 *
 * TEST INFRASTRUCTURE ONLY: the checker that the GPU library is compared with.
 * Nothing in the product path links, loads or calls this file.  It shares no
 * code with the HIP library.
 *
 * Every loop is written for clarity, not speed: no blocking, no fusion, no
 * reordering beyond what the definitions state.  OpenMP only splits the
 * independent per-particle (or per-face) work across host threads; every
 * accumulation into a particle happens serially, in a fixed order.
 *
 * Readings of the paper where it is silent are marked "reading:".
 */
#include "mfm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Kernel (sec. 2.3.2).  reading: the cubic spline in compact-support form,  */
/* W(r,H) = 8/(pi H^3) w(r/H), w = 1-6q^2+6q^3 (q<1/2), 2(1-q)^3 (q<1), 0     */
/* beyond; it vanishes for r >= H and integrates to one over 3D space.       */
/* ------------------------------------------------------------------------ */
static double w_shape(double q) {
  if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
  if (q < 1.0) {
    double t = 1.0 - q;
    return 2.0 * t * t * t;
  }
  return 0.0;
}

/* dw/dq of the shape above. */
static double w_shape_dq(double q) {
  if (q < 0.5) return -12.0 * q + 18.0 * q * q;
  if (q < 1.0) {
    double t = 1.0 - q;
    return -6.0 * t * t;
  }
  return 0.0;
}

double orc_kernel_W(double r, double H) {
  return 8.0 / (M_PI * H * H * H) * w_shape(r / H);
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
static int is_periodic(const orc_params *p) {
  return p->box[0] > 0.0 && p->box[1] > 0.0 && p->box[2] > 0.0;
}

/* Minimum-image separation along one axis of side L (L == 0: open axis). */
static double min_image(double d, double L) {
  if (L > 0.0) {
    if (d > 0.5 * L)
      d -= L;
    else if (d < -0.5 * L)
      d += L;
  }
  return d;
}

/* d = x_j - x_i (minimum image). */
static void separation(const orc_params *p, const double *x, const double *y, const double *z,
                       int64_t i, int64_t j, double d[3]) {
  d[0] = min_image(x[j] - x[i], p->box[0]);
  d[1] = min_image(y[j] - y[i], p->box[1]);
  d[2] = min_image(z[j] - z[i], p->box[2]);
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets: N_i = { j : |x_j - x_i| < R_i }, self included.           */
/* The grid only prunes candidates; membership is always the exact distance  */
/* test, so grid and brute force must produce the same sets.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nc[3];
  int64_t *cell_start; /* ncells + 1 */
  int64_t *cell_idx;   /* n */
} orc_grid;

static int grid_build(const orc_params *p, int64_t n, const double *x, const double *y,
                      const double *z, double rmax, orc_grid *g) {
  if (!is_periodic(p) || !(rmax > 0.0)) return 0;
  const double *pos[3] = {x, y, z};
  for (int k = 0; k < 3; ++k) {
    double c = floor(p->box[k] / rmax);
    if (c < 3.0) return 0;
    if (c > 1024.0) c = 1024.0;
    g->nc[k] = (int)c;
  }
  int64_t ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
  g->cell_start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  g->cell_idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *cell_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) {
    int c[3];
    for (int k = 0; k < 3; ++k) {
      c[k] = (int)(pos[k][i] / p->box[k] * g->nc[k]);
      if (c[k] < 0) c[k] = 0;
      if (c[k] >= g->nc[k]) c[k] = g->nc[k] - 1;
    }
    cell_of[i] = ((int64_t)c[2] * g->nc[1] + c[1]) * g->nc[0] + c[0];
    g->cell_start[cell_of[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) g->cell_start[c + 1] += g->cell_start[c];
  int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  memcpy(fill, g->cell_start, (size_t)ncell * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) g->cell_idx[fill[cell_of[i]]++] = i;
  free(fill);
  free(cell_of);
  return 1;
}

static void grid_free(orc_grid *g) {
  free(g->cell_start);
  free(g->cell_idx);
}

/* Operation counting: oracle/opcount.cpp compiles this file with a counting
 * number type and defines these two hooks, so that the arithmetic of the
 * candidate scans is attributed to the neighbour search and not to the loop
 * that called it.  In the plain build they do nothing. */
#ifndef ORC_SEARCH_BEGIN
#define ORC_SEARCH_BEGIN()
#define ORC_SEARCH_END()
#endif

/* Visit the candidates of particle i.  The visitor returns nothing; it sees j
 * and the exact minimum-image separation. */
typedef void (*visit_fn)(void *ctx, int64_t j, const double d[3], double r2);

static void for_candidates(const orc_params *p, int64_t n, const double *x, const double *y,
                           const double *z, const orc_grid *g, int use_grid, int64_t i,
                           visit_fn f, void *ctx) {
  double d[3];
  ORC_SEARCH_BEGIN();
  if (!use_grid) {
    for (int64_t j = 0; j < n; ++j) {
      separation(p, x, y, z, i, j, d);
      f(ctx, j, d, d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    ORC_SEARCH_END();
    return;
  }
  const double *pos[3] = {x, y, z};
  int c[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = (int)(pos[k][i] / p->box[k] * g->nc[k]);
    if (c[k] < 0) c[k] = 0;
    if (c[k] >= g->nc[k]) c[k] = g->nc[k] - 1;
  }
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int cx = (c[0] + dx + g->nc[0]) % g->nc[0];
        int cy = (c[1] + dy + g->nc[1]) % g->nc[1];
        int cz = (c[2] + dz + g->nc[2]) % g->nc[2];
        int64_t cell = ((int64_t)cz * g->nc[1] + cy) * g->nc[0] + cx;
        for (int64_t k = g->cell_start[cell]; k < g->cell_start[cell + 1]; ++k) {
          int64_t j = g->cell_idx[k];
          separation(p, x, y, z, i, j, d);
          f(ctx, j, d, d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
      }
  ORC_SEARCH_END();
}

typedef struct {
  double R2;
  int64_t count;
  int32_t *out; /* may be NULL (count only) */
} collect_ctx;

static void collect_visit(void *vctx, int64_t j, const double d[3], double r2) {
  (void)d;
  collect_ctx *c = (collect_ctx *)vctx;
  if (r2 < c->R2) {
    if (c->out) c->out[c->count] = (int32_t)j;
    c->count++;
  }
}

int orc_neighbours(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *R, int use_grid, int64_t *start,
                   int32_t *idx) {
  if (!p || n < 0 || !x || !y || !z || !R || !start) return -1;
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (R[i] > rmax) rmax = R[i];
  orc_grid g;
  memset(&g, 0, sizeof(g));
  int have_grid = use_grid ? grid_build(p, n, x, y, z, rmax, &g) : 0;
  if (idx == NULL) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      collect_ctx c = {R[i] * R[i], 0, NULL};
      for_candidates(p, n, x, y, z, &g, have_grid, i, collect_visit, &c);
      start[i + 1] = c.count;
    }
    start[0] = 0;
    for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
  } else {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      collect_ctx c = {R[i] * R[i], 0, idx + start[i]};
      for_candidates(p, n, x, y, z, &g, have_grid, i, collect_visit, &c);
    }
  }
  if (have_grid) grid_free(&g);
  return 0;
}

/* Build CSR lists for radius R_i (helper used by the loops below). */
static int build_lists(const orc_params *p, int64_t n, const double *x, const double *y,
                       const double *z, const double *R, int64_t **start, int32_t **idx) {
  *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!*start) return -2;
  orc_neighbours(p, n, x, y, z, R, 1, *start, NULL);
  *idx = (int32_t *)malloc((size_t)((*start)[n] > 0 ? (*start)[n] : 1) * sizeof(int32_t));
  if (!*idx) return -2;
  orc_neighbours(p, n, x, y, z, R, 1, *start, *idx);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* 3x3 symmetric matrices stored as (xx, xy, xz, yy, yz, zz).               */
/* ------------------------------------------------------------------------ */
static double sym_inverse(const double e[6], double b[6]) {
  double c00 = e[3] * e[5] - e[4] * e[4];
  double c01 = e[2] * e[4] - e[1] * e[5];
  double c02 = e[1] * e[4] - e[2] * e[3];
  double c11 = e[0] * e[5] - e[2] * e[2];
  double c12 = e[1] * e[2] - e[0] * e[4];
  double c22 = e[0] * e[3] - e[1] * e[1];
  double det = e[0] * c00 + e[1] * c01 + e[2] * c02;
  b[0] = c00 / det;
  b[1] = c01 / det;
  b[2] = c02 / det;
  b[3] = c11 / det;
  b[4] = c12 / det;
  b[5] = c22 / det;
  return det;
}

static double sym_frob(const double a[6]) {
  return sqrt(a[0] * a[0] + a[3] * a[3] + a[5] * a[5] +
              2.0 * (a[1] * a[1] + a[2] * a[2] + a[4] * a[4]));
}

static void sym_mul(const double a[6], const double v[3], double out[3]) {
  out[0] = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
  out[1] = a[1] * v[0] + a[3] * v[1] + a[4] * v[2];
  out[2] = a[2] * v[0] + a[4] * v[1] + a[5] * v[2];
}

/* Condition number of eq. Ncond with nu = 3: the paper's norm is the sum of
 * squared entries, so (||B|| ||E||)^(1/2) is the product of Frobenius norms. */
static double cond_number(const double e[6]) {
  double b[6];
  double det = sym_inverse(e, b);
  if (!(det != 0.0) || !isfinite(det)) return INFINITY;
  return sym_frob(b) * sym_frob(e) / 3.0;
}

/* ------------------------------------------------------------------------ */
/* Density loop (loop 1 of sec. 2.2.3; sec. 2.3.2 and 2.3.5)                */
/* ------------------------------------------------------------------------ */

/* g(H) = (4 pi/3) H^3 omega^-1(H) - N_NGB = (32/3) sum_j w(r_j/H) - N_NGB and
 * its derivative in H.  g never decreases with H. */
static void g_eval(const double *r, int64_t nr, double H, double nngb, double *g,
                   double *dg) {
  double s = 0.0, ds = 0.0;
  for (int64_t k = 0; k < nr; ++k) {
    double q = r[k] / H;
    if (q < 1.0) {
      s += w_shape(q);
      ds += q * w_shape_dq(q);
    }
  }
  *g = 32.0 / 3.0 * s - nngb;
  *dg = -32.0 / 3.0 * ds / H;
}

/* reading: Newton's method on g(H) = 0 kept inside a bisection bracket
 * (lo, hi); stop when a Newton step (not a bisection step) is below
 * h_tol * H, so the last step converges quadratically and H is the root to
 * roundoff.  Returns iterations, or -1 when the cap was reached. */
static int solve_h(const double *r, int64_t nr, double nngb, double hi, double tol, int maxit,
                   double *H) {
  double lo = 0.0;
  double h = *H;
  if (!(h > lo && h < hi)) h = 0.5 * (lo + hi);
  for (int it = 1; it <= maxit; ++it) {
    double g, dg;
    g_eval(r, nr, h, nngb, &g, &dg);
    if (g == 0.0) {
      *H = h;
      return it;
    }
    if (g < 0.0)
      lo = h;
    else
      hi = h;
    double hn = (dg > 0.0) ? h - g / dg : NAN;
    if (fabs(hn - h) <= tol * hn) { /* a small Newton step: converged */
      *H = hn;
      return it;
    }
    if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
    h = hn;
  }
  *H = h;
  return -1;
}

/* Unweighted E~ = sum_{j != i, r < H} W(r, H) d d^T, used for the anisotropy
 * check while the neighbour volumes are not yet known (reading). */
static double ncond_unweighted(const double *dd, const double *r, int64_t nr, double H) {
  double e[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = 0; k < nr; ++k) {
    if (!(r[k] < H) || r[k] == 0.0) continue;
    double w = orc_kernel_W(r[k], H);
    const double *d = dd + 3 * k;
    e[0] += w * d[0] * d[0];
    e[1] += w * d[0] * d[1];
    e[2] += w * d[0] * d[2];
    e[3] += w * d[1] * d[1];
    e[4] += w * d[1] * d[2];
    e[5] += w * d[2] * d[2];
  }
  return cond_number(e);
}

typedef struct {
  double *r;
  double *d;
  int64_t count, cap;
  double R2;
} cand_ctx;

static void cand_visit(void *vctx, int64_t j, const double d[3], double r2) {
  (void)j;
  cand_ctx *c = (cand_ctx *)vctx;
  if (!(r2 < c->R2)) return;
  if (c->count == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 256;
    c->r = (double *)realloc(c->r, (size_t)c->cap * sizeof(double));
    c->d = (double *)realloc(c->d, (size_t)c->cap * 3 * sizeof(double));
  }
  c->r[c->count] = sqrt(r2);
  c->d[3 * c->count + 0] = d[0];
  c->d[3 * c->count + 1] = d[1];
  c->d[3 * c->count + 2] = d[2];
  c->count++;
}

/* One particle of the density loop: H from the start value H0 within the
 * candidate radius R, the anisotropy boosts, V, and the counts of what went
 * wrong.  use_grid = 0 takes every particle as a candidate. */
typedef struct {
  int64_t noconv, boosts, fails, fallback;
} dens_counts;

static void density_one(const orc_params *p, int64_t n, const double *x, const double *y,
                        const double *z, const orc_grid *g, int use_grid, int periodic,
                        double half, double R, int64_t i, double H0, double *H, double *V,
                        double *ncond, double *nngb, dens_counts *k) {
  cand_ctx c = {NULL, NULL, 0, 0, R * R};
  for_candidates(p, n, x, y, z, g, use_grid, i, cand_visit, &c);
  double hi = R;
  double gv, dg;
  g_eval(c.r, c.count, hi, p->n_ngb, &gv, &dg);
  if (!periodic || gv < 0.0) {
    /* widen: every particle is a candidate */
    k->fallback += periodic ? 1 : 0;
    c.count = 0;
    c.R2 = INFINITY;
    for_candidates(p, n, x, y, z, g, 0, i, cand_visit, &c);
    if (periodic) {
      hi = half;
    } else {
      double rm = 0.0;
      for (int64_t q = 0; q < c.count; ++q) rm = fmax(rm, c.r[q]);
      hi = 2.0 * rm + 1e-300;
    }
  }
  double target = p->n_ngb;
  double h = H0;
  int b = 0;
  double nc;
  for (;;) {
    int it = solve_h(c.r, c.count, target, hi, p->h_tol, p->h_maxit, &h);
    if (it < 0) k->noconv++;
    nc = ncond_unweighted(c.d, c.r, c.count, h);
    if (!(nc > p->ncond_max)) break;
    if (b == p->max_boosts) {
      k->fails++;
      break;
    }
    target *= p->ngb_boost;
    b++;
    k->boosts++;
  }
  double winv = 0.0;
  for (int64_t q = 0; q < c.count; ++q)
    if (c.r[q] < h) winv += orc_kernel_W(c.r[q], h);
  *H = h;
  *V = 1.0 / winv;
  *ncond = nc;
  *nngb = target;
  free(c.r);
  free(c.d);
}

static void density_limits(const orc_params *p, int *periodic, double *half) {
  *periodic = is_periodic(p);
  *half = INFINITY;
  if (*periodic)
    for (int k = 0; k < 3; ++k) *half = fmin(*half, 0.5 * p->box[k]);
}

/* The density loop for the particles with act[i] != 0 (all when act is
 * NULL); the others keep their H, V, ncond and nngb. */
static int density_mask(const orc_params *p, int64_t n, const double *x, const double *y,
                        const double *z, double *H, double *V, double *ncond, double *nngb,
                        const uint8_t *act, orc_counters *cnt) {
  if (!p || n <= 0 || !x || !y || !z || !H || !V || !ncond || !nngb || !cnt) return -1;
  if (!(p->n_ngb > 32.0 / 3.0)) return -1; /* the self term alone would exceed N_NGB */
  int periodic;
  double half;
  density_limits(p, &periodic, &half);
  /* Candidate radius: twice the start value (covers the N_NGB boosts), at
   * most half the box.  A particle whose root is not bracketed falls back to
   * a brute-force search with the widest radius. */
  double *R = (double *)malloc((size_t)n * sizeof(double));
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    R[i] = fmin(2.0 * H[i], half);
    if ((!act || act[i]) && R[i] > rmax) rmax = R[i];
  }
  orc_grid g;
  memset(&g, 0, sizeof(g));
  int have_grid = grid_build(p, n, x, y, z, rmax, &g);
  int64_t noconv = 0, boosts = 0, fails = 0, fallback = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : noconv, boosts, fails, fallback)
  for (int64_t i = 0; i < n; ++i) {
    if (act && !act[i]) continue;
    dens_counts k = {0, 0, 0, 0};
    density_one(p, n, x, y, z, &g, have_grid, periodic, half, R[i], i, H[i], &H[i], &V[i],
                &ncond[i], &nngb[i], &k);
    noconv += k.noconv;
    boosts += k.boosts;
    fails += k.fails;
    fallback += k.fallback;
  }
  if (have_grid) grid_free(&g);
  free(R);
  cnt->h_noconv += noconv;
  cnt->ncond_boosts += boosts;
  cnt->ncond_fail += fails;
  cnt->h_fallback += fallback;
  return 0;
}

int orc_density(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, double *H, double *V, double *ncond, double *nngb,
                orc_counters *cnt) {
  return density_mask(p, n, x, y, z, H, V, ncond, nngb, NULL, cnt);
}

/* The density loop for the nq particles listed in idx only (every particle
 * a candidate, so that a sample of a large set costs nq n separations): the
 * same H, V, ncond and N_NGB as orc_density gives them, written to entry q
 * of the outputs for particle idx[q]. */
int orc_density_at(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *H0, int64_t nq, const int64_t *idx,
                   double *H, double *V, double *ncond, double *nngb, orc_counters *cnt) {
  if (!p || n <= 0 || nq < 0 || !x || !y || !z || !H0 || !idx || !H || !V || !ncond || !nngb ||
      !cnt)
    return -1;
  if (!(p->n_ngb > 32.0 / 3.0)) return -1;
  for (int64_t q = 0; q < nq; ++q)
    if (idx[q] < 0 || idx[q] >= n) return -1;
  int periodic;
  double half;
  density_limits(p, &periodic, &half);
  int64_t noconv = 0, boosts = 0, fails = 0, fallback = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : noconv, boosts, fails, fallback)
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t i = idx[q];
    dens_counts k = {0, 0, 0, 0};
    density_one(p, n, x, y, z, NULL, 0, periodic, half, fmin(2.0 * H0[i], half), i, H0[i],
                &H[q], &V[q], &ncond[q], &nngb[q], &k);
    noconv += k.noconv;
    boosts += k.boosts;
    fails += k.fails;
    fallback += k.fallback;
  }
  cnt->h_noconv += noconv;
  cnt->ncond_boosts += boosts;
  cnt->ncond_fail += fails;
  cnt->h_fallback += fallback;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient loop (loop 2) and time step (loop 4)                             */
/* ------------------------------------------------------------------------ */
enum { Q_RHO = 0, Q_VX = 1, Q_VY = 2, Q_VZ = 3, Q_P = 4, NQ = 5 };

/* The gradient loop for the particles with act[i] != 0 (all when act is
 * NULL); the primitives are set for every particle. */
static int gradients_mask(const orc_params *p, int64_t n, const double *x, const double *y,
                          const double *z, const double *H, const double *V, const double *m,
                          const double *vx, const double *vy, const double *vz,
                          const double *U, double *rho, double *P, double *c, double *B,
                          double *grad, double *alpha, double *ncond, double *dt_i,
                          const uint8_t *act, orc_counters *cnt) {
  if (!p || n <= 0) return -1;
  const double gam = p->gamma;
  /* Primitives: rho = m omega^-1, P = (gamma-1) U omega^-1 (sec. 2.3.7),
   * c = sqrt(gamma P / rho). */
  for (int64_t i = 0; i < n; ++i) {
    rho[i] = m[i] / V[i];
    P[i] = (gam - 1.0) * U[i] / V[i];
    c[i] = sqrt(gam * P[i] / rho[i]);
  }
  const double *qs[NQ] = {rho, vx, vy, vz, P};
  int64_t *start;
  int32_t *idx;
  if (build_lists(p, n, x, y, z, H, &start, &idx)) return -2;
  int64_t pairs = 0, singular = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : pairs, singular)
  for (int64_t i = 0; i < n; ++i) {
    if (act && !act[i]) continue;
    double e[6] = {0, 0, 0, 0, 0, 0};
    double s[NQ][3];
    double qmax[NQ], qmin[NQ];
    for (int q = 0; q < NQ; ++q) {
      s[q][0] = s[q][1] = s[q][2] = 0.0;
      qmax[q] = qmin[q] = qs[q][i];
    }
    double vsig = 0.0;
    for (int64_t k = start[i]; k < start[i + 1]; ++k) {
      int64_t j = idx[k];
      if (j == i) continue;
      double d[3];
      separation(p, x, y, z, i, j, d);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      pairs++;
      if (r == 0.0) continue; /* coincident particles add nothing (reading) */
      /* eq. E_matrix with omega_j = V_j and mu(x_i, x_j) = (x_j - x_i) W(r, H_i) */
      double wv = V[j] * orc_kernel_W(r, H[i]);
      e[0] += wv * d[0] * d[0];
      e[1] += wv * d[0] * d[1];
      e[2] += wv * d[0] * d[2];
      e[3] += wv * d[1] * d[1];
      e[4] += wv * d[1] * d[2];
      e[5] += wv * d[2] * d[2];
      /* eq. LV_gradient: sum_j omega_j (f_j - f_i) mu(x_i, x_j), B applied after */
      for (int q = 0; q < NQ; ++q) {
        double df = qs[q][j] - qs[q][i];
        s[q][0] += wv * df * d[0];
        s[q][1] += wv * df * d[1];
        s[q][2] += wv * df * d[2];
        if (qs[q][j] > qmax[q]) qmax[q] = qs[q][j];
        if (qs[q][j] < qmin[q]) qmin[q] = qs[q][j];
      }
      /* signal velocity (sec. 2.3.10); x_i - x_j = -d */
      double proj = -(d[0] * (vx[i] - vx[j]) + d[1] * (vy[i] - vy[j]) + d[2] * (vz[i] - vz[j])) / r;
      double vs = c[i] + c[j] - fmin(0.0, proj);
      if (vs > vsig) vsig = vs;
    }
    double b[6];
    double det = sym_inverse(e, b);
    if (!(det != 0.0) || !isfinite(det)) singular++;
    double g[NQ][3];
    for (int q = 0; q < NQ; ++q) sym_mul(b, s[q], g[q]);
    double nc = sym_frob(b) * sym_frob(e) / 3.0;
    /* Conditioned Barth-Jespersen limiter (sec. 2.3.6).  reading: the face
     * extrapolations d_j = grad q . (x_j - x_i)/2 are bounded by the
     * neighbour extrema; the bound is relaxed by beta in [1, 2], beta = 2 for
     * a perfectly isotropic neighbourhood and 1 at the N_cond threshold. */
    double a[NQ] = {1, 1, 1, 1, 1};
    if (p->limiter & 1) {
      double dmax[NQ], dmin[NQ];
      for (int q = 0; q < NQ; ++q) dmax[q] = dmin[q] = 0.0;
      for (int64_t k = start[i]; k < start[i + 1]; ++k) {
        int64_t j = idx[k];
        if (j == i) continue;
        double d[3];
        separation(p, x, y, z, i, j, d);
        for (int q = 0; q < NQ; ++q) {
          double ex = 0.5 * (g[q][0] * d[0] + g[q][1] * d[1] + g[q][2] * d[2]);
          if (ex > dmax[q]) dmax[q] = ex;
          if (ex < dmin[q]) dmin[q] = ex;
        }
      }
      double t = (p->ncond_max - nc) / (p->ncond_max - 1.0);
      if (!(t > 0.0)) t = 0.0;
      if (t > 1.0) t = 1.0;
      double beta = 1.0 + t;
      for (int q = 0; q < NQ; ++q) {
        double rp = INFINITY, rm = INFINITY;
        if (dmax[q] > 0.0) rp = (qmax[q] - qs[q][i]) / dmax[q];
        if (dmin[q] < 0.0) rm = (qs[q][i] - qmin[q]) / (-dmin[q]);
        double lim = beta * fmin(rp, rm);
        a[q] = lim < 1.0 ? lim : 1.0;
      }
    }
    for (int k = 0; k < 6; ++k) B[(int64_t)k * n + i] = b[k];
    for (int q = 0; q < NQ; ++q) {
      alpha[(int64_t)q * n + i] = a[q];
      for (int k = 0; k < 3; ++k) grad[(int64_t)(3 * q + k) * n + i] = a[q] * g[q][k];
    }
    ncond[i] = nc;
    dt_i[i] = vsig > 0.0 ? p->c_cfl * H[i] / vsig : INFINITY;
  }
  free(start);
  free(idx);
  cnt->grad_pairs += pairs;
  cnt->singular_e += singular;
  return 0;
}

int orc_gradients(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *H, const double *V, const double *m,
                  const double *vx, const double *vy, const double *vz, const double *U,
                  double *rho, double *P, double *c, double *B, double *grad, double *alpha,
                  double *ncond, double *dt_i, orc_counters *cnt) {
  return gradients_mask(p, n, x, y, z, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha, ncond,
                        dt_i, NULL, cnt);
}

/* ------------------------------------------------------------------------ */
/* Exact Riemann solver (Toro 2009), the solver the paper names in 2.3.3     */
/* ------------------------------------------------------------------------ */

/* Pressure function f_K(p) of one side and its derivative: a shock branch for
 * p > p_K, a rarefaction branch otherwise. */
static void pressure_fn(double gam, double p, double rhoK, double pK, double cK, double *f,
                        double *df) {
  if (p <= pK) {
    double pr = p / pK;
    *f = 2.0 * cK / (gam - 1.0) * (pow(pr, (gam - 1.0) / (2.0 * gam)) - 1.0);
    *df = pow(pr, -(gam + 1.0) / (2.0 * gam)) / (rhoK * cK);
  } else {
    double A = 2.0 / ((gam + 1.0) * rhoK);
    double Bk = (gam - 1.0) / (gam + 1.0) * pK;
    double q = sqrt(A / (Bk + p));
    *f = (p - pK) * q;
    *df = q * (1.0 - 0.5 * (p - pK) / (Bk + p));
  }
}

/* reading: Toro's adaptive starting value of the Newton iteration
 * (primitive-variable guess when the states are close, two-rarefaction or
 * two-shock otherwise), floored at 1e-10 of the mean pressure */
static double riemann_guess(double gam, double rhoL, double PL, double cL, double rhoR,
                            double PR, double cR, double du, double floor_p, int *branch) {
  double pmin = fmin(PL, PR), pmax = fmax(PL, PR);
  double ppv = 0.5 * (PL + PR) - 0.125 * du * (rhoL + rhoR) * (cL + cR);
  if (ppv < 0.0) ppv = 0.0;
  double p0;
  if (pmax / pmin <= 2.0 && pmin <= ppv && ppv <= pmax) {
    p0 = ppv;
    *branch = 0;
  } else if (ppv < pmin) {
    *branch = 1;
    double zz = (gam - 1.0) / (2.0 * gam);
    double num = cL + cR - 0.5 * (gam - 1.0) * du;
    double den = cL / pow(PL, zz) + cR / pow(PR, zz);
    p0 = pow(num / den, 1.0 / zz);
  } else {
    double gL = sqrt(2.0 / ((gam + 1.0) * rhoL) / ((gam - 1.0) / (gam + 1.0) * PL + ppv));
    double gR = sqrt(2.0 / ((gam + 1.0) * rhoR) / ((gam - 1.0) / (gam + 1.0) * PR + ppv));
    p0 = (gL * PL + gR * PR - du) / (gL + gR);
    *branch = 2;
  }
  if (!(p0 > floor_p)) p0 = floor_p;
  return p0;
}

double orc_riemann_guess(double gam, double rhoL, double uL, double PL, double rhoR, double uR,
                         double PR, int *branch) {
  double cL = sqrt(gam * PL / rhoL), cR = sqrt(gam * PR / rhoR);
  int b;
  double p0 = riemann_guess(gam, rhoL, PL, cL, rhoR, PR, cR, uR - uL, 1e-10 * 0.5 * (PL + PR), &b);
  if (branch) *branch = b;
  return p0;
}

int orc_riemann(double gam, double rhoL, double uL, double PL, double rhoR, double uR,
                double PR, double tol, int maxit, double *pstar, double *ustar, int *iters) {
  double cL = sqrt(gam * PL / rhoL), cR = sqrt(gam * PR / rhoR);
  double du = uR - uL;
  *iters = 0;
  /* vacuum is generated when the two rarefactions cannot meet */
  if (2.0 / (gam - 1.0) * (cL + cR) <= du) {
    *pstar = 0.0;
    *ustar = 0.5 * (uL + uR);
    return 1;
  }
  double floor_p = 1e-10 * 0.5 * (PL + PR);
  int branch;
  double p = riemann_guess(gam, rhoL, PL, cL, rhoR, PR, cR, du, floor_p, &branch), fL, dfL, fR,
         dfR;
  int status = 2;
  for (int it = 1; it <= maxit; ++it) {
    pressure_fn(gam, p, rhoL, PL, cL, &fL, &dfL);
    pressure_fn(gam, p, rhoR, PR, cR, &fR, &dfR);
    double pn = p - (fL + fR + du) / (dfL + dfR);
    if (pn < 0.0) pn = floor_p;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    *iters = it;
    if (change < tol) {
      status = 0;
      break;
    }
  }
  pressure_fn(gam, p, rhoL, PL, cL, &fL, &dfL);
  pressure_fn(gam, p, rhoR, PR, cR, &fR, &dfR);
  *pstar = p;
  *ustar = 0.5 * (uL + uR) + 0.5 * (fR - fL);
  return status;
}

int orc_riemann_sample(double gam, double rhoL, double uL, double PL, double rhoR, double uR,
                       double PR, double ps, double us, double xi, double *rho, double *u,
                       double *P) {
  double cL = sqrt(gam * PL / rhoL), cR = sqrt(gam * PR / rhoR);
  double g1 = (gam - 1.0) / (2.0 * gam), g2 = (gam + 1.0) / (2.0 * gam);
  double g4 = 2.0 / (gam - 1.0), g5 = 2.0 / (gam + 1.0), g6 = (gam - 1.0) / (gam + 1.0);
  double g7 = 0.5 * (gam - 1.0), g3 = 2.0 * gam / (gam - 1.0);
  if (xi <= us) { /* left of the contact */
    if (ps <= PL) { /* left rarefaction */
      if (xi <= uL - cL) {
        *rho = rhoL; *u = uL; *P = PL;
      } else {
        double cml = cL * pow(ps / PL, g1);
        if (xi > us - cml) {
          *rho = rhoL * pow(ps / PL, 1.0 / gam); *u = us; *P = ps;
        } else { /* inside the fan */
          double cc = g5 * (cL + g7 * (uL - xi));
          *u = g5 * (cL + g7 * uL + xi);
          *rho = rhoL * pow(cc / cL, g4);
          *P = PL * pow(cc / cL, g3);
        }
      }
    } else { /* left shock */
      double pml = ps / PL;
      double sl = uL - cL * sqrt(g2 * pml + g1);
      if (xi <= sl) {
        *rho = rhoL; *u = uL; *P = PL;
      } else {
        *rho = rhoL * (pml + g6) / (pml * g6 + 1.0); *u = us; *P = ps;
      }
    }
  } else { /* right of the contact */
    if (ps > PR) { /* right shock */
      double pmr = ps / PR;
      double sr = uR + cR * sqrt(g2 * pmr + g1);
      if (xi >= sr) {
        *rho = rhoR; *u = uR; *P = PR;
      } else {
        *rho = rhoR * (pmr + g6) / (pmr * g6 + 1.0); *u = us; *P = ps;
      }
    } else { /* right rarefaction */
      if (xi >= uR + cR) {
        *rho = rhoR; *u = uR; *P = PR;
      } else {
        double cmr = cR * pow(ps / PR, g1);
        if (xi <= us + cmr) {
          *rho = rhoR * pow(ps / PR, 1.0 / gam); *u = us; *P = ps;
        } else {
          double cc = g5 * (cR - g7 * (uR - xi));
          *u = g5 * (-cR + g7 * uR + xi);
          *rho = rhoR * pow(cc / cR, g4);
          *P = PR * pow(cc / cR, g3);
        }
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Flux loop (loop 3)                                                        */
/* ------------------------------------------------------------------------ */

/* reading of the pairwise limiter (sec. 2.3.6, psi_1 and psi_2): the face
 * value qf extrapolated from the own side (value qo) towards the other side
 * (value qn) may overshoot the midpoint by at most psi_2 |qo - qn| and the
 * pair minimum / maximum by psi_1 |qo - qn| (a sign-preserving ratio when that
 * would cross zero). */
double orc_pair_limit(double qf, double qo, double qn, double psi1, double psi2) {
  if (qo == qn) return qo;
  double dq = fabs(qo - qn);
  double d1 = psi1 * dq, d2 = psi2 * dq;
  double qbar = 0.5 * (qo + qn);
  if (qo < qn) {
    double lo = qo;
    double lower = ((lo - d1) * lo > 0.0) ? lo - d1 : lo / (1.0 + d1 / fabs(lo));
    return fmax(lower, fmin(qbar + d2, qf));
  } else {
    double hi = qo;
    double upper = ((hi + d1) * hi > 0.0) ? hi + d1 : hi / (1.0 + d1 / fabs(hi));
    return fmin(upper, fmax(qbar - d2, qf));
  }
}

/* The face contribution A_ij F_ij of the pair (i, j), each side's primitives
 * predicted over its own time ti, tj (half the step on a global step). */
static int face_tau(const orc_params *p, int64_t n, int64_t i, int64_t j, const double *x,
                    const double *y, const double *z, const double *H, const double *V,
                    const double *rho, const double *vx, const double *vy, const double *vz,
                    const double *P, const double *B, const double *grad, double ti, double tj,
                    double *c, orc_counters *cnt) {
  const double gam = p->gamma;
  for (int k = 0; k < 5; ++k) c[k] = 0.0;
  double d[3];
  separation(p, x, y, z, i, j, d);
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == 0.0) return 0; /* coincident particles exchange nothing (reading) */
  double r = sqrt(r2);
  /* Face vector A_ij = V_i omega_j B_i mu(x_i,x_j) - V_j omega_i B_j mu(x_j,x_i)
   * with omega = V and mu(a, b) = (b - a) W(|b - a|, H_a): it points from i to j. */
  double bi[6], bj[6];
  for (int k = 0; k < 6; ++k) {
    bi[k] = B[(int64_t)k * n + i];
    bj[k] = B[(int64_t)k * n + j];
  }
  double Bd_i[3], Bd_j[3];
  sym_mul(bi, d, Bd_i);
  sym_mul(bj, d, Bd_j);
  double Wi = orc_kernel_W(r, H[i]), Wj = orc_kernel_W(r, H[j]);
  double A[3];
  for (int k = 0; k < 3; ++k) A[k] = V[i] * V[j] * (Wi * Bd_i[k] + Wj * Bd_j[k]);
  double Amag = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
  if (Amag == 0.0) return 0;
  double nv[3] = {A[0] / Amag, A[1] / Amag, A[2] / Amag};

  double qi[NQ] = {rho[i], vx[i], vy[i], vz[i], P[i]};
  double qj[NQ] = {rho[j], vx[j], vy[j], vz[j], P[j]};
  double gi[NQ][3], gj[NQ][3];
  for (int q = 0; q < NQ; ++q)
    for (int k = 0; k < 3; ++k) {
      gi[q][k] = grad[(int64_t)(3 * q + k) * n + i];
      gj[q][k] = grad[(int64_t)(3 * q + k) * n + j];
    }
  /* Half-step time extrapolation (sec. 2.3.4).  reading: the Lagrangian
   * primitive equations, drho/dt = -rho div v, dv/dt = -grad P / rho,
   * dP/dt = -gamma P div v, with the limited gradients. */
  double qpi[NQ], qpj[NQ];
  {
    double dvi = gi[Q_VX][0] + gi[Q_VY][1] + gi[Q_VZ][2];
    double dvj = gj[Q_VX][0] + gj[Q_VY][1] + gj[Q_VZ][2];
    qpi[Q_RHO] = qi[Q_RHO] - ti * qi[Q_RHO] * dvi;
    qpj[Q_RHO] = qj[Q_RHO] - tj * qj[Q_RHO] * dvj;
    for (int k = 0; k < 3; ++k) {
      qpi[Q_VX + k] = qi[Q_VX + k] - ti * gi[Q_P][k] / qi[Q_RHO];
      qpj[Q_VX + k] = qj[Q_VX + k] - tj * gj[Q_P][k] / qj[Q_RHO];
    }
    qpi[Q_P] = qi[Q_P] - ti * gam * qi[Q_P] * dvi;
    qpj[Q_P] = qj[Q_P] - tj * gam * qj[Q_P] * dvj;
  }
  /* Spatial extrapolation to the mid-point face (sec. 2.3.6), primitives. */
  double qL[NQ], qR[NQ];
  for (int q = 0; q < NQ; ++q) {
    qL[q] = qpi[q] + 0.5 * (gi[q][0] * d[0] + gi[q][1] * d[1] + gi[q][2] * d[2]);
    qR[q] = qpj[q] - 0.5 * (gj[q][0] * d[0] + gj[q][1] * d[1] + gj[q][2] * d[2]);
  }
  if (p->limiter & 2) {
    for (int q = 0; q < NQ; ++q) {
      qL[q] = orc_pair_limit(qL[q], qi[q], qj[q], p->psi1, p->psi2);
      qR[q] = orc_pair_limit(qR[q], qj[q], qi[q], p->psi1, p->psi2);
    }
  }
  /* reading: a non-positive reconstructed density or pressure falls back to
   * the first-order (particle) states for this face */
  if (!(qL[Q_RHO] > 0.0 && qR[Q_RHO] > 0.0 && qL[Q_P] > 0.0 && qR[Q_P] > 0.0)) {
    for (int q = 0; q < NQ; ++q) {
      qL[q] = qi[q];
      qR[q] = qj[q];
    }
    if (cnt) cnt->positivity++;
  }
  /* Boost into the frame of the face, v_frame = (v_i + v_j)/2, and project on
   * the face normal (sec. 2.3.3).  reading: v_i and v_j at the half step (the
   * predicted velocities above), the time the fluxes stand for (eq.
   * hydro_discr); with the start-of-step velocities the MFV sound wave
   * (sec. 3.1.1) converges only at first order. */
  double vf[3] = {0.5 * (qpi[Q_VX] + qpj[Q_VX]), 0.5 * (qpi[Q_VY] + qpj[Q_VY]),
                  0.5 * (qpi[Q_VZ] + qpj[Q_VZ])};
  double wL[3], wR[3];
  for (int k = 0; k < 3; ++k) {
    wL[k] = qL[Q_VX + k] - vf[k];
    wR[k] = qR[Q_VX + k] - vf[k];
  }
  double uL = wL[0] * nv[0] + wL[1] * nv[1] + wL[2] * nv[2];
  double uR = wR[0] * nv[0] + wR[1] * nv[1] + wR[2] * nv[2];
  double ps, us;
  int iters;
  int st = orc_riemann(gam, qL[Q_RHO], uL, qL[Q_P], qR[Q_RHO], uR, qR[Q_P], p->riemann_tol,
                       p->riemann_maxit, &ps, &us, &iters);
  if (cnt) cnt->riemann_iters += iters;
  if (st == 1) {
    if (cnt) cnt->vacuum++;
    return 0;
  }
  if (st == 2 && cnt) cnt->riemann_maxit++;
  double vfn = vf[0] * nv[0] + vf[1] * nv[1] + vf[2] * nv[2];
  double F[5];
  if (p->scheme == 1) {
    /* MFM: the face moves with the contact, so no mass crosses it */
    F[0] = 0.0;
    for (int k = 0; k < 3; ++k) F[1 + k] = ps * nv[k];
    F[4] = ps * (us + vfn);
  } else {
    /* MFV: the face moves with v_frame; the Riemann solution is sampled on the
     * face (xi = 0).  reading: the transverse velocity is taken from the side
     * the contact leaves behind (left when u* >= 0). */
    double rf, uf, pf;
    orc_riemann_sample(gam, qL[Q_RHO], uL, qL[Q_P], qR[Q_RHO], uR, qR[Q_P], ps, us, 0.0, &rf,
                       &uf, &pf);
    const double *wu = (us >= 0.0) ? wL : wR;
    double wun = wu[0] * nv[0] + wu[1] * nv[1] + wu[2] * nv[2];
    double vfa[3];
    for (int k = 0; k < 3; ++k) vfa[k] = uf * nv[k] + (wu[k] - wun * nv[k]);
    double v2 = vfa[0] * vfa[0] + vfa[1] * vfa[1] + vfa[2] * vfa[2];
    double Fm = rf * uf;
    double Fp[3];
    for (int k = 0; k < 3; ++k) Fp[k] = Fm * vfa[k] + pf * nv[k];
    double FE = uf * (pf / (gam - 1.0) + 0.5 * rf * v2 + pf);
    /* back to the lab frame */
    double vf2 = vf[0] * vf[0] + vf[1] * vf[1] + vf[2] * vf[2];
    F[0] = Fm;
    for (int k = 0; k < 3; ++k) F[1 + k] = Fp[k] + vf[k] * Fm;
    F[4] = FE + (vf[0] * Fp[0] + vf[1] * Fp[1] + vf[2] * Fp[2]) + 0.5 * vf2 * Fm;
  }
  for (int k = 0; k < 5; ++k) c[k] = Amag * F[k];
  return 0;
}

int orc_face(const orc_params *p, int64_t n, int64_t i, int64_t j, const double *x,
             const double *y, const double *z, const double *H, const double *V,
             const double *rho, const double *vx, const double *vy, const double *vz,
             const double *P, const double *B, const double *grad, double dt, double *c,
             orc_counters *cnt) {
  /* a global step: both sides to the half step */
  return face_tau(p, n, i, j, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, 0.5 * dt, 0.5 * dt, c,
                  cnt);
}

int orc_face_list(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *H, int64_t *nf_out, int64_t **fa_out,
                  int64_t **fb_out) {
  if (!p || n <= 0 || !nf_out || !fa_out || !fb_out) return -1;
  int64_t *start;
  int32_t *idx;
  if (build_lists(p, n, x, y, z, H, &start, &idx)) return -2;
  /* Unordered pairs with r_ij < max(H_i, H_j): take {i, j} from i's list when
   * j > i, or when i is not in j's list (r_ij >= H_j). */
  int64_t *fcount = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    int64_t cc = 0;
    for (int64_t k = start[i]; k < start[i + 1]; ++k) {
      int64_t j = idx[k];
      if (j == i) continue;
      double d[3];
      separation(p, x, y, z, i, j, d);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (j > i || !(r2 < H[j] * H[j])) cc++;
    }
    fcount[i + 1] = cc;
  }
  for (int64_t i = 0; i < n; ++i) fcount[i + 1] += fcount[i];
  int64_t nf = fcount[n];
  int64_t *fa = (int64_t *)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(int64_t));
  int64_t *fb = (int64_t *)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    int64_t f = fcount[i];
    for (int64_t k = start[i]; k < start[i + 1]; ++k) {
      int64_t j = idx[k];
      if (j == i) continue;
      double d[3];
      separation(p, x, y, z, i, j, d);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (j > i || !(r2 < H[j] * H[j])) {
        fa[f] = i < j ? i : j; /* left state: the lower index */
        fb[f] = i < j ? j : i;
        f++;
      }
    }
  }
  free(start);
  free(idx);
  free(fcount);
  *nf_out = nf;
  *fa_out = fa;
  *fb_out = fb;
  return 0;
}

int orc_face_list_copy(const orc_params *p, int64_t n, const double *x, const double *y,
                       const double *z, const double *H, int64_t cap, int64_t *fa,
                       int64_t *fb, int64_t *nf_out) {
  int64_t nf, *a, *b;
  int rc = orc_face_list(p, n, x, y, z, H, &nf, &a, &b);
  if (rc) return rc;
  *nf_out = nf;
  if (fa && fb)
    for (int64_t f = 0; f < nf && f < cap; ++f) {
      fa[f] = a[f];
      fb[f] = b[f];
    }
  free(a);
  free(b);
  return 0;
}

int orc_fluxes(const orc_params *p, int64_t n, const double *x, const double *y,
               const double *z, const double *H, const double *V, const double *rho,
               const double *vx, const double *vy, const double *vz, const double *P,
               const double *B, const double *grad, double dt, double *dQ, double *scale,
               orc_counters *cnt) {
  return orc_fluxes_src(p, n, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt, 1.0, dQ, scale,
                        NULL, cnt);
}

int orc_fluxes_src(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *H, const double *V, const double *rho,
                   const double *vx, const double *vy, const double *vz, const double *P,
                   const double *B, const double *grad, double dt, double inv_a, double *dQ,
                   double *scale, double *gwork, orc_counters *cnt) {
  if (!p || n <= 0) return -1;
  int64_t nf, *fa, *fb;
  int rc = orc_face_list(p, n, x, y, z, H, &nf, &fa, &fb);
  if (rc) return rc;
  double *fc = (double *)malloc((size_t)(nf > 0 ? nf : 1) * 5 * sizeof(double));
  const double dte = dt * inv_a;
  /* Each face once; counters are per-thread then summed. */
  int64_t iters = 0, vac = 0, pos = 0, mx = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : iters, vac, pos, mx)
  for (int64_t f = 0; f < nf; ++f) {
    orc_counters local;
    memset(&local, 0, sizeof(local));
    orc_face(p, n, fa[f], fb[f], x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dte, fc + 5 * f,
             &local);
    iters += local.riemann_iters;
    vac += local.vacuum;
    pos += local.positivity;
    mx += local.riemann_maxit;
  }
  /* eq. hydro_discr: U_i <- U_i - dt sum_j F_ij A_ij, applied as -c to i and
   * +c to j so that the pair is exactly antisymmetric.  In comoving
   * coordinates every spatial derivative carries 1/a (sec. 2.3.9): the
   * fluxes, and (reading) the gradients of the half-step predictor, which
   * the faces above were given with dt / a. */
  for (int64_t k = 0; k < 5 * n; ++k) {
    dQ[k] = 0.0;
    scale[k] = 0.0;
  }
  if (gwork)
    for (int64_t k = 0; k < 3 * n; ++k) gwork[k] = 0.0;
  for (int64_t f = 0; f < nf; ++f) {
    int64_t a = fa[f], b = fb[f];
    for (int k = 0; k < 5; ++k) {
      double v = dte * fc[5 * f + k];
      dQ[(int64_t)k * n + a] -= v;
      dQ[(int64_t)k * n + b] += v;
      scale[(int64_t)k * n + a] += fabs(v);
      scale[(int64_t)k * n + b] += fabs(v);
    }
    if (gwork) {
      /* eq. gravity_source: the mass dm that goes from a to b crosses
       * x_b - x_a; each side is credited half of the work a.dm (x_b - x_a)
       * with its own acceleration, so both add dm (x_b - x_a) */
      double d[3];
      separation(p, x, y, z, a, b, d);
      double dm = dte * fc[5 * f];
      for (int k = 0; k < 3; ++k) {
        gwork[(int64_t)k * n + a] += dm * d[k];
        gwork[(int64_t)k * n + b] += dm * d[k];
      }
    }
  }
  free(fa);
  free(fb);
  free(fc);
  cnt->faces += nf;
  cnt->riemann_iters += iters;
  cnt->vacuum += vac;
  cnt->positivity += pos;
  cnt->riemann_maxit += mx;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Close of the step                                                         */
/* ------------------------------------------------------------------------ */
int orc_update(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
               double *vx, double *vy, double *vz, double *E, double *U, const double *dQ,
               double dt, orc_counters *cnt) {
  return orc_update_src(p, n, x, y, z, m, vx, vy, vz, E, U, dQ, dt, NULL, NULL, NULL, NULL, NULL,
                        cnt);
}

/* The implicit Hubble-source update of sec. 2.3.9:
 * X^{n+1} = (X~ - eta dt H^n X^n) / (1 + eta dt H^{n+1}). */
static double hubble(double xt, double x0, double eta, double dt, double hn, double hn1) {
  return (xt - eta * dt * hn * x0) / (1.0 + eta * dt * hn1);
}

/* The close of the step for particle i over its step dt: the conserved
 * update, the source terms, the pressure switch and the drift (x, v, E, U and
 * m in place).  dQ holds its summed flux contributions at dQ[k n + i]. */
typedef struct {
  int64_t neg, guard;
} close_counts;

static void close_one(const orc_params *p, int64_t n, int64_t i, double *const pos[3], double *m,
                      double *vx, double *vy, double *vz, double *E, double *U, const double *dQ,
                      double dt, const orc_sources *src, const double *gwork,
                      const double *ekin_max, const double *H, close_counts *cc) {
  const double gam = p->gamma;
  const double *acc = src ? src->accel : NULL;
  const double inv_a = src ? src->inv_a : 1.0;
  const double hn = src ? src->hubble_n : 0.0, hn1 = src ? src->hubble_np1 : 0.0;
  const int comoving = hn != 0.0 || hn1 != 0.0;
  /* reading: eta of each equation from its source term as printed, with
   * u-hat = u and p-hat = p a^3: momentum -H P (eta 1/2); total energy
   * -H (rho v^2 + 3 p) = -2 H E for gamma = 5/3 (eta 1); internal energy
   * -3 H (gamma - 1) U and the entropy of a comoving adiabat likewise
   * (eta 3 (gamma - 1) / 2, which is 1 for gamma = 5/3) */
  const double eta_u = 1.5 * (gam - 1.0);
  {
    double dm = dQ[i], dp[3] = {dQ[n + i], dQ[2 * n + i], dQ[3 * n + i]}, dE = dQ[4 * n + i];
    double v0[3] = {vx[i], vy[i], vz[i]};
    /* eq. internal_energy_integration with the start-of-step velocity (reading) */
    double v0sq = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double dU = dE - (v0[0] * dp[0] + v0[1] * dp[1] + v0[2] * dp[2]) + 0.5 * v0sq * dm;
    double m1 = m[i] + dm;
    if (!(m1 > 0.0)) cc->neg++; /* MFV mass depletion is counted, not clamped */
    double p0[3] = {m[i] * v0[0], m[i] * v0[1], m[i] * v0[2]};
    double p1[3] = {p0[0] + dp[0], p0[1] + dp[1], p0[2] + dp[2]};
    double E1 = E[i] + dE;
    double U1 = U[i] + dU;
    double amag = 0.0;
    if (acc) {
      /* gravity, eq. gravity_source integrated by eq. source_term_discr:
       * S = (0, m a, P.a + W/dt) at the start of the step and at the hydro
       * update U~, with W = 1/2 a . sum_j dm_ij r_ij over the step; the
       * acceleration is the caller's, the same at both ends (reading) */
      double a3[3] = {acc[i], acc[n + i], acc[2 * n + i]};
      amag = sqrt(a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2]);
      double work = 0.0;
      if (gwork)
        work = 0.5 * (a3[0] * gwork[i] + a3[1] * gwork[n + i] + a3[2] * gwork[2 * n + i]);
      double pa = 0.5 * dt * ((p0[0] + p1[0]) * a3[0] + (p0[1] + p1[1]) * a3[1] +
                              (p0[2] + p1[2]) * a3[2]);
      for (int k = 0; k < 3; ++k) p1[k] += 0.5 * dt * (m[i] + m1) * a3[k];
      E1 += pa + work;
    }
    if (comoving) {
      for (int k = 0; k < 3; ++k) p1[k] = hubble(p1[k], p0[k], 0.5, dt, hn, hn1);
      E1 = hubble(E1, E[i], 1.0, dt, hn, hn1);
      U1 = hubble(U1, U[i], eta_u, dt, hn, hn1);
      if (src->S) src->S[i] = hubble(src->S[i], src->S[i], eta_u, dt, hn, hn1);
    }
    double v1[3] = {p1[0] / m1, p1[1] / m1, p1[2] / m1};
    /* Pressure switch (sec. 2.3.7).  reading: the test of criterion (i) is
     * made on the internal energy the total energy gives, E - E_kin >
     * alpha_1 (E_grav + E_kin) (the dual-energy test of the method the
     * section cites).  Tested on the integrated U instead, a particle whose
     * momentum changes by more than its integrated internal energy allows
     * (|dP|^2 / 2m > U) is handed a negative E - E_kin, hence a negative
     * pressure.  Criterion (ii), when the entropy switch is on: the flow is
     * cold and smooth, U < alpha_2 (E_kin^max + U) or U < alpha_3 E_grav,
     * and the next density pass takes the pressure from the entropy.
     * Otherwise (iii) the integrated U is kept. */
    double ekin = (p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2]) / (2.0 * m1);
    double egrav = (acc && H) ? m1 * amag * H[i] : 0.0;
    int mode = 0;
    if (E1 - ekin > p->alpha1 * (egrav + ekin)) {
      U1 = E1 - ekin;
    } else if (p->entropy_switch && src && src->S && ekin_max &&
               (U1 < p->alpha2 * (ekin_max[i] + U1) || U1 < p->alpha3 * egrav)) {
      mode = 1;
    }
    if (src && src->emode) src->emode[i] = mode;
    /* reading: where the kinetic energy dominates, dE ~ v.dP and the
     * integrated U can be driven through zero by that noise (the section
     * names the regime); the internal energy then keeps its value from the
     * start of the step (counted), so the pressure stays positive. */
    if (!(U1 > 0.0)) {
      U1 = U[i];
      cc->guard++;
    }
    /* reading: drift with the mean of the old and new velocities (comoving:
     * dx/dt = v / a), periodic wrap */
    for (int k = 0; k < 3; ++k) {
      double xn = pos[k][i] + dt * inv_a * 0.5 * (v0[k] + v1[k]);
      double L = p->box[k];
      if (L > 0.0) {
        if (xn < 0.0) xn += L;
        if (xn >= L) xn -= L;
      }
      pos[k][i] = xn;
    }
    m[i] = m1;
    vx[i] = v1[0];
    vy[i] = v1[1];
    vz[i] = v1[2];
    E[i] = E1;
    U[i] = U1;
  }
}

int orc_update_src(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                   double *vx, double *vy, double *vz, double *E, double *U, const double *dQ,
                   double dt, const orc_sources *src, const double *gwork,
                   const double *ekin_max, const double *V, const double *H,
                   orc_counters *cnt) {
  if (!p || n <= 0) return -1;
  double *const pos[3] = {x, y, z};
  close_counts cc = {0, 0};
  for (int64_t i = 0; i < n; ++i)
    close_one(p, n, i, pos, m, vx, vy, vz, E, U, dQ, dt, src, gwork, ekin_max, H, &cc);
  (void)V;
  cnt->neg_mass += cc.neg;
  cnt->u_guard += cc.guard;
  return 0;
}

int orc_ekin_max(const orc_params *p, int64_t n, const double *x, const double *y,
                 const double *z, const double *H, const double *m, const double *vx,
                 const double *vy, const double *vz, double *ekin_max) {
  if (!p || n <= 0 || !ekin_max) return -1;
  int64_t *start;
  int32_t *idx;
  if (build_lists(p, n, x, y, z, H, &start, &idx)) return -2;
  for (int64_t i = 0; i < n; ++i) {
    double e = 0.0;
    for (int64_t k = start[i]; k < start[i + 1]; ++k) {
      int64_t j = idx[k];
      if (j == i) continue;
      double d0 = vx[j] - vx[i], d1 = vy[j] - vy[i], d2 = vz[j] - vz[i];
      double ek = 0.5 * m[i] * (d0 * d0 + d1 * d1 + d2 * d2);
      if (ek > e) e = ek;
    }
    ekin_max[i] = e;
  }
  free(start);
  free(idx);
  return 0;
}

int orc_entropy_pressure(const orc_params *p, int64_t n, const double *m, const double *V,
                         double *U, double *S, const int32_t *emode) {
  if (!p || n <= 0 || !m || !V || !U || !S) return -1;
  const double gam = p->gamma;
  for (int64_t i = 0; i < n; ++i) {
    double rho = m[i] / V[i];
    if (emode && emode[i]) {
      /* p = S omega^-1 rho^(gamma-1) = (S / m) rho^gamma (reading of the
       * printed p = S omega rho^(gamma-1), whose omega is read as omega^-1:
       * with S extensive this is the adiabat P / rho^gamma = S / m) */
      double P = S[i] / m[i] * pow(rho, gam);
      U[i] = P * V[i] / (gam - 1.0);
    } else {
      double P = (gam - 1.0) * U[i] / V[i];
      S[i] = m[i] * P / pow(rho, gam);
    }
  }
  return 0;
}

int orc_step_src(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                 double *vx, double *vy, double *vz, double *E, double *U, double *H,
                 double dt_max, const orc_sources *src, double *dt_out, orc_counters *cnt) {
  if (!p || n <= 0 || !dt_out || !cnt) return -1;
  size_t sz = (size_t)n * sizeof(double);
  double *V = (double *)malloc(sz), *nc0 = (double *)malloc(sz), *nng = (double *)malloc(sz);
  double *rho = (double *)malloc(sz), *P = (double *)malloc(sz), *c = (double *)malloc(sz);
  double *B = (double *)malloc(6 * sz), *grad = (double *)malloc(15 * sz);
  double *alpha = (double *)malloc(5 * sz), *nc = (double *)malloc(sz);
  double *dti = (double *)malloc(sz), *dQ = (double *)malloc(5 * sz);
  double *scale = (double *)malloc(5 * sz), *ekm = (double *)malloc(sz);
  double *gw = (double *)malloc(3 * sz);
  int rc = orc_density(p, n, x, y, z, H, V, nc0, nng, cnt);
  if (!rc && src && src->S) rc = orc_entropy_pressure(p, n, m, V, U, src->S, src->emode);
  if (!rc)
    rc = orc_gradients(p, n, x, y, z, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha, nc, dti,
                       cnt);
  if (!rc && p->entropy_switch) rc = orc_ekin_max(p, n, x, y, z, H, m, vx, vy, vz, ekm);
  double dt = dt_max;
  const int grav_work = src && src->accel && p->scheme == 0;
  if (!rc) {
    for (int64_t i = 0; i < n; ++i)
      if (dti[i] < dt) dt = dti[i];
    rc = orc_fluxes_src(p, n, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt,
                        src ? src->inv_a : 1.0, dQ, scale, grav_work ? gw : NULL, cnt);
  }
  if (!rc)
    rc = orc_update_src(p, n, x, y, z, m, vx, vy, vz, E, U, dQ, dt, src, grav_work ? gw : NULL,
                        p->entropy_switch ? ekm : NULL, V, H, cnt);
  *dt_out = dt;
  free(V); free(nc0); free(nng); free(rho); free(P); free(c); free(B); free(grad);
  free(alpha); free(nc); free(dti); free(dQ); free(scale); free(ekm); free(gw);
  return rc;
}

int orc_step(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
             double *vx, double *vy, double *vz, double *E, double *U, double *H,
             double dt_max, double *dt_out, orc_counters *cnt) {
  if (!p || n <= 0 || !dt_out || !cnt) return -1;
  size_t sz = (size_t)n * sizeof(double);
  double *V = (double *)malloc(sz), *nc0 = (double *)malloc(sz), *nng = (double *)malloc(sz);
  double *rho = (double *)malloc(sz), *P = (double *)malloc(sz), *c = (double *)malloc(sz);
  double *B = (double *)malloc(6 * sz), *grad = (double *)malloc(15 * sz);
  double *alpha = (double *)malloc(5 * sz), *nc = (double *)malloc(sz);
  double *dti = (double *)malloc(sz), *dQ = (double *)malloc(5 * sz);
  double *scale = (double *)malloc(5 * sz);
  int rc = orc_density(p, n, x, y, z, H, V, nc0, nng, cnt);
  if (!rc)
    rc = orc_gradients(p, n, x, y, z, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha, nc, dti,
                       cnt);
  double dt = dt_max;
  if (!rc) {
    for (int64_t i = 0; i < n; ++i)
      if (dti[i] < dt) dt = dti[i];
    rc = orc_fluxes(p, n, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, dt, dQ, scale, cnt);
  }
  if (!rc) rc = orc_update(p, n, x, y, z, m, vx, vy, vz, E, U, dQ, dt, cnt);
  *dt_out = dt;
  free(V); free(nc0); free(nng); free(rho); free(P); free(c); free(B); free(grad);
  free(alpha); free(nc); free(dti); free(dQ); free(scale);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Individual time steps (sec. 2.3.4, last paragraphs; sec. 2.3.10)          */
/* ------------------------------------------------------------------------ */

/* 2^-r dt0, by halving (exact in floating point). */
static double rung_step(double dt0, int r) {
  double s = dt0;
  for (int k = 0; k < r; ++k) s *= 0.5;
  return s;
}

/* The rung of a particle whose own step is dti: the smallest r >= 0 with
 * dti > 2^-r dt0 (sec. 2.3.10), by halving (exact in floating point);
 * ORC_RUNG_MAX + 1 when no rung up to ORC_RUNG_MAX will do. */
static int rung_of(double dti, double dt0) {
  double s = dt0;
  for (int r = 0; r <= ORC_RUNG_MAX; ++r) {
    if (dti > s) return r;
    s *= 0.5;
  }
  return ORC_RUNG_MAX + 1;
}

int orc_rungs(const orc_params *p, int64_t n, const double *x, const double *y,
              const double *z, const double *H, const double *dt_i, double dt0, int32_t *rung) {
  if (!p || n <= 0 || !dt_i || !rung || !(dt0 > 0.0)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    rung[i] = rung_of(dt_i[i], dt0);
    if (rung[i] > ORC_RUNG_MAX) return -3;
  }
  /* The rung limiter (sec. 2.3.10): interacting particles -- the pairs of
   * the flux loop, r < max(H_i, H_j) -- differ by at most two rungs; the
   * lower rung is raised, until no pair violates the bound. */
  int64_t nf, *fa, *fb;
  int rc = orc_face_list(p, n, x, y, z, H, &nf, &fa, &fb);
  if (rc) return rc;
  for (int changed = 1; changed;) {
    changed = 0;
    for (int64_t f = 0; f < nf; ++f) {
      int32_t *ra = rung + fa[f], *rb = rung + fb[f];
      if (*ra < *rb - 2) {
        *ra = *rb - 2;
        changed = 1;
      }
      if (*rb < *ra - 2) {
        *rb = *ra - 2;
        changed = 1;
      }
    }
  }
  free(fa);
  free(fb);
  return 0;
}

/* One base step dt0 on individual power-of-two steps.  reading (sec. 2.3.4,
 * sec. 2.3.10), step by step:
 *   - the rungs are set at the start of the base step, when every particle
 *     is synchronised, from the CFL step (orc_rungs), and kept through it;
 *   - the base step is cut into 2^r_max sub-steps of 2^-r_max dt0; a
 *     particle is active at the sub-steps where its own step starts;
 *   - at each sub-step the density and gradient loops run for the active
 *     particles, at the positions of that time (an inactive particle at its
 *     step-start position plus the elapsed time times its step-start
 *     velocity); an inactive particle keeps its H, V, B and gradients, and
 *     its state (m, v, E, U), from the start of its step;
 *   - every face with an active end is evaluated (sec. 2.3.4, after
 *     Springel 2010) with dt = min(dt_i, dt_j): each side's primitives are
 *     predicted from its step start over the elapsed time plus dt / 2, and
 *     dt A_ij F_ij goes to both particles;
 *   - a particle whose step ends closes it (orc_update's close with its own
 *     step and the contributions summed over it).
 * With every rung equal this is the global step with dt = 2^-r dt0. */
int orc_step_rungs(const orc_params *p, int64_t n, double *x, double *y, double *z, double *m,
                   double *vx, double *vy, double *vz, double *E, double *U, double *H,
                   double dt0, int32_t *rung, int rungs_given, int64_t *nsub_out,
                   orc_counters *cnt) {
  if (!p || n <= 0 || !rung || !nsub_out || !cnt || !(dt0 > 0.0)) return -1;
  if (rungs_given)
    for (int64_t i = 0; i < n; ++i)
      if (rung[i] < 0 || rung[i] > ORC_RUNG_MAX) return -1;
  size_t sz = (size_t)n * sizeof(double);
  double *V = (double *)malloc(sz), *nc0 = (double *)malloc(sz), *nng = (double *)malloc(sz);
  double *rho = (double *)malloc(sz), *P = (double *)malloc(sz), *c = (double *)malloc(sz);
  double *B = (double *)malloc(6 * sz), *grad = (double *)malloc(15 * sz);
  double *alpha = (double *)malloc(5 * sz), *nc = (double *)malloc(sz);
  double *dti = (double *)malloc(sz), *dQ = (double *)calloc(5 * (size_t)n, sizeof(double));
  double *xc = (double *)malloc(sz), *yc = (double *)malloc(sz), *zc = (double *)malloc(sz);
  int64_t *s0 = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  uint8_t *act = (uint8_t *)malloc((size_t)n);
  double *pos[3] = {x, y, z}, *cur[3] = {xc, yc, zc};
  double *const state_pos[3] = {x, y, z};
  int rc = orc_density(p, n, x, y, z, H, V, nc0, nng, cnt);
  if (!rc)
    rc = orc_gradients(p, n, x, y, z, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha, nc, dti,
                       cnt);
  if (!rc && !rungs_given) rc = orc_rungs(p, n, x, y, z, H, dti, dt0, rung);
  int rmax = 0;
  for (int64_t i = 0; !rc && i < n; ++i)
    if (rung[i] > rmax) rmax = rung[i];
  const int64_t nsub = (int64_t)1 << rmax;
  const double delta = rung_step(dt0, rmax);
  close_counts cc = {0, 0};
  for (int64_t k = 0; !rc && k < nsub; ++k) {
    for (int64_t i = 0; i < n; ++i) act[i] = (k % ((int64_t)1 << (rmax - rung[i]))) == 0;
    for (int q = 0; q < 3; ++q)
      for (int64_t i = 0; i < n; ++i) {
        const double *v = q == 0 ? vx : (q == 1 ? vy : vz);
        double xn = pos[q][i];
        if (!act[i]) {
          xn += (double)(k - s0[i]) * delta * v[i];
          const double L = p->box[q];
          if (L > 0.0) {
            if (xn < 0.0) xn += L;
            if (xn >= L) xn -= L;
          }
        }
        cur[q][i] = xn;
      }
    if (k > 0) {
      rc = density_mask(p, n, xc, yc, zc, H, V, nc0, nng, act, cnt);
      if (!rc)
        rc = gradients_mask(p, n, xc, yc, zc, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha,
                            nc, dti, act, cnt);
      if (rc) break;
    }
    int64_t nf, *fa, *fb;
    rc = orc_face_list(p, n, xc, yc, zc, H, &nf, &fa, &fb);
    if (rc) break;
    double *fc = (double *)malloc((size_t)(nf > 0 ? nf : 1) * 6 * sizeof(double));
    int64_t iters = 0, vac = 0, npos = 0, mx = 0, used = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : iters, vac, npos, mx, used)
    for (int64_t f = 0; f < nf; ++f) {
      const int64_t a = fa[f], b = fb[f];
      fc[6 * f + 5] = 0.0;
      if (!act[a] && !act[b]) continue;
      const int rf = rung[a] > rung[b] ? rung[a] : rung[b];
      const double dtf = rung_step(dt0, rf); /* min(dt_a, dt_b) */
      const double ta = (double)(k - s0[a]) * delta + 0.5 * dtf;
      const double tb = (double)(k - s0[b]) * delta + 0.5 * dtf;
      orc_counters local;
      memset(&local, 0, sizeof(local));
      face_tau(p, n, a, b, xc, yc, zc, H, V, rho, vx, vy, vz, P, B, grad, ta, tb, fc + 6 * f,
               &local);
      fc[6 * f + 5] = dtf;
      used++;
      iters += local.riemann_iters;
      vac += local.vacuum;
      npos += local.positivity;
      mx += local.riemann_maxit;
    }
    /* each contribution to both ends, in face order */
    for (int64_t f = 0; f < nf; ++f) {
      const double dtf = fc[6 * f + 5];
      if (dtf == 0.0) continue;
      for (int q = 0; q < 5; ++q) {
        const double v = dtf * fc[6 * f + q];
        dQ[(int64_t)q * n + fa[f]] -= v;
        dQ[(int64_t)q * n + fb[f]] += v;
      }
    }
    free(fa);
    free(fb);
    free(fc);
    cnt->faces += used;
    cnt->riemann_iters += iters;
    cnt->vacuum += vac;
    cnt->positivity += npos;
    cnt->riemann_maxit += mx;
    /* the particles whose step ends now close it */
    for (int64_t i = 0; i < n; ++i) {
      if ((k + 1) % ((int64_t)1 << (rmax - rung[i])) != 0) continue;
      close_one(p, n, i, state_pos, m, vx, vy, vz, E, U, dQ, rung_step(dt0, rung[i]), NULL, NULL,
                NULL, H, &cc);
      for (int q = 0; q < 5; ++q) dQ[(int64_t)q * n + i] = 0.0;
      s0[i] = k + 1;
    }
  }
  cnt->neg_mass += cc.neg;
  cnt->u_guard += cc.guard;
  *nsub_out = rc ? 0 : nsub;
  free(V); free(nc0); free(nng); free(rho); free(P); free(c); free(B); free(grad);
  free(alpha); free(nc); free(dti); free(dQ); free(xc); free(yc); free(zc); free(s0); free(act);
  return rc;
}
