// density.hip -- loop (1) of the scheme: smoothing length and number density
// (sec. 2.3.2 and 2.3.5), and the neighbour lists the next two loops read.
//
// One lane per particle.  The lanes of a wavefront are 64 consecutive
// particles of the Z-ordered cell list, so their 27-cell stencils overlap and
// the candidate reads are served from L1/L2.  Each lane solves
//   g(H) = (32/3) sum_j w(r_ij / H) - N_NGB = 0
// ((4 pi / 3) H^3 omega^-1 = N_NGB with omega^-1 = sum_j W(r_ij, H)) by Newton
// steps kept inside a bisection bracket whose upper end is the smallest cell
// side (beyond it the stencil would miss neighbours; reaching it is flagged
// and the host rebuilds the grid).  The solve ends on a small Newton step.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr double PI = 3.14159265358979323846;

// Visit every particle in the 27 cells around (cx, cy, cz).
template <typename F>
__device__ __forceinline__ void for_stencil(const CellGrid &g, int cx, int cy, int cz, F &&f) {
  for (int dz = -1; dz <= 1; ++dz) {
    int zz = cz + dz;
    zz = zz < 0 ? zz + g.nc[2] : (zz >= g.nc[2] ? zz - g.nc[2] : zz);
    for (int dy = -1; dy <= 1; ++dy) {
      int yy = cy + dy;
      yy = yy < 0 ? yy + g.nc[1] : (yy >= g.nc[1] ? yy - g.nc[1] : yy);
      for (int dx = -1; dx <= 1; ++dx) {
        int xx = cx + dx;
        xx = xx < 0 ? xx + g.nc[0] : (xx >= g.nc[0] ? xx - g.nc[0] : xx);
        uint32_t code = morton3(xx, yy, zz);
        int s = g.start[code];
        int e = s + g.count[code];
        for (int j = s; j < e; ++j) f(j);
      }
    }
  }
}

struct DensityArgs {
  int64_t n;
  const double *x, *y, *z, *m, *U;
  double *H, *V, *rho, *P, *c, *ncond;
  double gamma, n_ngb, ncond_max, ngb_boost, h_tol;
  int h_maxit, max_boosts;
  int64_t *counters;
};

__device__ __forceinline__ double frob_sym(const double e[6]) {
  return sqrt(e[0] * e[0] + e[3] * e[3] + e[5] * e[5] +
              2.0 * (e[1] * e[1] + e[2] * e[2] + e[4] * e[4]));
}

// Condition number ||E^-1||_F ||E||_F / 3 of a symmetric 3x3 (infinite when singular).
__device__ double cond3(const double e[6]) {
  double c00 = e[3] * e[5] - e[4] * e[4];
  double c01 = e[2] * e[4] - e[1] * e[5];
  double c02 = e[1] * e[4] - e[2] * e[3];
  double c11 = e[0] * e[5] - e[2] * e[2];
  double c12 = e[1] * e[2] - e[0] * e[4];
  double c22 = e[0] * e[3] - e[1] * e[1];
  double det = e[0] * c00 + e[1] * c01 + e[2] * c02;
  if (!(det != 0.0) || !isfinite(det)) return __builtin_huge_val();
  double b[6] = {c00, c01, c02, c11, c12, c22};
  return frob_sym(b) / fabs(det) * frob_sym(e) / 3.0;
}

__global__ void __launch_bounds__(BS) density_k(DensityArgs a, CellGrid g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < a.n;
  int64_t noconv = 0, boosts = 0, fails = 0, overflow = 0;
  if (active) {
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
    const int cx = cell_coord(xi, g.inv[0], g.nc[0]);
    const int cy = cell_coord(yi, g.inv[1], g.nc[1]);
    const int cz = cell_coord(zi, g.inv[2], g.nc[2]);
    const double cover = g.side_min;
    double h = a.H[i];
    double target = a.n_ngb;
    double winv = 0.0, nc = 1.0;
    for (int b = 0;; ++b) {
      double lo = 0.0, hi = cover;
      if (!(h > lo && h < hi)) h = 0.5 * hi;
      bool conv = false;
      for (int it = 0; it < a.h_maxit; ++it) {
        const double h2 = h * h, ih = 1.0 / h;
        double s = 0.0, ds = 0.0;
        for_stencil(g, cx, cy, cz, [&](int j) {
          double dx = min_image(a.x[j] - xi, g.box[0], g.half[0]);
          double dy = min_image(a.y[j] - yi, g.box[1], g.half[1]);
          double dz = min_image(a.z[j] - zi, g.box[2], g.half[2]);
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < h2) {
            double q = sqrt(r2) * ih;
            s += spline_w(q);
            ds += spline_qdw(q);
          }
        });
        double gv = (32.0 / 3.0) * s - target;
        double dg = -(32.0 / 3.0) * ds * ih;
        if (gv == 0.0) {
          conv = true;
          break;
        }
        if (gv < 0.0)
          lo = h;
        else
          hi = h;
        double hn = (dg > 0.0) ? h - gv / dg : -1.0;
        // stop on a small Newton step only (never on a bisection step): its
        // quadratic convergence leaves H at the root to roundoff
        if (fabs(hn - h) <= a.h_tol * hn) {
          h = hn;
          conv = true;
          break;
        }
        if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
        h = hn;
      }
      if (!conv) ++noconv;
      // number density at the solution and the unweighted E~ of the check
      const double h2 = h * h, ih = 1.0 / h;
      double ws = 0.0;
      double e[6] = {0, 0, 0, 0, 0, 0};
      for_stencil(g, cx, cy, cz, [&](int j) {
        double dx = min_image(a.x[j] - xi, g.box[0], g.half[0]);
        double dy = min_image(a.y[j] - yi, g.box[1], g.half[1]);
        double dz = min_image(a.z[j] - zi, g.box[2], g.half[2]);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < h2) {
          double w = spline_w(sqrt(r2) * ih);
          ws += w;
          if (r2 > 0.0) {
            e[0] += w * dx * dx;
            e[1] += w * dx * dy;
            e[2] += w * dx * dz;
            e[3] += w * dy * dy;
            e[4] += w * dy * dz;
            e[5] += w * dz * dz;
          }
        }
      });
      winv = 8.0 / (PI * h * h2) * ws;
      nc = cond3(e);  // the kernel's normalisation drops out of the condition number
      if (!(nc > a.ncond_max)) break;
      if (b == a.max_boosts) {
        ++fails;
        break;
      }
      target *= a.ngb_boost;
      ++boosts;
    }
    if (h >= cover * (1.0 - 1e-12)) ++overflow;
    const double V = 1.0 / winv;
    const double rho = a.m[i] / V;
    const double P = (a.gamma - 1.0) * a.U[i] / V;
    a.H[i] = h;
    a.V[i] = V;
    a.rho[i] = rho;
    a.P[i] = P;
    a.c[i] = sqrt(a.gamma * P / rho);
    a.ncond[i] = nc;
  }
  count_add(a.counters + C_PASS_NOCONV, noconv);
  count_add(a.counters + C_PASS_BOOSTS, boosts);
  count_add(a.counters + C_PASS_FAIL, fails);
  count_add(a.counters + C_CELL_OVERFLOW, overflow);
}

// Symmetric neighbour lists: j != i with r_ij < max(H_i, H_j).  The gradient
// loop keeps the entries with r_ij < H_i, the flux loop uses them all.
__global__ void __launch_bounds__(BS)
    lists_k(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
            const double *__restrict__ z, const double *__restrict__ H, CellGrid g,
            int max_list, int32_t *__restrict__ list, int32_t *__restrict__ cnt,
            int64_t *counters) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t overflow = 0;
  if (i < n) {
    const double xi = x[i], yi = y[i], zi = z[i], hi = H[i];
    const int cx = cell_coord(xi, g.inv[0], g.nc[0]);
    const int cy = cell_coord(yi, g.inv[1], g.nc[1]);
    const int cz = cell_coord(zi, g.inv[2], g.nc[2]);
    int k = 0;
    for_stencil(g, cx, cy, cz, [&](int j) {
      if (j == i) return;
      double dx = min_image(x[j] - xi, g.box[0], g.half[0]);
      double dy = min_image(y[j] - yi, g.box[1], g.half[1]);
      double dz = min_image(z[j] - zi, g.box[2], g.half[2]);
      double r2 = dx * dx + dy * dy + dz * dz;
      double hm = fmax(hi, H[j]);
      if (r2 < hm * hm) {
        if (k < max_list) list[(int64_t)k * n + i] = j;
        ++k;
      }
    });
    if (k > max_list) {
      overflow = 1;
      k = max_list;
    }
    cnt[i] = k;
  }
  count_add(counters + C_LIST_OVERFLOW, overflow);
}

}  // namespace

hipError_t launch_density(mfm_ctx *ctx, const mfm_particles *pp) {
  DensityArgs a;
  a.n = pp->n;
  a.x = pp->x; a.y = pp->y; a.z = pp->z; a.m = pp->m; a.U = pp->U;
  a.H = pp->H; a.V = pp->V; a.rho = pp->rho; a.P = pp->P; a.c = pp->c; a.ncond = pp->ncond;
  a.gamma = ctx->p.gamma;
  a.n_ngb = ctx->p.n_ngb;
  a.ncond_max = ctx->p.ncond_max;
  a.ngb_boost = ctx->p.ngb_boost;
  a.h_tol = ctx->p.h_tol;
  a.h_maxit = ctx->p.h_maxit;
  a.max_boosts = ctx->p.max_boosts;
  a.counters = ctx->counters;
  density_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a, ctx->grid);
  return hipGetLastError();
}

hipError_t launch_build_lists(mfm_ctx *ctx, const mfm_particles *pp) {
  lists_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(pp->n, pp->x, pp->y, pp->z, pp->H,
                                                          ctx->grid, ctx->p.max_list, ctx->list,
                                                          ctx->list_cnt, ctx->counters);
  return hipGetLastError();
}
