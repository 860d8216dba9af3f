// density.hip -- loop (1) of the scheme: smoothing length and number density
// (sec. 2.3.2 and 2.3.5), plus the one neighbour search of the step.
//
// cand_k: one lane per particle scans the 27 cells around its own (cell side
// >= cell_margin * max H, so every pair closer than the side is found) and
// keeps the candidates with r < side as (index, r^2) in the k-major list
// (list_at), staged through LDS so that HBM sees whole planes.  The list is a
// superset of every neighbour set the step uses:
// the gradient loop filters r < H_i and the flux loop r < max(H_i, H_j).
//
// density_k: each lane solves
//   g(H) = (32/3) sum_j w(r_ij / H) - N_NGB = 0
// ((4 pi / 3) H^3 omega^-1 = N_NGB with omega^-1 = sum_j W(r_ij, H)) by Newton
// steps kept inside a bisection bracket (0, side); each evaluation streams only
// the lane's own r^2 list.  The solve ends on a small Newton step, so H is the
// root to roundoff.  Reaching the side is flagged and the host rebuilds the
// grid with larger cells.  Then the number density, the unweighted E~ of the
// condition-number check (with N_NGB boosts), the primitives and the packed
// 128-byte record the gradient loop gathers.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr double PI = 3.14159265358979323846;

struct CandArgs {
  int64_t n;
  const double4 *pos;
  int max_list;
  int32_t *cand;
  double *cand_r2;
  int32_t *cand_cnt;
  int64_t *counters;
};

// The search runs one wavefront per workgroup.  List entries are appended in
// a per-lane order, so a lane's k-th entry would be a lone 4- and 8-byte store
// into plane k; such scattered partial lines were evicted from L2 and written
// to HBM several times over.  Each lane therefore keeps its newest entries in
// a ring of RING planes in LDS (lane-private columns: no barrier is needed),
// and a plane is written out -- 64 consecutive particles, one coalesced
// store per array -- as soon as every lane of the wave has passed it.  An
// entry more than RING planes ahead of the slowest lane is stored directly; a
// per-lane mask records which ring slots hold entries still to be written.
constexpr int CBS = 64;
constexpr int RING = 16;
constexpr int UNR = 8;  // candidate loads issued together

__global__ void __launch_bounds__(CBS) cand_k(CandArgs a, CellGrid g) {
  __shared__ int32_t s_idx[RING][CBS];
  __shared__ double s_r2[RING][CBS];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * CBS + lane;
  const int64_t n = a.n;
  const bool active = i < n;
  const int cap = a.max_list;
  const double4 pi = a.pos[active ? i : n - 1];
  const int cx = cell_coord(pi.x, g.inv[0], g.nc[0]);
  const int cy = cell_coord(pi.y, g.inv[1], g.nc[1]);
  const int cz = cell_coord(pi.z, g.inv[2], g.nc[2]);
  const double R2 = g.side_min * g.side_min;
  // position inside the own cell in cell units; a neighbour cell whose
  // nearest point is farther than the search radius is skipped (the test is
  // in FP32 with a margin, so it only ever skips cells that hold no candidate)
  const float fx = (float)(pi.x * g.inv[0] - cx), fy = (float)(pi.y * g.inv[1] - cy),
              fz = (float)(pi.z * g.inv[2] - cz);
  const float sx = (float)(1.0 / g.inv[0]), sy = (float)(1.0 / g.inv[1]),
              sz = (float)(1.0 / g.inv[2]);
  const float lim = (float)R2 * 1.0001f;
  int k = 0;          // entries found (may exceed cap: overflow)
  uint32_t held = 0;  // bit s: ring slot s holds an entry not yet written out
  int base = 0;       // planes [0, base) are written out (wave-uniform)
  for (int dz = -1; dz <= 1; ++dz) {
    const float gz = sz * fmaxf(dz > 0 ? 1.0f - fz : (dz < 0 ? fz : 0.0f), 0.0f);
    int zz = cz + dz;
    zz = zz < 0 ? zz + g.nc[2] : (zz >= g.nc[2] ? zz - g.nc[2] : zz);
    for (int dy = -1; dy <= 1; ++dy) {
      const float gy = sy * fmaxf(dy > 0 ? 1.0f - fy : (dy < 0 ? fy : 0.0f), 0.0f);
      int yy = cy + dy;
      yy = yy < 0 ? yy + g.nc[1] : (yy >= g.nc[1] ? yy - g.nc[1] : yy);
      for (int dx = -1; dx <= 1; ++dx) {
        const float gx = sx * fmaxf(dx > 0 ? 1.0f - fx : (dx < 0 ? fx : 0.0f), 0.0f);
        if (active && gx * gx + gy * gy + gz * gz <= lim) {
          int xx = cx + dx;
          xx = xx < 0 ? xx + g.nc[0] : (xx >= g.nc[0] ? xx - g.nc[0] : xx);
          const int2 rg = g.range[morton3(xx, yy, zz)];
          const int jend = rg.x + rg.y;
          // UNR independent loads in flight per lane, then the tests in order
          for (int j0 = rg.x; j0 < jend; j0 += UNR) {
            double4 pj[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) pj[u] = a.pos[j0 + u < jend ? j0 + u : j0];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
              const int j = j0 + u;
              const double ex = min_image(pj[u].x - pi.x, g.box[0], g.half[0]);
              const double ey = min_image(pj[u].y - pi.y, g.box[1], g.half[1]);
              const double ez = min_image(pj[u].z - pi.z, g.box[2], g.half[2]);
              const double r2 = ex * ex + ey * ey + ez * ez;
              if (j < jend && r2 < R2 && j != i) {
                if (k < cap) {
                  if (k < base + RING) {
                    s_idx[k % RING][lane] = j;
                    s_r2[k % RING][lane] = r2;
                    held |= 1u << (k % RING);
                  } else {
                    const int64_t at = list_at(i, k, n);
                    a.cand[at] = j;
                    a.cand_r2[at] = r2;
                  }
                }
                ++k;
              }
            }
          }
        }
        // write out the planes every lane has passed
        int done = wave_min_i32(active ? min(k, cap) : (1 << 30));
        if (done >= (1 << 30)) done = base;
        for (int p = base; p < done; ++p) {
          const uint32_t bit = 1u << (p % RING);
          if (active && (held & bit)) {
            const int64_t at = list_at(i, p, n);
            a.cand[at] = s_idx[p % RING][lane];
            a.cand_r2[at] = s_r2[p % RING][lane];
            held &= ~bit;
          }
        }
        base = done > base ? done : base;
      }
    }
  }
  const int kc = min(k, cap);
  const int last = wave_max_i32(active ? kc : 0);
  for (int p = base; p < last; ++p) {
    const uint32_t bit = 1u << (p % RING);
    if (active && p < kc && (held & bit)) {
      const int64_t at = list_at(i, p, n);
      a.cand[at] = s_idx[p % RING][lane];
      a.cand_r2[at] = s_r2[p % RING][lane];
      held &= ~bit;
    }
  }
  int64_t overflow = 0;
  if (active) {
    overflow = k > cap ? 1 : 0;
    a.cand_cnt[i] = kc;
  }
  count_add(a.counters + C_LIST_OVERFLOW, overflow);
}

struct DensityArgs {
  int64_t n;
  const double4 *pos;
  const double *m, *U, *vx, *vy, *vz;
  double *H, *V, *rho, *P, *c, *ncond;
  double *gin;  // GIN_STRIDE doubles per particle
  const int32_t *cand, *cand_cnt;
  const double *cand_r2;
  int32_t *gl, *gl_cnt;
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

__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(7))) density_k(DensityArgs a, CellGrid g) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = a.n;
  const bool active = i < n;
  int64_t noconv = 0, boosts = 0, fails = 0, overflow = 0;
  int cnt = 0, gc = 0;
  if (active) {
    cnt = a.cand_cnt[i];
    const double cover = g.side_min;
    double h = a.H[i];
    double target = a.n_ngb;
    double winv = 0.0, nc = 1.0, s_last = 1.0;
    for (int b = 0;; ++b) {
      double lo = 0.0, hi = cover;
      if (!(h > lo && h < hi)) h = 0.5 * hi;
      bool conv = false;
      for (int it = 0; it < a.h_maxit; ++it) {
        const double h2 = h * h, ih = 1.0 / h;
        double s = 1.0, ds = 0.0;  // the particle itself: w(0) = 1
        for (int k = 0; k < cnt; ++k) {
          const double r2 = a.cand_r2[list_at(i, k, n)];
          if (r2 < h2) {
            const double q = sqrt(r2) * ih;
            s += spline_w(q);
            ds += spline_qdw(q);
          }
        }
        s_last = s;
        const double gv = (32.0 / 3.0) * s - target;
        const double dg = -(32.0 / 3.0) * ds * ih;
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
      const double4 pi = a.pos[i];
      double ws = 1.0;
      double e[6] = {0, 0, 0, 0, 0, 0};
      // this pass also writes the gather set r < H_i for the gradient loop
      // (rewritten if a boost follows)
      gc = 0;
      for (int k = 0; k < cnt; ++k) {
        const double r2 = a.cand_r2[list_at(i, k, n)];
        if (r2 < h2) {
          const int j = a.cand[list_at(i, k, n)];
          a.gl[list_at(i, gc++, n)] = j;
          const double w = spline_w(sqrt(r2) * ih);
          ws += w;
          if (r2 > 0.0) {
            const double4 pj = a.pos[j];
            const double dx = min_image(pj.x - pi.x, g.box[0], g.half[0]);
            const double dy = min_image(pj.y - pi.y, g.box[1], g.half[1]);
            const double dz = min_image(pj.z - pi.z, g.box[2], g.half[2]);
            e[0] += w * dx * dx;
            e[1] += w * dx * dy;
            e[2] += w * dx * dz;
            e[3] += w * dy * dy;
            e[4] += w * dy * dz;
            e[5] += w * dz * dz;
          }
        }
      }
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
    if (h >= cover * (1.0 - 1e-12)) {
      // the root lies beyond the cell side: this pass is redone on a coarser
      // grid, sized from an estimate of the root (at fixed number density the
      // neighbour number grows as H^3), written as the start value
      ++overflow;
      h = cover * cbrt(target / fmax((32.0 / 3.0) * s_last, 1.0)) * 1.05;
    }
    const double V = 1.0 / winv;
    const double rho = a.m[i] / V;
    const double P = (a.gamma - 1.0) * a.U[i] / V;
    const double cs = sqrt(a.gamma * P / rho);
    a.H[i] = h;
    a.V[i] = V;
    a.rho[i] = rho;
    a.P[i] = P;
    a.c[i] = cs;
    a.ncond[i] = nc;
    const double4 pi = a.pos[i];
    double4 *gr = reinterpret_cast<double4 *>(a.gin + i * GIN_STRIDE);
    gr[0] = make_double4(pi.x, pi.y, pi.z, h);
    gr[1] = make_double4(V, rho, a.vx[i], a.vy[i]);
    gr[2] = make_double4(a.vz[i], P, cs, 0.0);
    float4 *gf = reinterpret_cast<float4 *>(a.gin + i * GIN_STRIDE + GIN_F32);
    gf[0] = make_float4((float)V, (float)rho, (float)a.vx[i], (float)a.vy[i]);
    gf[1] = make_float4((float)a.vz[i], (float)P, (float)cs, 0.0f);
    a.gl_cnt[i] = gc;
  }
  count_add(a.counters + C_PASS_NOCONV, noconv);
  count_add(a.counters + C_PASS_BOOSTS, boosts);
  count_add(a.counters + C_PASS_FAIL, fails);
  count_add(a.counters + C_CELL_OVERFLOW, overflow);
}

}  // namespace

hipError_t launch_candidates(mfm_ctx *ctx, const mfm_particles *pp) {
  CandArgs a;
  a.n = pp->n;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.max_list = ctx->p.max_list;
  a.cand = ctx->cand;
  a.cand_r2 = ctx->cand_r2;
  a.cand_cnt = ctx->cand_cnt;
  a.counters = ctx->counters;
  cand_k<<<blocks_for(pp->n, CBS), CBS, 0, ctx->stream>>>(a, ctx->grid);
  return hipGetLastError();
}

hipError_t launch_density(mfm_ctx *ctx, const mfm_particles *pp) {
  DensityArgs a;
  a.n = pp->n;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.m = pp->m; a.U = pp->U; a.vx = pp->vx; a.vy = pp->vy; a.vz = pp->vz;
  a.H = pp->H; a.V = pp->V; a.rho = pp->rho; a.P = pp->P; a.c = pp->c; a.ncond = pp->ncond;
  a.gin = ctx->gin;
  a.cand = ctx->cand;
  a.cand_cnt = ctx->cand_cnt;
  a.cand_r2 = ctx->cand_r2;
  a.gl = ctx->gl;
  a.gl_cnt = ctx->gl_cnt;
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
