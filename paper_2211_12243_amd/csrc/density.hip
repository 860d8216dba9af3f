// density.hip -- loop (1) of the scheme: smoothing length and number density
// (sec. 2.3.2 and 2.3.5), plus the one neighbour search of the step.
//
// cand_cell_k: for every particle, the candidates in the 27 cells around its
// own (cell side >= cell_margin * max H, so every pair closer than the side
// is found) with r < side, as (index, r^2) in the k-major list (list_at).
// The list is a superset of every neighbour set the step uses: the density
// loop solves over it, the gradient loop takes r < H_i and the flux loop
// r < max(H_i, H_j).
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
  int64_t ncodes;       // Morton codes of the grid (cell search)
  const double4 *pos;
  int max_list;
  int32_t *cand;
  double *cand_r2;
  int32_t *cand_cnt;
  int64_t *counters;
};

// The neighbour search: one wavefront per cell.  The 27 cells
// around it hold every candidate of every particle of the cell; the lanes load
// those candidates once (coalesced ranges, SLOTS per lane) and keep them in
// registers, then take the cell's particles one at a time: each lane tests
// its candidates against the particle (a uniform load), and the matches are
// compacted with a ballot into that particle's list, staged in LDS.  The lists
// of up to TCH particles leave as k-major planes: each plane of a chunk is a
// run of consecutive particles.  Candidate order is the per-lane search's
// (cells in dz, dy, dx order, particles in index order).  Against one lane
// per particle walking its own 27 cells (measured 3.2 ms at 128^3 against
// 2.4 ms for this form), the candidate positions cross the cache-to-register
// path once per cell instead of once per particle, the particle positions
// arrive by scalar broadcast, and the lists leave HBM-friendly: 2.2 GB
// written instead of 4.9.
constexpr int SLOTS = 6;   // candidates per lane per round: 384 per wavefront
constexpr int TCH = 16;    // particles per staged chunk
constexpr int LCAP = 64;   // list entries per particle staged in LDS (more are stored directly)

__device__ __forceinline__ uint32_t compact_bits3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

// Lane l's value in every lane (a scalar broadcast, no memory traffic).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int2 w = *reinterpret_cast<const int2 *>(&v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(w.x, l);
  r.y = __builtin_amdgcn_readlane(w.y, l);
  return *reinterpret_cast<const double *>(&r);
}

__global__ void __launch_bounds__(64) cand_cell_k(CandArgs a, CellGrid g) {
  __shared__ int32_t s_idx[TCH][LCAP];
  __shared__ double s_r2[TCH][LCAP];
  __shared__ int s_start[27];
  __shared__ int s_pre[28];
  __shared__ int s_cnt[TCH];
  const int lane = threadIdx.x;
  const int64_t n = a.n;
  int64_t overflow = 0;
  const uint32_t code = blockIdx.x;
  const int cx = (int)compact_bits3(code), cy = (int)compact_bits3(code >> 1),
            cz = (int)compact_bits3(code >> 2);
  if (cx >= g.nc[0] || cy >= g.nc[1] || cz >= g.nc[2]) return;
  const int2 own = g.range[code];
  if (own.y == 0) return;
  const int cap = a.max_list;
  // the 27 neighbour ranges in the search order, and their prefix sums
  int cnt27 = 0, st27 = 0;
  if (lane < 27) {
    int zz = cz + lane / 9 - 1, yy = cy + (lane / 3) % 3 - 1, xx = cx + lane % 3 - 1;
    zz = zz < 0 ? zz + g.nc[2] : (zz >= g.nc[2] ? zz - g.nc[2] : zz);
    yy = yy < 0 ? yy + g.nc[1] : (yy >= g.nc[1] ? yy - g.nc[1] : yy);
    xx = xx < 0 ? xx + g.nc[0] : (xx >= g.nc[0] ? xx - g.nc[0] : xx);
    const int2 rg = g.range[morton3(xx, yy, zz)];
    st27 = rg.x;
    cnt27 = rg.y;
  }
  int inc = cnt27;
  for (int o = 1; o < 32; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane < 27) {
    s_start[lane] = st27;
    s_pre[lane + 1] = inc;
  }
  if (lane == 0) s_pre[0] = 0;
  __syncthreads();
  const int C = s_pre[27];
  const double R2 = g.side_min * g.side_min;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int t0 = 0; t0 < own.y; t0 += TCH) {
    const int T = min(TCH, own.y - t0);
    if (lane < TCH) s_cnt[lane] = 0;
    // lane t holds particle t of the chunk; the loop below broadcasts it
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (lane < T) {
      const double4 pt = a.pos[own.x + t0 + lane];
      tx = pt.x; ty = pt.y; tz = pt.z;
    }
    __syncthreads();
    for (int cb = 0; cb < C; cb += 64 * SLOTS) {
      double px[SLOTS], py[SLOTS], pz[SLOTS];
      int jj[SLOTS];
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int c = cb + s * 64 + lane;
        jj[s] = -1;
        px[s] = py[s] = pz[s] = 0.0;
        if (c < C) {
          int lo = 0, hi = 27;  // range r with s_pre[r] <= c < s_pre[r + 1]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pre[mid] <= c) lo = mid; else hi = mid;
          }
          const int j = s_start[lo] + (c - s_pre[lo]);
          const double4 pj = a.pos[j];
          jj[s] = j;
          px[s] = pj.x; py[s] = pj.y; pz[s] = pj.z;
        }
      }
      for (int t = 0; t < T; ++t) {
        const int ti = own.x + t0 + t;
        const double ptx = readlane_f64(tx, t), pty = readlane_f64(ty, t),
                     ptz = readlane_f64(tz, t);
        int base = s_cnt[t];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          bool hit = false;
          double r2 = 0.0;
          if (jj[s] >= 0 && jj[s] != ti) {
            const double ex = min_image(px[s] - ptx, g.box[0], g.half[0]);
            const double ey = min_image(py[s] - pty, g.box[1], g.half[1]);
            const double ez = min_image(pz[s] - ptz, g.box[2], g.half[2]);
            r2 = ex * ex + ey * ey + ez * ez;
            hit = r2 < R2;
          }
          const uint64_t m = __ballot(hit);
          if (hit) {
            const int k = base + __popcll(m & below);
            if (k < LCAP) {
              s_idx[t][k] = jj[s];
              s_r2[t][k] = r2;
            } else if (k < cap) {
              const int64_t at = list_at(ti, k, n);
              a.cand[at] = jj[s];
              a.cand_r2[at] = r2;
            }
          }
          base += __popcll(m);
        }
        if (lane == 0) s_cnt[t] = base;  // read again by this wavefront only: LDS keeps its order
      }
      __syncthreads();
    }
    // the chunk's staged lists, plane by plane: lane -> (plane kk + lane / TCH, particle lane % TCH)
    int mine = lane < T ? min(s_cnt[lane], min(LCAP, cap)) : 0;
    const int kmax = wave_max_i32(mine);
    const int tl = lane % TCH;
    const int lim = tl < T ? min(s_cnt[tl], min(LCAP, cap)) : 0;
    for (int kk = 0; kk < kmax; kk += 64 / TCH) {
      const int k = kk + lane / TCH;
      if (k < lim) {
        const int64_t at = list_at(own.x + t0 + tl, k, n);
        a.cand[at] = s_idx[tl][k];
        a.cand_r2[at] = s_r2[tl][k];
      }
    }
    if (lane < T) {
      const int c = s_cnt[lane];
      a.cand_cnt[own.x + t0 + lane] = min(c, cap);
      overflow += c > cap ? 1 : 0;
    }
    __syncthreads();
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
  a.ncodes = ctx->ncodes;
  cand_cell_k<<<(unsigned)ctx->ncodes, 64, 0, ctx->stream>>>(a, ctx->grid);
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
