// gradients.hip -- loops (2) and (4) of the scheme: the renormalised
// (Lanson-Vila) gradients with the conditioned slope limiter (sec. 2.3.3 and
// 2.3.6) and the CFL time step (sec. 2.3.10), then the global minimum step.
//
// One lane per particle over its candidate list.  Each
// neighbour (r < H_i) is gathered as one 128-byte record written by the
// density loop.  Pass one accumulates E_i, the five gradient sums, the
// neighbour extrema and the signal velocity, and records the faces this
// particle will evaluate in the flux loop; B_i = E_i^-1 is the FP64 cofactor
// inverse; pass two finds the extreme face extrapolations for the limiter.
// The particle's flux record (positions, 1/H, V, primitives, 1/rho, B,
// limited gradients: 256 bytes) is written packed.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 1024;
constexpr double PI = 3.14159265358979323846;

struct GradArgs {
  int64_t n;
  const double *gin;
  const double *H;      // converged support radii (SoA: 16 particles per cache line)
  const double4 *pos;   // (x, y, z, 0) per particle
  const int32_t *cand, *cand_cnt;
  const double *cand_r2;
  double *B, *grad, *ncond, *dt_i, *rec;
  int32_t *fslot, *fcnt;
  double box[3], half[3];
  double ncond_max, c_cfl;
  int limiter;
  int64_t *counters;
};

__global__ void __launch_bounds__(BS) gradients_k(GradArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = a.n;
  int64_t pairs = 0, singular = 0;
  if (i < n) {
    const double *gi = a.gin + i * GIN_STRIDE;
    const double xi = gi[GIN_X], yi = gi[GIN_Y], zi = gi[GIN_Z], hi = gi[GIN_H];
    const double h2 = hi * hi, ih = 1.0 / hi, wnorm = 8.0 / (PI * hi * h2);
    const double qi[5] = {gi[GIN_RHO], gi[GIN_VX], gi[GIN_VY], gi[GIN_VZ], gi[GIN_P]};
    const double ci = gi[GIN_C];
    const int b0 = (int)(i / FLUX_BLOCK) * FLUX_BLOCK;
    double e[6] = {0, 0, 0, 0, 0, 0};
    double s[5][3];
    double qmax[5], qmin[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s[q][0] = s[q][1] = s[q][2] = 0.0;
      qmax[q] = qmin[q] = qi[q];
    }
    double vsig = 0.0;
    int nf = 0;
    const int cnt = a.cand_cnt[i];
    for (int k = 0; k < cnt; ++k) {
      const int64_t at = list_at(i, k, n);
      const int j = a.cand[at];
      const double r2 = a.cand_r2[at];
      // faces of the flux loop: r < max(H_i, H_j); one evaluation per face
      // inside a block, one per side across blocks
      const bool gather = r2 < h2;  // j is in the gather set of i (then also a face)
      if ((gather || r2 < a.H[j] * a.H[j]) &&
          ((j < b0 || j >= b0 + FLUX_BLOCK) || emit_face((int)i, j))) {
        a.fslot[list_at(i, nf, n)] = j;
        ++nf;
      }
      if (!gather) continue;
      const double *gj = a.gin + (int64_t)j * GIN_STRIDE;
      ++pairs;
      if (r2 == 0.0) continue;
      const double d0 = min_image(gj[GIN_X] - xi, a.box[0], a.half[0]);
      const double d1 = min_image(gj[GIN_Y] - yi, a.box[1], a.half[1]);
      const double d2 = min_image(gj[GIN_Z] - zi, a.box[2], a.half[2]);
      const double r = sqrt(r2);
      const double wv = gj[GIN_V] * wnorm * spline_w(r * ih);
      e[0] += wv * d0 * d0;
      e[1] += wv * d0 * d1;
      e[2] += wv * d0 * d2;
      e[3] += wv * d1 * d1;
      e[4] += wv * d1 * d2;
      e[5] += wv * d2 * d2;
      const double qj[5] = {gj[GIN_RHO], gj[GIN_VX], gj[GIN_VY], gj[GIN_VZ], gj[GIN_P]};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double df = wv * (qj[q] - qi[q]);
        s[q][0] += df * d0;
        s[q][1] += df * d1;
        s[q][2] += df * d2;
        qmax[q] = fmax(qmax[q], qj[q]);
        qmin[q] = fmin(qmin[q], qj[q]);
      }
      // signal velocity: x_i - x_j = -d
      const double proj =
          -(d0 * (qi[1] - qj[1]) + d1 * (qi[2] - qj[2]) + d2 * (qi[3] - qj[3])) / r;
      vsig = fmax(vsig, ci + gj[GIN_C] - fmin(0.0, proj));
    }
    // B = E^-1 by cofactors
    double cf[6];
    cf[0] = e[3] * e[5] - e[4] * e[4];
    cf[1] = e[2] * e[4] - e[1] * e[5];
    cf[2] = e[1] * e[4] - e[2] * e[3];
    cf[3] = e[0] * e[5] - e[2] * e[2];
    cf[4] = e[1] * e[2] - e[0] * e[4];
    cf[5] = e[0] * e[3] - e[1] * e[1];
    const double det = e[0] * cf[0] + e[1] * cf[1] + e[2] * cf[2];
    if (!(det != 0.0) || !isfinite(det)) ++singular;
    double b[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) b[k] = cf[k] / det;
    double g[5][3];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      g[q][0] = b[0] * s[q][0] + b[1] * s[q][1] + b[2] * s[q][2];
      g[q][1] = b[1] * s[q][0] + b[3] * s[q][1] + b[4] * s[q][2];
      g[q][2] = b[2] * s[q][0] + b[4] * s[q][1] + b[5] * s[q][2];
    }
    const double nb = sqrt(b[0] * b[0] + b[3] * b[3] + b[5] * b[5] +
                           2.0 * (b[1] * b[1] + b[2] * b[2] + b[4] * b[4]));
    const double ne = sqrt(e[0] * e[0] + e[3] * e[3] + e[5] * e[5] +
                           2.0 * (e[1] * e[1] + e[2] * e[2] + e[4] * e[4]));
    const double nc = nb * ne / 3.0;
    double alpha[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
    if (a.limiter & MFM_LIMIT_BJ) {
      double dmax[5] = {0, 0, 0, 0, 0}, dmin[5] = {0, 0, 0, 0, 0};
      for (int k = 0; k < cnt; ++k) {
        const int64_t at = list_at(i, k, n);
        const double r2 = a.cand_r2[at];
        if (!(r2 < h2)) continue;
        const double4 pj = a.pos[a.cand[at]];
        const double d0 = min_image(pj.x - xi, a.box[0], a.half[0]);
        const double d1 = min_image(pj.y - yi, a.box[1], a.half[1]);
        const double d2 = min_image(pj.z - zi, a.box[2], a.half[2]);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const double ex = 0.5 * (g[q][0] * d0 + g[q][1] * d1 + g[q][2] * d2);
          dmax[q] = fmax(dmax[q], ex);
          dmin[q] = fmin(dmin[q], ex);
        }
      }
      double t = (a.ncond_max - nc) / (a.ncond_max - 1.0);
      t = t > 0.0 ? (t < 1.0 ? t : 1.0) : 0.0;
      const double beta = 1.0 + t;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double rp = __builtin_huge_val(), rm = __builtin_huge_val();
        if (dmax[q] > 0.0) rp = (qmax[q] - qi[q]) / dmax[q];
        if (dmin[q] < 0.0) rm = (qi[q] - qmin[q]) / (-dmin[q]);
        alpha[q] = fmin(1.0, beta * fmin(rp, rm));
      }
    }
    double *rec = a.rec + i * R_STRIDE;
    rec[R_X] = xi;
    rec[R_Y] = yi;
    rec[R_Z] = zi;
    rec[R_IH] = ih;
    rec[R_V] = gi[GIN_V];
    rec[R_RHO] = qi[0];
    rec[R_IRHO] = 1.0 / qi[0];
    rec[R_VX] = qi[1];
    rec[R_VY] = qi[2];
    rec[R_VZ] = qi[3];
    rec[R_P] = qi[4];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      a.B[k * n + i] = b[k];
      rec[R_B + k] = b[k];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double v = alpha[q] * g[q][k];
        a.grad[(3 * q + k) * n + i] = v;
        rec[R_G + 3 * q + k] = v;
      }
    a.ncond[i] = nc;
    a.dt_i[i] = vsig > 0.0 ? a.c_cfl * hi / vsig : __builtin_huge_val();
    a.fcnt[i] = nf;
  }
  count_add(a.counters + C_GRAD_PAIRS, pairs);
  count_add(a.counters + C_SINGULAR_E, singular);
}

__global__ void min_partial_k(const double *__restrict__ v, int64_t n, double *partial) {
  __shared__ double s[BS / 64];
  double m = __builtin_huge_val();
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    m = fmin(m, v[k]);
  m = wave_min_f64(m);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BS / 64; ++w) m = fmin(m, s[w]);
    partial[blockIdx.x] = m;
  }
}

__global__ void dt_final_k(const double *partial, int np, double dt_max, double *dt,
                           int64_t *counters) {
  __shared__ double s[BS / 64];
  double m = __builtin_huge_val();
  for (int k = threadIdx.x; k < np; k += blockDim.x) m = fmin(m, partial[k]);
  m = wave_min_f64(m);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BS / 64; ++w) m = fmin(m, s[w]);
    const double v = fmin(dt_max, m);
    if (!(v > 0.0) || !isfinite(v))
      atomicAdd((unsigned long long *)(counters + C_NONFINITE), 1ull);
    dt[0] = v;
  }
}

}  // namespace

hipError_t launch_gradients(mfm_ctx *ctx, const mfm_particles *pp, double dt_max,
                            double *dt_dev) {
  GradArgs a;
  a.n = pp->n;
  a.gin = ctx->gin;
  a.H = pp->H;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.cand = ctx->cand;
  a.cand_cnt = ctx->cand_cnt;
  a.cand_r2 = ctx->cand_r2;
  a.B = pp->B; a.grad = pp->grad; a.ncond = pp->ncond; a.dt_i = pp->dt_i; a.rec = ctx->rec;
  a.fslot = ctx->fslot;
  a.fcnt = ctx->fcnt;
  for (int k = 0; k < 3; ++k) {
    a.box[k] = ctx->p.box[k];
    a.half[k] = 0.5 * ctx->p.box[k];
  }
  a.ncond_max = ctx->p.ncond_max;
  a.c_cfl = ctx->p.c_cfl;
  a.limiter = ctx->p.limiter;
  a.counters = ctx->counters;
  gradients_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
  min_partial_k<<<RED_BLOCKS, BS, 0, ctx->stream>>>(pp->dt_i, pp->n, ctx->red);
  dt_final_k<<<1, BS, 0, ctx->stream>>>(ctx->red, RED_BLOCKS, dt_max, dt_dev, ctx->counters);
  return hipGetLastError();
}
