// gradients.hip -- loops (2) and (4) of the scheme: the renormalised
// (Lanson-Vila) gradients with the conditioned slope limiter (sec. 2.3.3 and
// 2.3.6) and the CFL time step (sec. 2.3.10), then the global minimum step.
//
// One lane per particle over its neighbour list (k-major layout, so the list
// reads of a wavefront are coalesced).  Pass one accumulates E_i, the five
// gradient sums, the neighbour extrema and the signal velocity; B_i = E_i^-1 is
// the cofactor inverse in FP64; pass two finds the extreme face extrapolations
// for the limiter.  The particle's flux-pass record (positions, primitives, B,
// limited gradients: 256 bytes) is written packed, so the flux loop gathers
// each neighbour with two cache lines instead of thirty scattered ones.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 1024;
constexpr double PI = 3.14159265358979323846;

struct GradArgs {
  int64_t n;
  const double *x, *y, *z, *H, *V, *rho, *vx, *vy, *vz, *P, *c;
  double *B, *grad, *ncond, *dt_i, *rec;
  const int32_t *list, *cnt;
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
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i], hi = a.H[i];
    const double h2 = hi * hi, ih = 1.0 / hi, wnorm = 8.0 / (PI * hi * h2);
    double qi[5] = {a.rho[i], a.vx[i], a.vy[i], a.vz[i], a.P[i]};
    const double ci = a.c[i];
    double e[6] = {0, 0, 0, 0, 0, 0};
    double s[5][3];
    double qmax[5], qmin[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s[q][0] = s[q][1] = s[q][2] = 0.0;
      qmax[q] = qmin[q] = qi[q];
    }
    double vsig = 0.0;
    const int cnt = a.cnt[i];
    for (int k = 0; k < cnt; ++k) {
      const int j = a.list[(int64_t)k * n + i];
      double d0 = min_image(a.x[j] - xi, a.box[0], a.half[0]);
      double d1 = min_image(a.y[j] - yi, a.box[1], a.half[1]);
      double d2 = min_image(a.z[j] - zi, a.box[2], a.half[2]);
      double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      if (!(r2 < h2)) continue;
      ++pairs;
      if (r2 == 0.0) continue;
      double r = sqrt(r2);
      double wv = a.V[j] * wnorm * spline_w(r * ih);
      e[0] += wv * d0 * d0;
      e[1] += wv * d0 * d1;
      e[2] += wv * d0 * d2;
      e[3] += wv * d1 * d1;
      e[4] += wv * d1 * d2;
      e[5] += wv * d2 * d2;
      double qj[5] = {a.rho[j], a.vx[j], a.vy[j], a.vz[j], a.P[j]};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double df = wv * (qj[q] - qi[q]);
        s[q][0] += df * d0;
        s[q][1] += df * d1;
        s[q][2] += df * d2;
        qmax[q] = fmax(qmax[q], qj[q]);
        qmin[q] = fmin(qmin[q], qj[q]);
      }
      // signal velocity: x_i - x_j = -d
      double proj = -(d0 * (qi[1] - qj[1]) + d1 * (qi[2] - qj[2]) + d2 * (qi[3] - qj[3])) / r;
      vsig = fmax(vsig, ci + a.c[j] - fmin(0.0, proj));
    }
    // B = E^-1 by cofactors
    double cf[6];
    cf[0] = e[3] * e[5] - e[4] * e[4];
    cf[1] = e[2] * e[4] - e[1] * e[5];
    cf[2] = e[1] * e[4] - e[2] * e[3];
    cf[3] = e[0] * e[5] - e[2] * e[2];
    cf[4] = e[1] * e[2] - e[0] * e[4];
    cf[5] = e[0] * e[3] - e[1] * e[1];
    double det = e[0] * cf[0] + e[1] * cf[1] + e[2] * cf[2];
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
        const int j = a.list[(int64_t)k * n + i];
        double d0 = min_image(a.x[j] - xi, a.box[0], a.half[0]);
        double d1 = min_image(a.y[j] - yi, a.box[1], a.half[1]);
        double d2 = min_image(a.z[j] - zi, a.box[2], a.half[2]);
        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (!(r2 < h2)) continue;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          double ex = 0.5 * (g[q][0] * d0 + g[q][1] * d1 + g[q][2] * d2);
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
    rec[R_H] = hi;
    rec[R_V] = a.V[i];
#pragma unroll
    for (int q = 0; q < 5; ++q) rec[R_RHO + q] = qi[q];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      a.B[k * n + i] = b[k];
      rec[R_B + k] = b[k];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double v = alpha[q] * g[q][k];
        a.grad[(3 * q + k) * n + i] = v;
        rec[R_G + 3 * q + k] = v;
      }
    rec[R_STRIDE - 1] = 0.0;
    a.ncond[i] = nc;
    a.dt_i[i] = vsig > 0.0 ? a.c_cfl * hi / vsig : __builtin_huge_val();
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
    double v = fmin(dt_max, m);
    if (!(v > 0.0) || !isfinite(v)) atomicAdd((unsigned long long *)(counters + C_NONFINITE), 1ull);
    dt[0] = v;
  }
}

}  // namespace

hipError_t launch_gradients(mfm_ctx *ctx, const mfm_particles *pp, double dt_max,
                            double *dt_dev) {
  GradArgs a;
  a.n = pp->n;
  a.x = pp->x; a.y = pp->y; a.z = pp->z; a.H = pp->H; a.V = pp->V; a.rho = pp->rho;
  a.vx = pp->vx; a.vy = pp->vy; a.vz = pp->vz; a.P = pp->P; a.c = pp->c;
  a.B = pp->B; a.grad = pp->grad; a.ncond = pp->ncond; a.dt_i = pp->dt_i; a.rec = ctx->rec;
  a.list = ctx->list; a.cnt = ctx->list_cnt;
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
