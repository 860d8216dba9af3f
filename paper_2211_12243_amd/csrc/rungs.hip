// rungs.hip -- individual time steps (sec. 2.3.4, last paragraphs; sec.
// 2.3.10): each particle's rung from its CFL step, the limiter that keeps the
// rungs of interacting particles within two of each other, and the start of a
// sub-step (which particles begin a step, where the others are).
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;

// The smallest r >= 0 with dt_i > 2^-r dt0, by halving (exact); a step that
// needs a rung beyond MFM_RUNG_MAX is counted and gets MFM_RUNG_MAX.
__global__ void rungs_from_dt_k(int64_t n, const double *__restrict__ dt_i, double dt0,
                                int32_t *rung, int64_t *counters) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t deep = 0;
  if (i < n) {
    const double d = dt_i[i];
    double s = dt0;
    int r = 0;
    while (!(d > s) && r <= MFM_RUNG_MAX) {
      s *= 0.5;
      ++r;
    }
    if (r > MFM_RUNG_MAX) {
      deep = 1;
      r = MFM_RUNG_MAX;
    }
    rung[i] = r;
  }
  count_add(counters + C_RUNG_DEEP, deep);
}

// One sweep of the rung limiter over the faces of the lists the gradient loop
// built when every particle was active (each pair r < max(H_i, H_j) once):
// the lower rung of a pair more than two apart is raised.  Rungs only grow,
// and never beyond the least solution, so sweeps repeated until none raises
// a rung end at it whatever the order of the updates.
__global__ void rung_limiter_k(int64_t n, const int32_t *__restrict__ fslot,
                               const int32_t *__restrict__ fcnt, const int64_t *lseg,
                               int32_t *rung, int64_t *counters) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t changed = 0;
  if (i < n) {
    const int nf = fcnt[i];
    const int64_t lb = list_base(lseg, i);
    for (int f = 0; f < nf; ++f) {
      const int j = fslot[list_at(lb, f)];
      const int ri = rung[i], rj = rung[j];
      if (ri < rj - 2) {
        atomicMax(rung + i, rj - 2);
        changed = 1;
      } else if (rj < ri - 2) {
        atomicMax(rung + j, ri - 2);
        changed = 1;
      }
    }
  }
  count_add(counters + C_RUNG_CHANGED, changed);
}

// Rungs given by the caller: each must lie in 0 .. MFM_RUNG_MAX.
__global__ void rung_check_k(int64_t n, const int32_t *__restrict__ rung, int64_t *counters) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t bad = 0;
  if (i < n) bad = (rung[i] < 0 || rung[i] > MFM_RUNG_MAX) ? 1 : 0;
  count_add(counters + C_RUNG_DEEP, bad);
}

__global__ void rmax_k(int64_t n, const int32_t *__restrict__ rung, int32_t *out) {
  int m = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = max(m, rung[i]);
  m = wave_max_i32(m);
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

// Sub-step k: which particles begin a step, the time since each particle's
// step began, and the positions of that time in pos4 (a particle in mid-step
// at its step-start position plus the elapsed time times its velocity; its H
// is the one of its last density pass).  The search, the density and
// gradient loops and the flux loop take every position from pos4 on a
// sub-step.
__global__ void substep_begin_k(int64_t n, Rungs R, const double *__restrict__ x,
                                const double *__restrict__ y, const double *__restrict__ z,
                                const double *__restrict__ vx, const double *__restrict__ vy,
                                const double *__restrict__ vz, const double *__restrict__ H,
                                double bx, double by, double bz, uint8_t *act, double *elapsed,
                                double4 *pos4) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = R.rung[i];
  const int64_t period = (int64_t)1 << (R.rmax - r);
  const bool on = R.k % period == 0;
  const double e = (double)(R.k - R.s0[i]) * rung_step(R.dt0, R.rmax);
  act[i] = on ? 1 : 0;
  elapsed[i] = e;
  double p[3] = {x[i], y[i], z[i]};
  const double h = H[i];
  if (!on) {
    const double v[3] = {vx[i], vy[i], vz[i]}, L[3] = {bx, by, bz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double q = p[k] + e * v[k];
      if (q < 0.0) q += L[k];
      if (q >= L[k]) q -= L[k];
      p[k] = q;
    }
  }
  pos4[i] = make_double4(p[0], p[1], p[2], h);
}

}  // namespace

hipError_t launch_rungs_from_dt(mfm_ctx *ctx, const mfm_particles *pp, double dt0) {
  rungs_from_dt_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(pp->n, pp->dt_i, dt0,
                                                                   ctx->rung_w, ctx->counters);
  return hipGetLastError();
}

hipError_t launch_rung_limiter(mfm_ctx *ctx, const mfm_particles *pp) {
  rung_limiter_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(
      pp->n, ctx->fslot, ctx->fcnt, ctx->lseg, const_cast<int32_t *>(ctx->rungs.rung),
      ctx->counters);
  return hipGetLastError();
}

hipError_t launch_rung_check(mfm_ctx *ctx, int64_t n) {
  rung_check_k<<<blocks_for(n, BS), BS, 0, ctx->stream>>>(n, ctx->rungs.rung, ctx->counters);
  return hipGetLastError();
}

hipError_t launch_rmax(mfm_ctx *ctx, int64_t n, int32_t *rmax_dev) {
  hipError_t e = hipMemsetAsync(rmax_dev, 0, sizeof(int32_t), ctx->stream);
  if (e != hipSuccess) return e;
  rmax_k<<<256, BS, 0, ctx->stream>>>(n, ctx->rungs.rung, rmax_dev);
  return hipGetLastError();
}

hipError_t launch_substep_begin(mfm_ctx *ctx, const mfm_particles *pp) {
  substep_begin_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(
      pp->n, ctx->rungs, pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz, pp->H, ctx->p.box[0],
      ctx->p.box[1], ctx->p.box[2], ctx->act_w, ctx->elapsed_w,
      reinterpret_cast<double4 *>(ctx->pos4));
  return hipGetLastError();
}
