// update.hip -- close of the step (eq. hydro_discr, the internal-energy
// integration and pressure switch of sec. 2.3.7, drift) and the conserved
// totals sum_i (m, m v, E)_i used by the diagnostics.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 1024;

struct UpdateArgs {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz, *m, *E, *U;
  const double *dQ, *dt;
  double box[3];
  double alpha1;
  int64_t *counters;
};

__global__ void __launch_bounds__(BS) update_k(UpdateArgs a) {
  if (a.counters[C_STEP_SKIP]) return;  // the density pass was rejected
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t neg = 0, bad = 0, guard = 0;
  if (i < a.n) {
    const int64_t n = a.n;
    const double dt = a.dt[0];
    const double dm = a.dQ[i], dpx = a.dQ[n + i], dpy = a.dQ[2 * n + i],
                 dpz = a.dQ[3 * n + i], dE = a.dQ[4 * n + i];
    const double v0x = a.vx[i], v0y = a.vy[i], v0z = a.vz[i], m0 = a.m[i];
    const double v0sq = v0x * v0x + v0y * v0y + v0z * v0z;
    // dU = dE - v . dP + v^2/2 dM with the start-of-step velocity
    const double dU = dE - (v0x * dpx + v0y * dpy + v0z * dpz) + 0.5 * v0sq * dm;
    const double m1 = m0 + dm;
    if (!(m1 > 0.0)) neg = 1;
    const double px = m0 * v0x + dpx, py = m0 * v0y + dpy, pz = m0 * v0z + dpz;
    const double v1x = px / m1, v1y = py / m1, v1z = pz / m1;
    const double E1 = a.E[i] + dE;
    double U1 = a.U[i] + dU;
    // dual-energy switch: U from the total energy when E - E_kin is not small
    // against E_kin (the test is made on E - E_kin itself, so the recovered
    // internal energy is positive), else the integrated U
    const double ekin = (px * px + py * py + pz * pz) / (2.0 * m1);
    if (E1 - ekin > a.alpha1 * ekin) U1 = E1 - ekin;
    // where kinetic energy dominates, the noise of dE - v.dP can drive the
    // integrated U through zero: it then keeps its start-of-step value
    if (!(U1 > 0.0)) {
      U1 = a.U[i];
      guard = 1;
    }
    double xn[3] = {a.x[i] + dt * 0.5 * (v0x + v1x), a.y[i] + dt * 0.5 * (v0y + v1y),
                    a.z[i] + dt * 0.5 * (v0z + v1z)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (xn[k] < 0.0) xn[k] += a.box[k];
      if (xn[k] >= a.box[k]) xn[k] -= a.box[k];
    }
    if (!isfinite(E1) || !isfinite(U1) || !isfinite(xn[0] + xn[1] + xn[2])) bad = 1;
    a.x[i] = xn[0];
    a.y[i] = xn[1];
    a.z[i] = xn[2];
    a.m[i] = m1;
    a.vx[i] = v1x;
    a.vy[i] = v1y;
    a.vz[i] = v1z;
    a.E[i] = E1;
    a.U[i] = U1;
  }
  count_add(a.counters + C_NEG_MASS, neg);
  count_add(a.counters + C_NONFINITE, bad);
  count_add(a.counters + C_U_GUARD, guard);
}

// Partial sums of (m, m vx, m vy, m vz, E) per block.
__global__ void conserved_partial_k(int64_t n, const double *__restrict__ m,
                                    const double *__restrict__ vx, const double *__restrict__ vy,
                                    const double *__restrict__ vz, const double *__restrict__ E,
                                    double *partial) {
  __shared__ double s[5][BS / 64];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double mk = m[k];
    acc[0] += mk;
    acc[1] += mk * vx[k];
    acc[2] += mk * vy[k];
    acc[3] += mk * vz[k];
    acc[4] += E[k];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = wave_sum_f64(acc[f]);
    if ((threadIdx.x & 63) == 0) s[f][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double v = 0.0;
    for (int w = 0; w < BS / 64; ++w) v += s[threadIdx.x][w];
    partial[threadIdx.x * RED_BLOCKS + blockIdx.x] = v;
  }
}

__global__ void conserved_final_k(const double *partial, double *out) {
  // one wave per quantity
  const int f = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (f >= 5) return;
  double v = 0.0;
  for (int k = lane; k < RED_BLOCKS; k += 64) v += partial[f * RED_BLOCKS + k];
  v = wave_sum_f64(v);
  if (lane == 0) out[f] = v;
}

}  // namespace

hipError_t launch_update(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  UpdateArgs a;
  a.n = pp->n;
  a.x = pp->x; a.y = pp->y; a.z = pp->z; a.vx = pp->vx; a.vy = pp->vy; a.vz = pp->vz;
  a.m = pp->m; a.E = pp->E; a.U = pp->U;
  a.dQ = pp->dQ;
  a.dt = dt_dev;
  for (int k = 0; k < 3; ++k) a.box[k] = ctx->p.box[k];
  a.alpha1 = ctx->p.alpha1;
  a.counters = ctx->counters;
  update_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_conserved(mfm_ctx *ctx, const mfm_particles *pp) {
  conserved_partial_k<<<RED_BLOCKS, BS, 0, ctx->stream>>>(pp->n, pp->m, pp->vx, pp->vy, pp->vz,
                                                          pp->E, ctx->red);
  conserved_final_k<<<1, 5 * 64, 0, ctx->stream>>>(ctx->red, ctx->scalars + 2);
  return hipGetLastError();
}
