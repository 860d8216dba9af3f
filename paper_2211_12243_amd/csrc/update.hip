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
  double alpha1, alpha2, alpha3;
  int entropy_switch;
  const double *accel;  // 3 n external acceleration (null: none)
  const double *gwork;  // 3 n sum_j dm_ij (x_j - x_i) (null: none)
  const double *ekm;    // E_kin^max (entropy switch)
  const double *H;      // support radii (E_grav = m |a| H)
  double *S;            // entropy (Hubble term)
  int32_t *emode;       // out: 1 where the next density pass takes P from S
  double inv_a, hubble_n, hubble_np1, eta_u;
  int64_t *counters;
  // individual time steps (R.rung null: every particle closes a global step):
  // only the particles whose step ends at this sub-step close it, with their
  // own step and the sums of its contributions, which are then cleared
  Rungs R;
  double *dQw;
};

// X^{n+1} = (X~ - eta dt H^n X^n) / (1 + eta dt H^{n+1}) (sec. 2.3.9)
__device__ __forceinline__ double hubble(double xt, double x0, double eta, double dt, double hn,
                                         double hn1) {
  return (xt - eta * dt * hn * x0) / (1.0 + eta * dt * hn1);
}

__global__ void __launch_bounds__(BS) update_k(UpdateArgs a) {
  if (a.counters[C_STEP_SKIP]) return;  // the density pass was rejected
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t neg = 0, bad = 0, guard = 0;
  bool close = i < a.n;
  double dt = 0.0;
  if (close && a.R.rung) {
    const int r = a.R.rung[i];
    close = (a.R.k + 1) % ((int64_t)1 << (a.R.rmax - r)) == 0;
    dt = rung_step(a.R.dt0, r);
  } else if (close) {
    dt = a.dt[0];
  }
  if (close) {
    const int64_t n = a.n;
    const double dm = a.dQ[i], dpx = a.dQ[n + i], dpy = a.dQ[2 * n + i],
                 dpz = a.dQ[3 * n + i], dE = a.dQ[4 * n + i];
    const double v0x = a.vx[i], v0y = a.vy[i], v0z = a.vz[i], m0 = a.m[i];
    const double v0sq = v0x * v0x + v0y * v0y + v0z * v0z;
    // dU = dE - v . dP + v^2/2 dM with the start-of-step velocity
    const double dU = dE - (v0x * dpx + v0y * dpy + v0z * dpz) + 0.5 * v0sq * dm;
    const double m1 = m0 + dm;
    if (!(m1 > 0.0)) neg = 1;
    const double p0x = m0 * v0x, p0y = m0 * v0y, p0z = m0 * v0z;
    double px = p0x + dpx, py = p0y + dpy, pz = p0z + dpz;
    const double E0 = a.E[i], U0 = a.U[i];
    double E1 = E0 + dE;
    double U1 = U0 + dU;
    double amag = 0.0;
    if (a.accel) {
      // gravity (sec. 2.3.8) by eq. source_term_discr: momentum m a, work P.a
      // at the start and at the hydro update, and the exchanged mass's work
      const double ax = a.accel[i], ay = a.accel[n + i], az = a.accel[2 * n + i];
      amag = sqrt(ax * ax + ay * ay + az * az);
      double work = 0.0;
      if (a.gwork) work = 0.5 * (ax * a.gwork[i] + ay * a.gwork[n + i] + az * a.gwork[2 * n + i]);
      const double pa = 0.5 * dt * ((p0x + px) * ax + (p0y + py) * ay + (p0z + pz) * az);
      const double hm = 0.5 * dt * (m0 + m1);
      px += hm * ax;
      py += hm * ay;
      pz += hm * az;
      E1 += pa + work;
    }
    if (a.hubble_n != 0.0 || a.hubble_np1 != 0.0) {
      const double hn = a.hubble_n, hn1 = a.hubble_np1;
      px = hubble(px, p0x, 0.5, dt, hn, hn1);
      py = hubble(py, p0y, 0.5, dt, hn, hn1);
      pz = hubble(pz, p0z, 0.5, dt, hn, hn1);
      E1 = hubble(E1, E0, 1.0, dt, hn, hn1);
      U1 = hubble(U1, U0, a.eta_u, dt, hn, hn1);
      if (a.S) a.S[i] = hubble(a.S[i], a.S[i], a.eta_u, dt, hn, hn1);
    }
    const double v1x = px / m1, v1y = py / m1, v1z = pz / m1;
    // pressure switch (sec. 2.3.7): U from the total energy when E - E_kin is
    // not small against E_grav + E_kin (the test is made on E - E_kin itself,
    // so the recovered internal energy is positive); else, with the entropy
    // switch, the pressure from the entropy where the flow is cold and
    // smooth; else the integrated U
    const double ekin = (px * px + py * py + pz * pz) / (2.0 * m1);
    const double egrav = a.accel ? m1 * amag * a.H[i] : 0.0;
    int mode = 0;
    if (E1 - ekin > a.alpha1 * (egrav + ekin)) {
      U1 = E1 - ekin;
    } else if (a.entropy_switch &&
               (U1 < a.alpha2 * (a.ekm[i] + U1) || U1 < a.alpha3 * egrav)) {
      mode = 1;
    }
    if (a.emode) a.emode[i] = mode;
    // where kinetic energy dominates, the noise of dE - v.dP can drive the
    // integrated U through zero: it then keeps its start-of-step value
    if (!(U1 > 0.0)) {
      U1 = U0;
      guard = 1;
    }
    const double dtx = dt * a.inv_a;  // comoving: dx/dt = v / a
    double xn[3] = {a.x[i] + dtx * 0.5 * (v0x + v1x), a.y[i] + dtx * 0.5 * (v0y + v1y),
                    a.z[i] + dtx * 0.5 * (v0z + v1z)};
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
    if (a.R.rung) {
#pragma unroll
      for (int q = 0; q < 5; ++q) a.dQw[q * n + i] = 0.0;
      a.R.s0[i] = (int32_t)(a.R.k + 1);
    }
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
  a.alpha2 = ctx->p.alpha2;
  a.alpha3 = ctx->p.alpha3;
  a.entropy_switch = ctx->p.entropy_switch;
  a.accel = pp->accel;
  a.gwork = (pp->accel && ctx->p.scheme == MFM_SCHEME_MFV) ? ctx->gwork : nullptr;
  a.ekm = ctx->ekm;
  a.H = pp->H;
  a.S = ctx->p.entropy_switch ? pp->S : nullptr;
  a.emode = ctx->p.entropy_switch ? pp->emode : nullptr;
  a.inv_a = ctx->inv_a;
  a.hubble_n = ctx->hubble_n;
  a.hubble_np1 = ctx->hubble_np1;
  a.eta_u = 1.5 * (ctx->p.gamma - 1.0);
  a.counters = ctx->counters;
  a.R = ctx->rungs;
  a.dQw = pp->dQ;
  update_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_conserved(mfm_ctx *ctx, const mfm_particles *pp) {
  conserved_partial_k<<<RED_BLOCKS, BS, 0, ctx->stream>>>(pp->n, pp->m, pp->vx, pp->vy, pp->vz,
                                                          pp->E, ctx->red);
  conserved_final_k<<<1, 5 * 64, 0, ctx->stream>>>(ctx->red, ctx->scalars + 2);
  return hipGetLastError();
}
