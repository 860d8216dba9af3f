// fluxes.hip -- loop (3) of the scheme: face vector, half-step extrapolation,
// pairwise limiter, exact Riemann solver and MFV/MFM fluxes (sec. 2.3.3, 2.3.4,
// 2.3.6), accumulated antisymmetrically (eq. hydro_discr).
//
// Work split.  A workgroup owns a block of BS consecutive particles of the
// Z-ordered list, one lane each, and an LDS accumulator per particle.  A face
// whose two particles are both in the block is computed once (by the lane the
// symmetric "emit" rule picks) and added to both LDS slots.  A face that crosses
// the block boundary is computed by both blocks, each keeping only its own side:
// the face function always takes the lower slot as the left state, so both
// evaluations are bitwise identical and the pair stays exactly antisymmetric.
// No global atomics: FP64 global atomic adds run at ~23 G/s on this part, far
// too slow for the ~10 per face a scatter would need.
#include "mfm_internal.h"

namespace {

constexpr double PI = 3.14159265358979323846;

struct Gas {
  double gamma, g1, g2, g3, g4, g5, g6, g7, inv_gm1;
};

struct FluxArgs {
  int64_t n;
  const double *rec;
  const int32_t *list, *cnt;
  const double *dt;
  double *dQ;
  double box[3], half[3];
  Gas G;
  double psi1, psi2, rtol;
  int rmaxit, limiter;
  int64_t *counters;
};

// Toro's pressure function of one side and its derivative.
__device__ __forceinline__ void pressure_fn(double p, double rk, double pk, double ck,
                                            const Gas &G, double &f, double &df) {
  if (p <= pk) {
    double pr = p / pk;
    double e = pow(pr, G.g1);
    f = G.g4 * ck * (e - 1.0);
    df = e / (pr * rk * ck);
  } else {
    double A = G.g5 / rk, Bk = G.g6 * pk;
    double q = sqrt(A / (Bk + p));
    f = (p - pk) * q;
    df = q * (1.0 - 0.5 * (p - pk) / (Bk + p));
  }
}

// Exact Riemann solve: 0 converged, 1 vacuum, 2 iteration cap.
__device__ int riemann_solve(const Gas &G, double rL, double uL, double pL, double cL, double rR,
                             double uR, double pR, double cR, double tol, int maxit, double &ps,
                             double &us, int &iters) {
  const double du = uR - uL;
  iters = 0;
  if (G.g4 * (cL + cR) <= du) {
    ps = 0.0;
    us = 0.5 * (uL + uR);
    return 1;
  }
  const double pmin = fmin(pL, pR), pmax = fmax(pL, pR);
  double ppv = 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (cL + cR);
  ppv = fmax(ppv, 0.0);
  double p0;
  if (pmax <= 2.0 * pmin && pmin <= ppv && ppv <= pmax) {
    p0 = ppv;
  } else if (ppv < pmin) {
    double num = cL + cR - G.g7 * du;
    double den = cL / pow(pL, G.g1) + cR / pow(pR, G.g1);
    p0 = pow(num / den, 1.0 / G.g1);
  } else {
    double gL = sqrt(G.g5 / rL / (G.g6 * pL + ppv));
    double gR = sqrt(G.g5 / rR / (G.g6 * pR + ppv));
    p0 = (gL * pL + gR * pR - du) / (gL + gR);
  }
  const double pfloor = 1e-10 * 0.5 * (pL + pR);
  if (!(p0 > pfloor)) p0 = pfloor;
  double p = p0, fL, dfL, fR, dfR;
  int status = 2;
  for (int it = 1; it <= maxit; ++it) {
    pressure_fn(p, rL, pL, cL, G, fL, dfL);
    pressure_fn(p, rR, pR, cR, G, fR, dfR);
    double pn = p - (fL + fR + du) / (dfL + dfR);
    if (pn < 0.0) pn = pfloor;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    iters = it;
    if (change < tol) {
      status = 0;
      break;
    }
  }
  pressure_fn(p, rL, pL, cL, G, fL, dfL);
  pressure_fn(p, rR, pR, cR, G, fR, dfR);
  ps = p;
  us = 0.5 * (uL + uR) + 0.5 * (fR - fL);
  return status;
}

// The exact solution at x/t = 0 in the face frame (Toro's sampling).
__device__ void sample_at_face(const Gas &G, double rL, double uL, double pL, double cL,
                               double rR, double uR, double pR, double cR, double ps, double us,
                               double &rf, double &uf, double &pf) {
  if (0.0 <= us) {
    if (ps <= pL) {
      if (0.0 <= uL - cL) {
        rf = rL; uf = uL; pf = pL;
      } else {
        double t = ps / pL;
        double cml = cL * pow(t, G.g1);
        if (0.0 > us - cml) {
          rf = rL * pow(t, 1.0 / G.gamma); uf = us; pf = ps;
        } else {
          double cc = G.g5 * (cL + G.g7 * uL);
          uf = cc;
          rf = rL * pow(cc / cL, G.g4);
          pf = pL * pow(cc / cL, G.g3);
        }
      }
    } else {
      double pml = ps / pL;
      double sl = uL - cL * sqrt(G.g2 * pml + G.g1);
      if (0.0 <= sl) {
        rf = rL; uf = uL; pf = pL;
      } else {
        rf = rL * (pml + G.g6) / (pml * G.g6 + 1.0); uf = us; pf = ps;
      }
    }
  } else {
    if (ps > pR) {
      double pmr = ps / pR;
      double sr = uR + cR * sqrt(G.g2 * pmr + G.g1);
      if (0.0 >= sr) {
        rf = rR; uf = uR; pf = pR;
      } else {
        rf = rR * (pmr + G.g6) / (pmr * G.g6 + 1.0); uf = us; pf = ps;
      }
    } else {
      if (0.0 >= uR + cR) {
        rf = rR; uf = uR; pf = pR;
      } else {
        double t = ps / pR;
        double cmr = cR * pow(t, G.g1);
        if (0.0 <= us + cmr) {
          rf = rR * pow(t, 1.0 / G.gamma); uf = us; pf = ps;
        } else {
          double cc = G.g5 * (cR - G.g7 * uR);
          uf = -cc;
          rf = rR * pow(cc / cR, G.g4);
          pf = pR * pow(cc / cR, G.g3);
        }
      }
    }
  }
}

// Pairwise limiter of a face value qf extrapolated from the own side (qo)
// towards the other side (qn).
__device__ __forceinline__ double pair_limit(double qf, double qo, double qn, double psi1,
                                             double psi2) {
  if (qo == qn) return qo;
  const double dq = fabs(qo - qn);
  const double d1 = psi1 * dq, d2 = psi2 * dq;
  const double qbar = 0.5 * (qo + qn);
  if (qo < qn) {
    double lower = ((qo - d1) * qo > 0.0) ? qo - d1 : qo / (1.0 + d1 / fabs(qo));
    return fmax(lower, fmin(qbar + d2, qf));
  }
  double upper = ((qo + d1) * qo > 0.0) ? qo + d1 : qo / (1.0 + d1 / fabs(qo));
  return fmin(upper, fmax(qbar - d2, qf));
}

enum { F_VACUUM = 1, F_POSITIVITY = 2, F_MAXIT = 4 };

// Contribution c = |A_ij| F_ij of the face between records Lr (left) and Rr.
template <int SCHEME>
__device__ void face_flux(const double *__restrict__ Lr, const double *__restrict__ Rr,
                          const FluxArgs &a, double dt, double c[5], int &iters, int &flags) {
  const Gas &G = a.G;
  iters = 0;
  flags = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = 0.0;
  double d[3];
  d[0] = min_image(Rr[R_X] - Lr[R_X], a.box[0], a.half[0]);
  d[1] = min_image(Rr[R_Y] - Lr[R_Y], a.box[1], a.half[1]);
  d[2] = min_image(Rr[R_Z] - Lr[R_Z], a.box[2], a.half[2]);
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == 0.0) return;
  const double r = sqrt(r2);
  // A_ij = V_i V_j (W(r, H_i) B_i + W(r, H_j) B_j) d
  const double hL = Lr[R_H], hR = Rr[R_H];
  const double WL = 8.0 / (PI * hL * hL * hL) * spline_w(r / hL);
  const double WR = 8.0 / (PI * hR * hR * hR) * spline_w(r / hR);
  const double *bL = Lr + R_B, *bR = Rr + R_B;
  const double VV = Lr[R_V] * Rr[R_V];
  double A[3];
  A[0] = VV * (WL * (bL[0] * d[0] + bL[1] * d[1] + bL[2] * d[2]) +
               WR * (bR[0] * d[0] + bR[1] * d[1] + bR[2] * d[2]));
  A[1] = VV * (WL * (bL[1] * d[0] + bL[3] * d[1] + bL[4] * d[2]) +
               WR * (bR[1] * d[0] + bR[3] * d[1] + bR[4] * d[2]));
  A[2] = VV * (WL * (bL[2] * d[0] + bL[4] * d[1] + bL[5] * d[2]) +
               WR * (bR[2] * d[0] + bR[4] * d[1] + bR[5] * d[2]));
  const double Am = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
  if (Am == 0.0) return;
  const double nv[3] = {A[0] / Am, A[1] / Am, A[2] / Am};

  double qi[5], qj[5], qL[5], qR[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    qi[q] = Lr[R_RHO + q];
    qj[q] = Rr[R_RHO + q];
  }
  const double *gi = Lr + R_G, *gj = Rr + R_G;
  {
    // half-step Lagrangian predictor plus extrapolation to the mid-point face
    const double hdt = 0.5 * dt;
    const double dvi = gi[3] + gi[7] + gi[11];
    const double dvj = gj[3] + gj[7] + gj[11];
    qL[0] = qi[0] - hdt * qi[0] * dvi;
    qR[0] = qj[0] - hdt * qj[0] * dvj;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qL[1 + k] = qi[1 + k] - hdt * gi[12 + k] / qi[0];
      qR[1 + k] = qj[1 + k] - hdt * gj[12 + k] / qj[0];
    }
    qL[4] = qi[4] - hdt * G.gamma * qi[4] * dvi;
    qR[4] = qj[4] - hdt * G.gamma * qj[4] * dvj;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] += 0.5 * (gi[3 * q] * d[0] + gi[3 * q + 1] * d[1] + gi[3 * q + 2] * d[2]);
      qR[q] -= 0.5 * (gj[3 * q] * d[0] + gj[3 * q + 1] * d[1] + gj[3 * q + 2] * d[2]);
    }
  }
  if (a.limiter & MFM_LIMIT_PAIRWISE) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] = pair_limit(qL[q], qi[q], qj[q], a.psi1, a.psi2);
      qR[q] = pair_limit(qR[q], qj[q], qi[q], a.psi1, a.psi2);
    }
  }
  if (!(qL[0] > 0.0 && qR[0] > 0.0 && qL[4] > 0.0 && qR[4] > 0.0)) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] = qi[q];
      qR[q] = qj[q];
    }
    flags |= F_POSITIVITY;
  }
  const double vf[3] = {0.5 * (qi[1] + qj[1]), 0.5 * (qi[2] + qj[2]), 0.5 * (qi[3] + qj[3])};
  double wL[3], wR[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    wL[k] = qL[1 + k] - vf[k];
    wR[k] = qR[1 + k] - vf[k];
  }
  const double uL = wL[0] * nv[0] + wL[1] * nv[1] + wL[2] * nv[2];
  const double uR = wR[0] * nv[0] + wR[1] * nv[1] + wR[2] * nv[2];
  const double cL = sqrt(G.gamma * qL[4] / qL[0]);
  const double cR = sqrt(G.gamma * qR[4] / qR[0]);
  double ps, us;
  int st = riemann_solve(G, qL[0], uL, qL[4], cL, qR[0], uR, qR[4], cR, a.rtol, a.rmaxit, ps, us,
                         iters);
  if (st == 1) {
    flags |= F_VACUUM;
    return;
  }
  if (st == 2) flags |= F_MAXIT;
  const double vfn = vf[0] * nv[0] + vf[1] * nv[1] + vf[2] * nv[2];
  if (SCHEME == MFM_SCHEME_MFM) {
    c[0] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = Am * ps * nv[k];
    c[4] = Am * ps * (us + vfn);
  } else {
    double rf, uf, pf;
    sample_at_face(G, qL[0], uL, qL[4], cL, qR[0], uR, qR[4], cR, ps, us, rf, uf, pf);
    const double *wu = (us >= 0.0) ? wL : wR;
    const double wun = wu[0] * nv[0] + wu[1] * nv[1] + wu[2] * nv[2];
    double vfa[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) vfa[k] = uf * nv[k] + (wu[k] - wun * nv[k]);
    const double v2 = vfa[0] * vfa[0] + vfa[1] * vfa[1] + vfa[2] * vfa[2];
    const double Fm = rf * uf;
    double Fp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Fp[k] = Fm * vfa[k] + pf * nv[k];
    const double FE = uf * (pf * G.inv_gm1 + 0.5 * rf * v2 + pf);
    const double vf2 = vf[0] * vf[0] + vf[1] * vf[1] + vf[2] * vf[2];
    c[0] = Am * Fm;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = Am * (Fp[k] + vf[k] * Fm);
    c[4] = Am * (FE + (vf[0] * Fp[0] + vf[1] * Fp[1] + vf[2] * Fp[2]) + 0.5 * vf2 * Fm);
  }
}

// Exactly one of emit(i, j), emit(j, i) holds, and about half of any
// particle's in-block faces are its own, whatever its rank in the block.
__device__ __forceinline__ bool emit(int i, int j) { return ((i ^ j) & 1) ? (i < j) : (i > j); }

template <int SCHEME, int BS>
__global__ void __launch_bounds__(BS) fluxes_k(FluxArgs a) {
  __shared__ double acc[5][BS];
  const int64_t n = a.n;
  const int tid = threadIdx.x;
  const int b0 = blockIdx.x * BS;
  const int b1 = (int)min((int64_t)b0 + BS, n);
  const int i = b0 + tid;
#pragma unroll
  for (int f = 0; f < 5; ++f) acc[f][tid] = 0.0;
  __syncthreads();
  double own[5] = {0, 0, 0, 0, 0};
  int64_t nfaces = 0, iters_sum = 0, vac = 0, pos = 0, maxit = 0;
  const double dt = a.dt[0];
  if (i < n) {
    const int cnt = a.cnt[i];
    for (int k = 0; k < cnt; ++k) {
      const int j = a.list[(int64_t)k * n + i];
      const bool inb = (j >= b0) && (j < b1);
      if (inb && !emit(i, j)) continue;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      double c[5];
      int it, fl;
      face_flux<SCHEME>(a.rec + (int64_t)lo * R_STRIDE, a.rec + (int64_t)hi * R_STRIDE, a, dt, c,
                        it, fl);
      const double sgn = (i == lo) ? -1.0 : 1.0;
#pragma unroll
      for (int f = 0; f < 5; ++f) own[f] += sgn * c[f];
      if (inb) {
#pragma unroll
        for (int f = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); f < 5; ++f)
          atomicAdd(&acc[f][j - b0], -sgn * c[f]);
      }
      if (inb || i < j) {
        ++nfaces;
        iters_sum += it;
        vac += (fl & F_VACUUM) ? 1 : 0;
        pos += (fl & F_POSITIVITY) ? 1 : 0;
        maxit += (fl & F_MAXIT) ? 1 : 0;
      }
    }
  }
  __syncthreads();
  if (i < n) {
#pragma unroll
    for (int f = 0; f < 5; ++f) a.dQ[(int64_t)f * n + i] = dt * (own[f] + acc[f][tid]);
  }
  count_add(a.counters + C_FACES, nfaces);
  count_add(a.counters + C_RIEMANN_ITERS, iters_sum);
  count_add(a.counters + C_VACUUM, vac);
  count_add(a.counters + C_POSITIVITY, pos);
  count_add(a.counters + C_RIEMANN_MAXIT, maxit);
}

constexpr int FLUX_BS = 256;

}  // namespace

hipError_t launch_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  FluxArgs a;
  a.n = pp->n;
  a.rec = ctx->rec;
  a.list = ctx->list;
  a.cnt = ctx->list_cnt;
  a.dt = dt_dev;
  a.dQ = pp->dQ;
  for (int k = 0; k < 3; ++k) {
    a.box[k] = ctx->p.box[k];
    a.half[k] = 0.5 * ctx->p.box[k];
  }
  const double g = ctx->p.gamma;
  a.G.gamma = g;
  a.G.g1 = (g - 1.0) / (2.0 * g);
  a.G.g2 = (g + 1.0) / (2.0 * g);
  a.G.g3 = 2.0 * g / (g - 1.0);
  a.G.g4 = 2.0 / (g - 1.0);
  a.G.g5 = 2.0 / (g + 1.0);
  a.G.g6 = (g - 1.0) / (g + 1.0);
  a.G.g7 = 0.5 * (g - 1.0);
  a.G.inv_gm1 = 1.0 / (g - 1.0);
  a.psi1 = ctx->p.psi1;
  a.psi2 = ctx->p.psi2;
  a.rtol = ctx->p.riemann_tol;
  a.rmaxit = ctx->p.riemann_maxit;
  a.limiter = ctx->p.limiter;
  a.counters = ctx->counters;
  const int nb = blocks_for(pp->n, FLUX_BS);
  if (ctx->p.scheme == MFM_SCHEME_MFM)
    fluxes_k<MFM_SCHEME_MFM, FLUX_BS><<<nb, FLUX_BS, 0, ctx->stream>>>(a);
  else
    fluxes_k<MFM_SCHEME_MFV, FLUX_BS><<<nb, FLUX_BS, 0, ctx->stream>>>(a);
  return hipGetLastError();
}
