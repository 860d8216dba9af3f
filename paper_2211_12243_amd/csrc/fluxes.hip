// fluxes.hip -- loop (3) of the scheme: face vector, half-step extrapolation,
// pairwise limiter, exact Riemann solver and MFV/MFM fluxes (sec. 2.3.3, 2.3.4,
// 2.3.6), accumulated antisymmetrically (eq. hydro_discr).
//
// Work split.  A workgroup owns a block of FLUX_BLOCK consecutive particles of
// the Z-ordered list and an LDS accumulator per particle.  The gradient loop
// has listed, per particle, the faces it evaluates: a face inside the block
// once (the side emit_face picks), a face crossing the block boundary on both
// sides.  Here the block's faces are laid out one per lane (a block prefix sum
// of the per-particle counts, then a binary search maps lane -> particle), so
// the Riemann solves run on full wavefronts.  The face function always takes
// the lower slot as the left state, so both evaluations of a crossing face are
// bitwise identical and every pair stays exactly antisymmetric.  The owning
// side is summed with a segmented wave reduction (a wave's faces belong to a
// few consecutive particles), the in-block other side with an LDS atomic.  No
// global atomics: FP64 global atomic adds run at ~23 G/s on this part, far
// too slow for a scatter of ~10 per face.
//
// Arithmetic.  For gamma = m / (m - 2) with integer m every power in the exact
// solver is an integer power of x^(1/m); for m = 5 (gamma 5/3) and m = 7
// (gamma 7/5) that root is an FP32 seed polished by two FP64 Newton steps on
// y^m = x (quadratic: 1e-7 -> 1e-14 -> roundoff).  Other gammas call pow().
#include "mfm_internal.h"

namespace {

constexpr int FBS = FLUX_BLOCK;

struct Gas {
  double gamma, g1, g2, g3, g4, g5, g6, g7, inv_gm1;
  int m;          // 1 / g1 when it is an integer (the root path), else 0
};

struct FluxArgs {
  int64_t n;
  const double *rec;
  const int32_t *fslot, *fcnt;
  const double *dt;
  double *dQ;
  double box[3], half[3];
  Gas G;
  double psi1, psi2, rtol;
  int rmaxit, limiter;
  int64_t *counters;
};

// x^(1/m), x > 0.
template <int M>
__device__ __forceinline__ double root_m(double x, const Gas &G) {
  if (M == 0) return pow(x, G.g1);
  double y = (double)exp2f((1.0f / (float)M) * log2f((float)x));
  if (!(y > 0.0) || !isfinite(y)) return pow(x, G.g1);  // outside the FP32 range
  constexpr double im = 1.0 / (double)(M > 0 ? M : 1);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double ym1 = 1.0;  // y^(m-1)
#pragma unroll
    for (int k = 1; k < M; ++k) ym1 *= y;
    y = y + (x / ym1 - y) * im;
  }
  return y;
}

template <int K>
__device__ __forceinline__ double ipow(double x) {
  double r = 1.0;
#pragma unroll
  for (int q = 0; q < K; ++q) r *= x;
  return r;
}

// x^(g4) and x^(g3) (g4 = m - 2 and g3 = m on the root path).
template <int M>
__device__ __forceinline__ double pow_g4(double x, const Gas &G) {
  return M ? ipow<(M > 2 ? M - 2 : 0)>(x) : pow(x, G.g4);
}
template <int M>
__device__ __forceinline__ double pow_g3(double x, const Gas &G) {
  return M ? ipow<M>(x) : pow(x, G.g3);
}

struct Side {
  double r, u, p, c;
  double ip;   // 1 / p
  double A;    // 2 / ((gamma + 1) rho)
  double B;    // (gamma - 1) / (gamma + 1) p
  double prc;  // p / (rho c)
  double g4c;  // 2 c / (gamma - 1)
};

__device__ __forceinline__ Side make_side(double r, double u, double p, double c, const Gas &G) {
  Side s;
  s.r = r; s.u = u; s.p = p; s.c = c;
  s.ip = 1.0 / p;
  s.A = G.g5 / r;
  s.B = G.g6 * p;
  s.prc = p / (r * c);
  s.g4c = G.g4 * c;
  return s;
}

// Toro's pressure function of one side and its derivative at pressure ps (ips = 1/ps).
template <int M>
__device__ __forceinline__ void pressure_fn(double ps, double ips, const Side &s, const Gas &G,
                                            double &f, double &df) {
  if (ps <= s.p) {
    const double e = root_m<M>(ps * s.ip, G);  // (p*/p_K)^((gamma-1)/(2 gamma))
    f = s.g4c * (e - 1.0);
    df = e * s.prc * ips;                          // (p*/p_K)^(g1 - 1) / (rho_K c_K)
  } else {
    const double t = 1.0 / (s.B + ps);
    const double q = sqrt(s.A * t);
    const double dp = ps - s.p;
    f = dp * q;
    df = q * (1.0 - 0.5 * dp * t);
  }
}

// Exact Riemann solve: 0 converged, 1 vacuum, 2 iteration cap.
template <int M>
__device__ int riemann_solve(const Gas &G, const Side &L, const Side &R, double tol, int maxit,
                             double &ps, double &us, int &iters) {
  const double du = R.u - L.u;
  iters = 0;
  if (G.g4 * (L.c + R.c) <= du) {
    ps = 0.0;
    us = 0.5 * (L.u + R.u);
    return 1;
  }
  const double pmin = fmin(L.p, R.p), pmax = fmax(L.p, R.p);
  double ppv = 0.5 * (L.p + R.p) - 0.125 * du * (L.r + R.r) * (L.c + R.c);
  ppv = fmax(ppv, 0.0);
  double p0;
  if (pmax <= 2.0 * pmin && pmin <= ppv && ppv <= pmax) {
    p0 = ppv;
  } else if (ppv < pmin) {
    // two-rarefaction value: [(cL + cR - g7 du) / (cL pL^-g1 + cR pR^-g1)]^(1/g1)
    const double num = L.c + R.c - G.g7 * du;
    const double den = L.c / root_m<M>(L.p, G) + R.c / root_m<M>(R.p, G);
    const double t = num / den;
    p0 = M ? ipow<M>(t) : pow(t, 1.0 / G.g1);
  } else {
    const double gL = sqrt(L.A / (L.B + ppv));
    const double gR = sqrt(R.A / (R.B + ppv));
    p0 = (gL * L.p + gR * R.p - du) / (gL + gR);
  }
  const double pfloor = 1e-10 * 0.5 * (L.p + R.p);
  if (!(p0 > pfloor)) p0 = pfloor;
  double p = p0, fL, dfL, fR, dfR;
  int status = 2;
  for (int it = 1; it <= maxit; ++it) {
    const double ip = 1.0 / p;
    pressure_fn<M>(p, ip, L, G, fL, dfL);
    pressure_fn<M>(p, ip, R, G, fR, dfR);
    double pn = p - (fL + fR + du) / (dfL + dfR);
    if (pn < 0.0) pn = pfloor;
    const bool done = 2.0 * fabs(pn - p) < tol * (pn + p);
    p = pn;
    iters = it;
    if (done) {
      status = 0;
      break;
    }
  }
  const double ip = 1.0 / p;
  pressure_fn<M>(p, ip, L, G, fL, dfL);
  pressure_fn<M>(p, ip, R, G, fR, dfR);
  ps = p;
  us = 0.5 * (L.u + R.u) + 0.5 * (fR - fL);
  return status;
}

// The exact solution at x/t = 0 in the face frame (Toro's sampling).
template <int M>
__device__ void sample_at_face(const Gas &G, const Side &L, const Side &R, double ps, double us,
                               double &rf, double &uf, double &pf) {
  if (0.0 <= us) {
    if (ps <= L.p) {
      if (0.0 <= L.u - L.c) {
        rf = L.r; uf = L.u; pf = L.p;
      } else {
        const double t = ps * L.ip;
        const double e = root_m<M>(t, G);
        if (0.0 > us - L.c * e) {
          rf = L.r * (M ? ipow<(M > 2 ? M - 2 : 0)>(e) : pow(t, 1.0 / G.gamma)); uf = us; pf = ps;
        } else {
          const double cc = G.g5 * (L.c + G.g7 * L.u);
          const double x = cc / L.c;
          uf = cc;
          rf = L.r * pow_g4<M>(x, G);
          pf = L.p * pow_g3<M>(x, G);
        }
      }
    } else {
      const double pml = ps * L.ip;
      const double sl = L.u - L.c * sqrt(G.g2 * pml + G.g1);
      if (0.0 <= sl) {
        rf = L.r; uf = L.u; pf = L.p;
      } else {
        rf = L.r * (pml + G.g6) / (pml * G.g6 + 1.0); uf = us; pf = ps;
      }
    }
  } else {
    if (ps > R.p) {
      const double pmr = ps * R.ip;
      const double sr = R.u + R.c * sqrt(G.g2 * pmr + G.g1);
      if (0.0 >= sr) {
        rf = R.r; uf = R.u; pf = R.p;
      } else {
        rf = R.r * (pmr + G.g6) / (pmr * G.g6 + 1.0); uf = us; pf = ps;
      }
    } else {
      if (0.0 >= R.u + R.c) {
        rf = R.r; uf = R.u; pf = R.p;
      } else {
        const double t = ps * R.ip;
        const double e = root_m<M>(t, G);
        if (0.0 <= us + R.c * e) {
          rf = R.r * (M ? ipow<(M > 2 ? M - 2 : 0)>(e) : pow(t, 1.0 / G.gamma)); uf = us; pf = ps;
        } else {
          const double cc = G.g5 * (R.c - G.g7 * R.u);
          const double x = cc / R.c;
          uf = -cc;
          rf = R.r * pow_g4<M>(x, G);
          pf = R.p * pow_g3<M>(x, G);
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
    const double lower = ((qo - d1) * qo > 0.0) ? qo - d1 : qo / (1.0 + d1 / fabs(qo));
    return fmax(lower, fmin(qbar + d2, qf));
  }
  const double upper = ((qo + d1) * qo > 0.0) ? qo + d1 : qo / (1.0 + d1 / fabs(qo));
  return fmin(upper, fmax(qbar - d2, qf));
}

enum { F_VACUUM = 1, F_POSITIVITY = 2, F_MAXIT = 4 };

constexpr double W_NORM = 8.0 / 3.14159265358979323846;

// Contribution c = |A_ij| F_ij of the face between records Lr (left) and Rr.
template <int SCHEME, int M>
__device__ void face_flux(const double *__restrict__ Lr, const double *__restrict__ Rr,
                          const FluxArgs &a, double hdt, double c[5], int &iters, int &flags) {
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
  const double ihL = Lr[R_IH], ihR = Rr[R_IH];
  const double WL = W_NORM * ihL * ihL * ihL * spline_w(r * ihL);
  const double WR = W_NORM * ihR * ihR * ihR * spline_w(r * ihR);
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
  const double iA = 1.0 / Am;
  const double nv[3] = {A[0] * iA, A[1] * iA, A[2] * iA};

  double qi[5], qj[5], qL[5], qR[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    qi[q] = Lr[R_RHO + (q ? q + 1 : 0)];
    qj[q] = Rr[R_RHO + (q ? q + 1 : 0)];
  }
  const double *gi = Lr + R_G, *gj = Rr + R_G;
  {
    // half-step Lagrangian predictor plus extrapolation to the mid-point face
    const double dvi = gi[3] + gi[7] + gi[11];
    const double dvj = gj[3] + gj[7] + gj[11];
    const double iri = Lr[R_IRHO], irj = Rr[R_IRHO];
    qL[0] = qi[0] - hdt * qi[0] * dvi;
    qR[0] = qj[0] - hdt * qj[0] * dvj;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qL[1 + k] = qi[1 + k] - hdt * gi[12 + k] * iri;
      qR[1 + k] = qj[1 + k] - hdt * gj[12 + k] * irj;
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
  const Side SL = make_side(qL[0], uL, qL[4], sqrt(G.gamma * qL[4] / qL[0]), G);
  const Side SR = make_side(qR[0], uR, qR[4], sqrt(G.gamma * qR[4] / qR[0]), G);
  double ps, us;
  const int st = riemann_solve<M>(G, SL, SR, a.rtol, a.rmaxit, ps, us, iters);
  if (st == 1) {
    flags |= F_VACUUM;
    return;
  }
  if (st == 2) flags |= F_MAXIT;
  const double vfn = vf[0] * nv[0] + vf[1] * nv[1] + vf[2] * nv[2];
  if (SCHEME == MFM_SCHEME_MFM) {
    const double Ap = Am * ps;
    c[0] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = Ap * nv[k];
    c[4] = Ap * (us + vfn);
  } else {
    double rf, uf, pf;
    sample_at_face<M>(G, SL, SR, ps, us, rf, uf, pf);
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

template <int SCHEME, int M>
__global__ void __launch_bounds__(FBS) fluxes_k(FluxArgs a) {
  __shared__ int pref[FBS + 1];
  __shared__ int wsum[FBS / 64];
  __shared__ double acc[5][FBS];
  const int64_t n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int b0 = blockIdx.x * FBS;
  const int nb = (int)min((int64_t)FBS, n - b0);
  // block exclusive prefix sum of the per-particle face counts
  int cnt = tid < nb ? a.fcnt[b0 + tid] : 0;
  int incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wid] = incl;
#pragma unroll
  for (int f = 0; f < 5; ++f) acc[f][tid] = 0.0;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += wsum[w];
  pref[tid] = woff + incl - cnt;
  if (tid == FBS - 1) pref[FBS] = woff + incl;
  __syncthreads();
  const int T = pref[FBS];
  const double dt = a.dt[0];
  const double hdt = 0.5 * dt;
  int64_t nfaces = 0, iters_sum = 0, vac = 0, pos = 0, maxit = 0;
  for (int base = 0; base < T; base += FBS) {
    const int f = base + tid;
    const bool active = f < T;
    int p = FBS;  // sentinel key for idle lanes (they sit at the wave's end)
    double c[5] = {0, 0, 0, 0, 0};
    if (active) {
      // particle p of this face: pref[p] <= f < pref[p + 1]
      int lo = 0, hi = FBS;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= f) lo = mid; else hi = mid;
      }
      p = lo;
      const int i = b0 + p;
      const int j = a.fslot[list_at(i, f - pref[p], n)];
      const int L = i < j ? i : j, R = i < j ? j : i;
      int it, fl;
      face_flux<SCHEME, M>(a.rec + (int64_t)L * R_STRIDE, a.rec + (int64_t)R * R_STRIDE, a,
                              hdt, c, it, fl);
      const double sgn = (i == L) ? -1.0 : 1.0;  // the left side loses c
#pragma unroll
      for (int q = 0; q < 5; ++q) c[q] *= sgn;
      const bool inb = (j >= b0) && (j < b0 + nb);
      if (inb) {
#pragma unroll
        for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q)
          atomicAdd(&acc[q][j - b0], -c[q]);
      }
      if (inb || i < j) {
        ++nfaces;
        iters_sum += it;
        vac += (fl & F_VACUUM) ? 1 : 0;
        pos += (fl & F_POSITIVITY) ? 1 : 0;
        maxit += (fl & F_MAXIT) ? 1 : 0;
      }
    }
    // segmented sum over lanes with the same particle (keys ascend across lanes)
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int kp = __shfl_up(p, o, 64);
      const bool same = lane >= o && kp == p;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double u = __shfl_up(c[q], o, 64);
        if (same) c[q] += u;
      }
    }
    const int kn = __shfl_down(p, 1, 64);
    if (active && (lane == 63 || kn != p)) {
#pragma unroll
      for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q) atomicAdd(&acc[q][p], c[q]);
    }
  }
  __syncthreads();
  if (tid < nb) {
#pragma unroll
    for (int q = 0; q < 5; ++q) a.dQ[(int64_t)q * n + b0 + tid] = dt * acc[q][tid];
  }
  count_add(a.counters + C_FACES, nfaces);
  count_add(a.counters + C_RIEMANN_ITERS, iters_sum);
  count_add(a.counters + C_VACUUM, vac);
  count_add(a.counters + C_POSITIVITY, pos);
  count_add(a.counters + C_RIEMANN_MAXIT, maxit);
}

template <int SCHEME>
void launch_scheme(const FluxArgs &a, int nb, hipStream_t st) {
  if (a.G.m == 5)
    fluxes_k<SCHEME, 5><<<nb, FBS, 0, st>>>(a);
  else if (a.G.m == 7)
    fluxes_k<SCHEME, 7><<<nb, FBS, 0, st>>>(a);
  else
    fluxes_k<SCHEME, 0><<<nb, FBS, 0, st>>>(a);
}

}  // namespace

hipError_t launch_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  FluxArgs a;
  a.n = pp->n;
  a.rec = ctx->rec;
  a.fslot = ctx->fslot;
  a.fcnt = ctx->fcnt;
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
  // root path when 1/g1 = 2 gamma / (gamma - 1) is an integer m (gamma = m/(m-2))
  const double mm = a.G.g3;
  const int mi = (int)(mm + 0.5);
  a.G.m = (mi >= 3 && mi <= 16 && fabs(mm - mi) < 1e-12 * mm) ? mi : 0;
  a.psi1 = ctx->p.psi1;
  a.psi2 = ctx->p.psi2;
  a.rtol = ctx->p.riemann_tol;
  a.rmaxit = ctx->p.riemann_maxit;
  a.limiter = ctx->p.limiter;
  a.counters = ctx->counters;
  const int nb = blocks_for(pp->n, FBS);
  if (ctx->p.scheme == MFM_SCHEME_MFM)
    launch_scheme<MFM_SCHEME_MFM>(a, nb, ctx->stream);
  else
    launch_scheme<MFM_SCHEME_MFV>(a, nb, ctx->stream);
  return hipGetLastError();
}
