// fluxes.hip -- loop (3) of the scheme: face vector, half-step extrapolation,
// pairwise limiter, exact Riemann solver and MFV/MFM fluxes (sec. 2.3.3, 2.3.4,
// 2.3.6), accumulated antisymmetrically (eq. hydro_discr).
//
// Work split.  A workgroup owns a block of FLUX_BLOCK consecutive particles of
// the Z-ordered list and an LDS accumulator per particle.  The gradient loop
// has listed every face once, under the particle emit_face picks.  Here the
// block's faces are laid out one per lane (a block prefix sum of the
// per-particle counts, then a binary search maps lane -> particle), so the
// Riemann solves run on full wavefronts.  The face function always takes the
// lower slot as the left state and the two particles receive exactly opposite
// values, so every pair stays antisymmetric.  Both sides of an in-block face
// are added with FP64 LDS atomics (measured 5% faster than a segmented wave
// reduction of the owning side), an other side in another block with a
// native FP64 global atomic add into dq_ext, which is folded into dQ after
// the loop.  Evaluating a block-crossing face on both sides instead (no
// global atomics) costs 25% more face evaluations at 1024 particles per
// block.  A set of few blocks (a few thousand particles) would leave most of
// the chip idle and each workgroup with a long serial face loop: there each
// block's faces are cut into contiguous slices, one workgroup per slice;
// slice 0 writes the block's sums and the others add theirs into dq_ext.
//
// Precision.  T = double is the FP64 path.  T = float is the mixed path: the
// separation is formed in FP64 from FP64 positions and rounded; the face
// vector, extrapolation, limiter and the Newton iteration of the Riemann solve
// run in FP32; the solve is then checked in FP64 (one FP64 Newton step from
// the FP32 root, more if that step is not already in the quadratic regime),
// and every contribution is accumulated in FP64.
//
// Powers.  For gamma = m / (m - 2) with integer m every power in the exact
// solver is an integer power of x^(1/m).  In FP64, for m = 5 (gamma 5/3) and
// m = 7 (gamma 7/5), that root is an FP32 seed polished by two FP64 Newton
// steps on y^m = x (quadratic: 1e-7 -> 1e-14 -> roundoff); in FP32 it is the
// hardware exp2/log2.  Other gammas call pow().
//
// Learned guess.  The first pass hands every face that may pass the guess
// network's gate to the FP64 second pass (hand_over).  There a wavefront of
// 16 faces holding a gated one evaluates the network (mlp_device.h) on one
// 16-row tile with BF16 MFMA, from a copy of the weights in LDS.  The network
// predicts the error of the plain starting value p0, y = ln(p* / p0), and Newton
// starts from p0 exp(y).  The exact iteration always finishes the solve; a
// guess that is not finite and above the pressure floor, whose first Newton
// step increases |f|, or that needs more than GUESS_MAXIT iterations is
// dropped for the plain guess (counted).
//
// Face dump.  With a dump buffer armed, every face (once) appends an 8-float
// record: the six guess features, ln(p* / p0) and the Newton iteration count
// of its solve -- the network's training data.
#include "mfm_internal.h"
#include "mlp_device.h"

namespace {

constexpr int FBS = FLUX_BLOCK;  // particles per workgroup
constexpr int FTH = 256;         // threads per workgroup
constexpr int PPT = FBS / FTH;   // particles per thread in the block prefix sum
static_assert(FBS % FTH == 0, "flux block must be a multiple of the workgroup size");
constexpr int GUESS_MAXIT = 8;
constexpr int FLUX_WG_TARGET = 1024;  // workgroups below which blocks are split
constexpr int FLUX_MAX_SPLIT = 32;

template <typename T>
struct Gas {
  T gamma, g1, g2, g3, g4, g5, g6, g7, inv_gm1;
  T sg5;  // sqrt(g5)
};

struct FluxArgs {
  int64_t n;
  const double *rec;
  const double4 *pos;
  const int32_t *fslot, *fcnt;
  const int64_t *lseg;  // list blocks of the chunks (list_at)
  const double *dt;
  double *dQ;
  double *dq_ext;  // dt F A of faces whose other particle lies outside the block
  double box[3], half[3];
  Gas<double> G;
  Gas<float> Gf;
  double psi1, psi2, rtol;
  float rtol_f;
  int rmaxit, limiter;
  int64_t *counters;
  mlp::Net net;             // learned guess (LEARNED kernels only)
  float *dump;              // face records (null: off)
  int64_t dump_cap;
  unsigned long long *dump_count;
  // the FP64 second pass: faces the first pass hands over
  int2 *hard_q;             // (lower, higher) slot of each queued face, HARD_SEGS segments
  int64_t hard_cap;         // of hard_cap / HARD_SEGS faces
  unsigned long long *hard_len;  // segment lengths, HARD_SEG_STRIDE apart
  float jump;               // mixed path: pressure or density ratio that sends a face to FP64
  // learned guess: the face-state pressure ratio and normal velocity jump
  // (in units of c_L + c_R) beyond which the first pass hands a face over,
  // a superset of the network's gate (0: off)
  float gate_p, gate_du;
  // workgroups per block of FBS particles (a small set: several share a
  // block, each solving a contiguous slice of its faces)
  int split;
  // the caller's FP64 particle arrays, which the second pass reads in place of
  // the mixed path's FP32 record (near the edge of the support, W(r, H) moves
  // by 3 (1 - r/H)^-1 times the relative error of 1/H)
  const double *x, *y, *z, *H, *V, *rho, *vx, *vy, *vz, *P;
  // comoving integration: every spatial derivative (fluxes, predictor
  // gradients) carries inv_a = 1/a; 1 in physical coordinates
  double inv_a;
  // MFV with gravity: sum_j dm_ij (x_j - x_i) per particle (3 n; null: off)
  double *gwork;
  // individual time steps (R.rung null: one global step): each face's step is
  // min(dt_i, dt_j), each side predicted over its elapsed time plus half of
  // it, positions from pos, and the flux sums are added to dQ
  Rungs R;
};

// The work term of the exchanged mass (sec. 2.3.8): the mass dm that goes
// from L to R crosses x_R - x_L; both sides add dm (x_R - x_L), each later
// weighted with its own acceleration.
__device__ __forceinline__ void add_gwork(const FluxArgs &a, int L, int R, double dm) {
  const double d0 = min_image(a.x[R] - a.x[L], a.box[0], a.half[0]);
  const double d1 = min_image(a.y[R] - a.y[L], a.box[1], a.half[1]);
  const double d2 = min_image(a.z[R] - a.z[L], a.box[2], a.half[2]);
  const int64_t n = a.n;
  const double d[3] = {d0, d1, d2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    unsafeAtomicAdd(&a.gwork[(int64_t)k * n + L], dm * d[k]);
    unsafeAtomicAdd(&a.gwork[(int64_t)k * n + R], dm * d[k]);
  }
}

template <typename T>
__device__ __forceinline__ const Gas<T> &gas_of(const FluxArgs &a);
template <>
__device__ __forceinline__ const Gas<double> &gas_of<double>(const FluxArgs &a) { return a.G; }
template <>
__device__ __forceinline__ const Gas<float> &gas_of<float>(const FluxArgs &a) { return a.Gf; }

template <int K, typename T>
__device__ __forceinline__ T ipow(T x) {
  T r = T(1);
#pragma unroll
  for (int q = 0; q < K; ++q) r *= x;
  return r;
}

// Reciprocal and reciprocal square root from the hardware estimates.  FP64:
// two Newton steps on the estimate (error a few ulp, against the half ulp of
// the IEEE division and square-root sequences, at half their instructions);
// FP32: the estimate itself (1 ulp).  Arguments are finite and positive.
template <typename T>
__device__ __forceinline__ T frcp(T x);
template <>
__device__ __forceinline__ double frcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
template <>
__device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ T frsq(T x);
template <>
__device__ __forceinline__ double frsq<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  return y * fma(-hx * y, y, 1.5);
}
template <>
__device__ __forceinline__ float frsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// The same for any x > 0: below the normal range (where the estimates flush
// to infinity) the IEEE sequences.  A face whose separation sits just inside
// the larger support radius has a kernel weight, and so a |A|^2, that can
// underflow FP32.
template <typename T>
__device__ __forceinline__ T rsq_any(T x) {
  constexpr T tiny = sizeof(T) == sizeof(float) ? T(1.17549435e-38f) : T(2.2250738585072014e-308);
  if (x >= tiny) return frsq<T>(x);
  return T(1) / sqrt(x);
}
template <typename T>
__device__ __forceinline__ T rcp_any(T x) {
  constexpr T tiny = sizeof(T) == sizeof(float) ? T(1.17549435e-38f) : T(2.2250738585072014e-308);
  if (x >= tiny) return frcp<T>(x);
  return T(1) / x;
}

// x^(-1/m) (= x^-g1), x > 0.  FP64 (m = 5, 7): an FP32 seed and two
// division-free Newton steps z += z (1 - x z^m) / m (quadratic: ~1e-7 ->
// ~1e-13 -> roundoff); FP32: the hardware exp2/log2.  Other m: pow().
template <typename T, int M>
__device__ __forceinline__ T iroot_m(T x, const Gas<T> &G) {
  if (M == 0) return pow(x, -G.g1);
  if (sizeof(T) == sizeof(float)) return (T)exp2f(log2f((float)x) * (-1.0f / (float)M));
  constexpr int MM = M > 0 ? M : 1;
  constexpr double im = 1.0 / (double)MM;
  double z = (double)exp2f((-1.0f / (float)MM) * log2f((float)x));
  if (!(z > 0.0) || !isfinite(z)) return pow(x, -G.g1);  // outside the FP32 range
#pragma unroll
  for (int it = 0; it < 2; ++it) z = fma(z * im, fma(-(double)x, ipow<MM>(z), 1.0), z);
  return (T)z;
}

// x^(1/m) = x * (x^(-1/m))^(m-1), x > 0.
template <typename T, int M>
__device__ __forceinline__ T root_m(T x, const Gas<T> &G) {
  if (M == 0) return pow(x, G.g1);
  if (sizeof(T) == sizeof(float)) return (T)exp2f(log2f((float)x) * (1.0f / (float)M));
  constexpr int MM = M > 0 ? M : 1;
  return x * ipow<MM - 1>(iroot_m<T, M>(x, G));
}

template <typename T>
struct Side {
  T r, u, p, c;
  T ip;   // 1 / p
  T A;    // 2 / ((gamma + 1) rho)
  T B;    // (gamma - 1) / (gamma + 1) p
  T prc;  // p / (rho c)
  T g4c;  // 2 c / (gamma - 1)
  T sA;   // sqrt(A)
};

template <typename T>
__device__ __forceinline__ Side<T> make_side(T r, T u, T p, const Gas<T> &G) {
  Side<T> s;
  const T ir = frcp<T>(r);
  const T c2 = G.gamma * p * ir;
  const T ic = frsq<T>(c2);  // 1 / c
  s.r = r; s.u = u; s.p = p;
  s.c = c2 * ic;
  s.ip = frcp<T>(p);
  s.A = G.g5 * ir;
  s.sA = G.sg5 * frsq<T>(r);
  s.B = G.g6 * p;
  s.prc = p * ir * ic;
  s.g4c = G.g4 * s.c;
  return s;
}

// Toro's pressure function of one side and its derivative at pressure ps (ips = 1/ps).
template <typename T, int M>
__device__ __forceinline__ void pressure_fn(T ps, T ips, const Side<T> &s, const Gas<T> &G, T &f,
                                            T &df) {
  if (ps <= s.p) {
    const T e = root_m<T, M>(ps * s.ip, G);  // (p*/p_K)^((gamma-1)/(2 gamma))
    f = s.g4c * (e - T(1));
    df = e * s.prc * ips;                     // (p*/p_K)^(g1 - 1) / (rho_K c_K)
  } else {
    const T y = frsq<T>(s.B + ps);  // (B + p)^(-1/2)
    const T q = s.sA * y;           // sqrt(A / (B + p))
    const T dp = ps - s.p;
    f = dp * q;
    df = q * (T(1) - T(0.5) * dp * y * y);
  }
}

// Newton iteration on f(p) = f_L(p) + f_R(p) + du from p0, then u*.
// qtol > 0: a relative step below sqrt(qtol) ends the iteration -- the error
// left after it is of the order of its square -- and u* takes the first-order
// update of f_L, f_R (this saves the final evaluation of both pressure
// functions).
// guard > 0: the start is a guess to be judged; return 3 (reject) if the
// second residual exceeds the first or more than guard iterations are needed.
// Returns 0 converged, 2 iteration cap, 3 guess rejected.
template <typename T, int M>
__device__ int riemann_newton(const Gas<T> &G, const Side<T> &L, const Side<T> &R, T p0,
                              T pfloor, T tol, int maxit, T qtol, int guard, T &ps, T &us,
                              int &iters) {
  const T du = R.u - L.u;
  T p = p0, fL, dfL, fR, dfR, res0 = T(0);
  int status = 2;
  for (int it = 1; it <= maxit; ++it) {
    const T ip = frcp<T>(p);
    pressure_fn<T, M>(p, ip, L, G, fL, dfL);
    pressure_fn<T, M>(p, ip, R, G, fR, dfR);
    const T res = fL + fR + du;
    if (guard) {
      if (it == 1) res0 = fabs(res);
      if ((it == 2 && fabs(res) > res0) || it > guard) return 3;
    }
    T pn = p - res * frcp<T>(dfL + dfR);
    if (pn < T(0)) pn = pfloor;
    const T step = T(2) * fabs(pn - p);  // relative change: step / (pn + p)
    ++iters;
    if (step * step < qtol * (pn + p) * (pn + p)) {
      const T dp = pn - p;
      ps = pn;
      us = T(0.5) * (L.u + R.u) + T(0.5) * ((fR + dfR * dp) - (fL + dfL * dp));
      return 0;
    }
    const bool done = step < tol * (pn + p);
    p = pn;
    if (done) {
      status = 0;
      break;
    }
  }
  const T ip = frcp<T>(p);
  pressure_fn<T, M>(p, ip, L, G, fL, dfL);
  pressure_fn<T, M>(p, ip, R, G, fR, dfR);
  ps = p;
  us = T(0.5) * (L.u + R.u) + T(0.5) * (fR - fL);
  return status;
}

// Toro's adaptive starting value: the primitive-variable pressure when the
// states are close, else the two-rarefaction or two-shock value (branch:
// which of the three, mlp::GuessBranch).
template <typename T, int M>
__device__ T plain_guess(const Gas<T> &G, const Side<T> &L, const Side<T> &R, int &branch) {
  const T du = R.u - L.u;
  const T pmin = fmin(L.p, R.p), pmax = fmax(L.p, R.p);
  T ppv = T(0.5) * (L.p + R.p) - T(0.125) * du * (L.r + R.r) * (L.c + R.c);
  ppv = fmax(ppv, T(0));
  branch = mlp::GUESS_PV;
  if (pmax <= T(2) * pmin && pmin <= ppv && ppv <= pmax) return ppv;
  if (ppv < pmin) {
    branch = mlp::GUESS_TR;
    // two-rarefaction value: [(cL + cR - g7 du) / (cL pL^-g1 + cR pR^-g1)]^(1/g1)
    const T num = L.c + R.c - G.g7 * du;
    const T den = L.c * iroot_m<T, M>(L.p, G) + R.c * iroot_m<T, M>(R.p, G);
    const T t = num * frcp<T>(den);
    return M ? ipow<(M > 0 ? M : 1)>(t) : pow(t, T(1) / G.g1);
  }
  branch = mlp::GUESS_TS;
  const T gL = L.sA * frsq<T>(L.B + ppv);
  const T gR = R.sA * frsq<T>(R.B + ppv);
  return (gL * L.p + gR * R.p - du) * frcp<T>(gL + gR);
}

// The plain starting value above the solver's pressure floor.
template <typename T, int M>
__device__ T floored_guess(const Gas<T> &G, const Side<T> &L, const Side<T> &R, int &branch) {
  const T pfloor = T(1e-10) * T(0.5) * (L.p + R.p);
  const T p0 = plain_guess<T, M>(G, L, R, branch);
  return p0 > pfloor ? p0 : pfloor;
}

// Exact Riemann solve: 0 converged, 1 vacuum, 2 iteration cap.  pguess and
// branch: the plain starting value and its estimate.  learned: the network's
// correction y to it, p0 exp(y), is tried first (guarded); fallback is set
// when it was rejected.
template <typename T, int M>
__device__ int riemann_solve(const Gas<T> &G, const Side<T> &L, const Side<T> &R, T tol, int maxit,
                             bool learned, float y, T &ps, T &us, int &iters, bool &fallback,
                             T &pguess, int &branch) {
  const T du = R.u - L.u;
  iters = 0;
  fallback = false;
  pguess = T(0);
  branch = mlp::GUESS_PV;
  if (G.g4 * (L.c + R.c) <= du) {
    ps = T(0);
    us = T(0.5) * (L.u + R.u);
    return 1;
  }
  const T pfloor = T(1e-10) * T(0.5) * (L.p + R.p);
  // FP64: stop once a step is below 1e-2 sqrt(tol); the root is then within
  // ~1e-4 tol.  FP32: stop once a step is below 1e-4, which leaves the root
  // at FP32 precision; the FP64 check that follows sets p* and u*.
  const T qtol = sizeof(T) == sizeof(double) ? T(1e-4) * tol : T(1e-8);
  const T p0 = floored_guess<T, M>(G, L, R, branch);
  pguess = p0;
  if (learned) {
    const T pl = p0 * T(expf(y));
    if (pl > pfloor && isfinite(pl)) {
      const int st = riemann_newton<T, M>(G, L, R, pl, pfloor, tol, maxit, qtol, GUESS_MAXIT,
                                          ps, us, iters);
      if (st != 3) return st;
    }
    fallback = true;
  }
  return riemann_newton<T, M>(G, L, R, p0, pfloor, tol, maxit, qtol, 0, ps, us, iters);
}

// The exact solution at x/t = 0 in the face frame (Toro's sampling).
template <typename T, int M>
__device__ void sample_at_face(const Gas<T> &G, const Side<T> &L, const Side<T> &R, T ps, T us,
                               T &rf, T &uf, T &pf) {
  constexpr int MG4 = M > 2 ? M - 2 : 0;  // g4 = m - 2, g3 = m, 1/gamma = (m - 2)/m
  if (T(0) <= us) {
    if (ps <= L.p) {
      if (T(0) <= L.u - L.c) {
        rf = L.r; uf = L.u; pf = L.p;
      } else {
        const T t = ps * L.ip;
        const T e = root_m<T, M>(t, G);
        if (T(0) > us - L.c * e) {
          rf = L.r * (M ? ipow<MG4>(e) : pow(t, T(1) / G.gamma)); uf = us; pf = ps;
        } else {
          const T cc = G.g5 * (L.c + G.g7 * L.u);
          const T x = cc / L.c;
          uf = cc;
          rf = L.r * (M ? ipow<MG4>(x) : pow(x, G.g4));
          pf = L.p * (M ? ipow<(M > 0 ? M : 1)>(x) : pow(x, G.g3));
        }
      }
    } else {
      const T pml = ps * L.ip;
      const T sl = L.u - L.c * sqrt(G.g2 * pml + G.g1);
      if (T(0) <= sl) {
        rf = L.r; uf = L.u; pf = L.p;
      } else {
        rf = L.r * (pml + G.g6) / (pml * G.g6 + T(1)); uf = us; pf = ps;
      }
    }
  } else {
    if (ps > R.p) {
      const T pmr = ps * R.ip;
      const T sr = R.u + R.c * sqrt(G.g2 * pmr + G.g1);
      if (T(0) >= sr) {
        rf = R.r; uf = R.u; pf = R.p;
      } else {
        rf = R.r * (pmr + G.g6) / (pmr * G.g6 + T(1)); uf = us; pf = ps;
      }
    } else {
      if (T(0) >= R.u + R.c) {
        rf = R.r; uf = R.u; pf = R.p;
      } else {
        const T t = ps * R.ip;
        const T e = root_m<T, M>(t, G);
        if (T(0) <= us + R.c * e) {
          rf = R.r * (M ? ipow<MG4>(e) : pow(t, T(1) / G.gamma)); uf = us; pf = ps;
        } else {
          const T cc = G.g5 * (R.c - G.g7 * R.u);
          const T x = cc / R.c;
          uf = -cc;
          rf = R.r * (M ? ipow<MG4>(x) : pow(x, G.g4));
          pf = R.p * (M ? ipow<(M > 0 ? M : 1)>(x) : pow(x, G.g3));
        }
      }
    }
  }
}

// Pairwise limiter of a face value qf extrapolated from the own side (qo)
// towards the other side (qn).
template <typename T>
__device__ __forceinline__ T pair_limit(T qf, T qo, T qn, T psi1, T psi2) {
  if (qo == qn) return qo;
  const T dq = fabs(qo - qn);
  const T d1 = psi1 * dq, d2 = psi2 * dq;
  const T qbar = T(0.5) * (qo + qn);
  // qo / (1 + d1 / |qo|) written with one reciprocal (d1 > 0 here)
  const T aq = fabs(qo);
  const T soft = qo * aq * rcp_any<T>(aq + d1);
  if (qo < qn) {
    const T lower = ((qo - d1) * qo > T(0)) ? qo - d1 : soft;
    return fmax(lower, fmin(qbar + d2, qf));
  }
  const T upper = ((qo + d1) * qo > T(0)) ? qo + d1 : soft;
  return fmin(upper, fmax(qbar - d2, qf));
}

template <typename T>
__device__ __forceinline__ T spline_wt(T q) {
  if (q < T(0.5)) return T(1) + q * q * (T(6) * q - T(6));
  if (q < T(1)) {
    const T t = T(1) - q;
    return T(2) * t * t * t;
  }
  return T(0);
}

// One side of a face as the face function reads it.
template <typename T>
struct FaceIn {
  double x, y, z;
  T ih, V, rho, irho, v[3], P, B[6], G[15];
};

__device__ __forceinline__ void load_side(const FluxArgs &a, int i, FaceIn<double> &s) {
  const double *r = a.rec + (int64_t)i * R_STRIDE;
  if (a.R.rung) {
    const double4 p = a.pos[i];  // the position of this sub-step
    s.x = p.x; s.y = p.y; s.z = p.z;
  } else {
    s.x = r[R_X]; s.y = r[R_Y]; s.z = r[R_Z];
  }
  s.ih = r[R_IH]; s.V = r[R_V]; s.rho = r[R_RHO]; s.irho = r[R_IRHO];
  s.v[0] = r[R_VX]; s.v[1] = r[R_VY]; s.v[2] = r[R_VZ]; s.P = r[R_P];
#pragma unroll
  for (int k = 0; k < 6; ++k) s.B[k] = r[R_B + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) s.G[k] = r[R_G + k];
}

__device__ __forceinline__ void load_side(const FluxArgs &a, int i, FaceIn<float> &s) {
  const double4 p = a.pos[i];
  s.x = p.x; s.y = p.y; s.z = p.z;
  const float4 *r = reinterpret_cast<const float4 *>(a.rec) + (int64_t)i * (F_STRIDE / 4);
  float f[F_STRIDE];
#pragma unroll
  for (int k = 0; k < F_STRIDE / 4; ++k) {
    const float4 q = r[k];
    f[4 * k] = q.x; f[4 * k + 1] = q.y; f[4 * k + 2] = q.z; f[4 * k + 3] = q.w;
  }
  s.ih = f[F_IH]; s.V = f[F_V]; s.rho = f[F_RHO]; s.irho = f[F_IRHO];
  s.v[0] = f[F_VX]; s.v[1] = f[F_VY]; s.v[2] = f[F_VZ]; s.P = f[F_P];
#pragma unroll
  for (int k = 0; k < 6; ++k) s.B[k] = f[F_B + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) s.G[k] = f[F_G + k];
}

enum { F_VACUUM = 1, F_POSITIVITY = 2, F_MAXIT = 4, F_FALLBACK = 8 };

constexpr double W_NORM = 8.0 / 3.14159265358979323846;

// A face after reconstruction, ready for the Riemann solve.
template <typename T>
struct FaceState {
  bool skip;  // coincident particles or a vanishing face: no exchange
  T Am, nv[3], vf[3], wL[3], wR[3];
  Side<T> SL, SR;
  int flags;
};

// On individual steps, a face's step is min(dt_L, dt_R), and each side is
// predicted from its own step start: over its elapsed time plus half the
// face's step.  On a global step dt and hL = hR = dt / 2 are left as given.
template <typename T>
__device__ __forceinline__ void face_step(const FluxArgs &a, int L, int R, double &dt, T &hL,
                                          T &hR) {
  if (!a.R.rung) return;
  const int rf = max(a.R.rung[L], a.R.rung[R]);
  dt = rung_step(a.R.dt0, rf);
  hL = T(a.R.elapsed[L] + 0.5 * dt);
  hR = T(a.R.elapsed[R] + 0.5 * dt);
}

// Face vector, half-step predictor, extrapolation, limiter, boost (sec. 2.3.3-2.3.6).
template <typename T>
__device__ void face_prepare(const FaceIn<T> &Ls, const FaceIn<T> &Rs, const FluxArgs &a, T hdtL,
                             T hdtR, FaceState<T> &fs) {
  const Gas<T> &G = gas_of<T>(a);
  fs.skip = true;
  fs.flags = 0;
  T d[3];
  d[0] = T(min_image(Rs.x - Ls.x, a.box[0], a.half[0]));
  d[1] = T(min_image(Rs.y - Ls.y, a.box[1], a.half[1]));
  d[2] = T(min_image(Rs.z - Ls.z, a.box[2], a.half[2]));
  const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == T(0)) return;
  const T r = r2 * rsq_any<T>(r2);
  // A_ij = V_i V_j (W(r, H_i) B_i + W(r, H_j) B_j) d
  const T WL = T(W_NORM) * Ls.ih * Ls.ih * Ls.ih * spline_wt<T>(r * Ls.ih);
  const T WR = T(W_NORM) * Rs.ih * Rs.ih * Rs.ih * spline_wt<T>(r * Rs.ih);
  const T *bL = Ls.B, *bR = Rs.B;
  const T VV = Ls.V * Rs.V;
  T A[3];
  A[0] = VV * (WL * (bL[0] * d[0] + bL[1] * d[1] + bL[2] * d[2]) +
               WR * (bR[0] * d[0] + bR[1] * d[1] + bR[2] * d[2]));
  A[1] = VV * (WL * (bL[1] * d[0] + bL[3] * d[1] + bL[4] * d[2]) +
               WR * (bR[1] * d[0] + bR[3] * d[1] + bR[4] * d[2]));
  A[2] = VV * (WL * (bL[2] * d[0] + bL[4] * d[1] + bL[5] * d[2]) +
               WR * (bR[2] * d[0] + bR[4] * d[1] + bR[5] * d[2]));
  const T Am2 = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
  if (Am2 == T(0)) return;
  const T iA = rsq_any<T>(Am2);
  fs.skip = false;
  fs.Am = Am2 * iA;
#pragma unroll
  for (int k = 0; k < 3; ++k) fs.nv[k] = A[k] * iA;

  const T qi[5] = {Ls.rho, Ls.v[0], Ls.v[1], Ls.v[2], Ls.P};
  const T qj[5] = {Rs.rho, Rs.v[0], Rs.v[1], Rs.v[2], Rs.P};
  const T *gi = Ls.G, *gj = Rs.G;
  T qL[5], qR[5];
  {
    // half-step Lagrangian predictor plus extrapolation to the mid-point face
    const T dvi = gi[3] + gi[7] + gi[11];
    const T dvj = gj[3] + gj[7] + gj[11];
    qL[0] = qi[0] - hdtL * qi[0] * dvi;
    qR[0] = qj[0] - hdtR * qj[0] * dvj;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qL[1 + k] = qi[1 + k] - hdtL * gi[12 + k] * Ls.irho;
      qR[1 + k] = qj[1 + k] - hdtR * gj[12 + k] * Rs.irho;
      // the face moves with the mean of the two particles' velocities at the
      // half step, the time the fluxes stand for
      fs.vf[k] = T(0.5) * (qL[1 + k] + qR[1 + k]);
    }
    qL[4] = qi[4] - hdtL * G.gamma * qi[4] * dvi;
    qR[4] = qj[4] - hdtR * G.gamma * qj[4] * dvj;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] += T(0.5) * (gi[3 * q] * d[0] + gi[3 * q + 1] * d[1] + gi[3 * q + 2] * d[2]);
      qR[q] -= T(0.5) * (gj[3 * q] * d[0] + gj[3 * q + 1] * d[1] + gj[3 * q + 2] * d[2]);
    }
  }
  if (a.limiter & MFM_LIMIT_PAIRWISE) {
    const T psi1 = T(a.psi1), psi2 = T(a.psi2);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] = pair_limit<T>(qL[q], qi[q], qj[q], psi1, psi2);
      qR[q] = pair_limit<T>(qR[q], qj[q], qi[q], psi1, psi2);
    }
  }
  if (!(qL[0] > T(0) && qR[0] > T(0) && qL[4] > T(0) && qR[4] > T(0))) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      qL[q] = qi[q];
      qR[q] = qj[q];
    }
    fs.flags |= F_POSITIVITY;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fs.wL[k] = qL[1 + k] - fs.vf[k];
    fs.wR[k] = qR[1 + k] - fs.vf[k];
  }
  const T uL = fs.wL[0] * fs.nv[0] + fs.wL[1] * fs.nv[1] + fs.wL[2] * fs.nv[2];
  const T uR = fs.wR[0] * fs.nv[0] + fs.wR[1] * fs.nv[1] + fs.wR[2] * fs.nv[2];
  fs.SL = make_side<T>(qL[0], uL, qL[4], G);
  fs.SR = make_side<T>(qR[0], uR, qR[4], G);
}

// Riemann solve and flux of a prepared face: c = |A_ij| F_ij (FP64).  learned,
// y: the network's correction to the plain starting value; pguess_out,
// branch: that plain value (0 for a vacuum or skipped face) and its estimate.
template <typename T, int SCHEME, int M>
__device__ void face_solve(FaceState<T> &fs, const FluxArgs &a, bool learned, float y,
                           double c[5], int &iters, double &ps_out, double &pguess_out,
                           int &branch) {
  const Gas<T> &G = gas_of<T>(a);
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = 0.0;
  iters = 0;
  ps_out = 0.0;
  pguess_out = 0.0;
  branch = mlp::GUESS_PV;
  if (fs.skip) return;
  const Side<T> &SL = fs.SL, &SR = fs.SR;
  T ps, us, pg;
  const T tol = sizeof(T) == sizeof(float) ? T(a.rtol_f) : T(a.rtol);
  bool fallback;
  int st = riemann_solve<T, M>(G, SL, SR, tol, a.rmaxit, learned, y, ps, us, iters, fallback,
                               pg, branch);
  pguess_out = (double)pg;
  if (fallback) fs.flags |= F_FALLBACK;
  if (st == 1) {
    fs.flags |= F_VACUUM;
    return;
  }
  double ps64 = (double)ps, us64 = (double)us;
  if (sizeof(T) == sizeof(float)) {
    // FP64 check of the FP32 root: Newton steps in FP64 until the step is in
    // the quadratic regime of the relative tolerance
    const Gas<double> &G64 = a.G;
    const double rl = SL.r, pl = SL.p, rr = SR.r, pr = SR.p;
    const Side<double> L64 = make_side<double>(rl, (double)SL.u, pl, G64);
    const Side<double> R64 = make_side<double>(rr, (double)SR.u, pr, G64);
    const double pfloor = 1e-10 * 0.5 * (pl + pr);
    st = riemann_newton<double, M>(G64, L64, R64, fmax(ps64, pfloor), pfloor, a.rtol, a.rmaxit,
                                   a.rtol, 0, ps64, us64, iters);
  }
  if (st == 2) fs.flags |= F_MAXIT;
  ps_out = ps64;
  const T *nv = fs.nv, *vf = fs.vf;
  const double vfn = (double)(vf[0] * nv[0] + vf[1] * nv[1] + vf[2] * nv[2]);
  if (SCHEME == MFM_SCHEME_MFM) {
    const double Ap = (double)fs.Am * ps64;
    c[0] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = Ap * (double)nv[k];
    c[4] = Ap * (us64 + vfn);
  } else {
    T rf, uf, pf;
    sample_at_face<T, M>(G, SL, SR, T(ps64), T(us64), rf, uf, pf);
    const T *wu = (us64 >= 0.0) ? fs.wL : fs.wR;
    const T wun = wu[0] * nv[0] + wu[1] * nv[1] + wu[2] * nv[2];
    T vfa[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) vfa[k] = uf * nv[k] + (wu[k] - wun * nv[k]);
    const T v2 = vfa[0] * vfa[0] + vfa[1] * vfa[1] + vfa[2] * vfa[2];
    const T Fm = rf * uf;
    T Fp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Fp[k] = Fm * vfa[k] + pf * nv[k];
    const T FE = uf * (pf * G.inv_gm1 + T(0.5) * rf * v2 + pf);
    const T vf2 = vf[0] * vf[0] + vf[1] * vf[1] + vf[2] * vf[2];
    const double Amd = (double)fs.Am;
    c[0] = Amd * (double)Fm;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[1 + k] = Amd * (double)(Fp[k] + vf[k] * Fm);
    c[4] = Amd * (double)(FE + (vf[0] * Fp[0] + vf[1] * Fp[1] + vf[2] * Fp[2]) +
                          T(0.5) * vf2 * Fm);
  }
}

// A slot in a shared append buffer for each lane with want set: one atomic
// per wavefront on the counter.  Every executing lane of the wavefront calls
// it; lanes without want get an unused value.
__device__ __forceinline__ unsigned long long wave_slot(unsigned long long *counter, bool want,
                                                        int lane) {
  const uint64_t m = __ballot(want);
  if (!m) return 0ull;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  return base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ void features_of(const FaceState<T> &fs, double p0, int branch,
                                            float x[mlp::NIN]) {
  mlp::face_features((float)fs.SL.r, (float)fs.SL.p, (float)fs.SR.r, (float)fs.SR.p,
                     (float)(fs.SR.u - fs.SL.u), (float)fs.SL.c, (float)fs.SR.c, (float)p0, branch,
                     x);
}

// Faces the first pass hands to the FP64 second pass, judged (besides the
// particles' own jump) on the face states it has reconstructed.  Mixed path:
// their pressures or densities differ by more than a.jump, or the face fell
// back to first-order states -- where FP32 extrapolations cancel and the
// Riemann problem is strongest.
// Learned guess: a superset of the network's gate (a.gate_p = 1.9 and
// a.gate_du = 0.24, a pressure ratio above 1.9 or a normal velocity jump
// above 0.48 of the mean sound speed, against 2 and 0.5 in the gate itself);
// the second pass applies the exact gate.  In the mixed path these are
// run-time values, so that the plain and the learned guess share one
// instance of the first pass.
template <typename T, bool LEARNED>
__device__ __forceinline__ bool hand_over(const FaceState<T> &fs, const FluxArgs &a) {
  if (fs.skip) return false;
  const T pL = fs.SL.p, pR = fs.SR.p;
  bool h = false;
  if (sizeof(T) == sizeof(float) && a.jump > 0.0f) {
    const T J = T(a.jump);
    h = fmax(pL, pR) > J * fmin(pL, pR) || fmax(fs.SL.r, fs.SR.r) > J * fmin(fs.SL.r, fs.SR.r) ||
        (fs.flags & F_POSITIVITY);
  }
  if (LEARNED || a.gate_p > 0.0f) {
    const T gp = T(a.gate_p);
    h = h || pL > gp * pR || pR > gp * pL ||
        fabs(fs.SR.u - fs.SL.u) > T(a.gate_du) * (fs.SL.c + fs.SR.c);
  }
  return h;
}

template <typename T, int SCHEME, int M, bool LEARNED>
__global__ void __launch_bounds__(FTH) __attribute__((amdgpu_waves_per_eu(2))) fluxes_k(FluxArgs a) {
  if (a.counters[C_STEP_SKIP]) return;  // the density pass was rejected
  __shared__ int pref[FBS + 1];
  __shared__ int wsum[FTH / 64];
  __shared__ double acc[5][FBS];
  const int64_t n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // a.split workgroups share a block, each taking one slice of its faces
  const int w = xcd_block(blockIdx.x, gridDim.x);
  const int slice = w % a.split;
  const int b0 = (w / a.split) * FBS;
  const int nb = (int)min((int64_t)FBS, n - b0);
  // block exclusive prefix sum of the per-particle face counts: each thread
  // sums PPT consecutive particles, then a wave scan and the wave offsets
  int cnt[PPT], tsum = 0;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int t = tid * PPT + q;
    cnt[q] = t < nb ? a.fcnt[b0 + t] : 0;
    tsum += cnt[q];
  }
  int incl = tsum;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wid] = incl;
  for (int t = tid; t < FBS; t += FTH) {
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[f][t] = 0.0;
  }
  __syncthreads();
  int run = incl - tsum;
  for (int w = 0; w < wid; ++w) run += wsum[w];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    pref[tid * PPT + q] = run;
    run += cnt[q];
  }
  if (tid == FTH - 1) pref[FBS] = run;
  __syncthreads();
  const int T_faces = pref[FBS];
  // a sub-step of individual time steps adds the block's sums to dQ: a block
  // without a face to solve has nothing to add
  if (a.R.rung && T_faces == 0) return;
  const int f_lo = (int)((int64_t)T_faces * slice / a.split);
  const int f_hi = (int)((int64_t)T_faces * (slice + 1) / a.split);
  if (slice > 0 && f_lo == f_hi) return;  // an empty slice adds nothing
  const double dt = a.dt[0] * a.inv_a;  // the step times 1/a (comoving)
  const T hdt = T(0.5 * dt);
  int64_t nfaces = 0, iters_sum = 0, vac = 0, pos = 0, maxit = 0, fb = 0, overflow = 0;
  // face f of the block: its particle p (pref[p] <= f < pref[p + 1]) and its
  // partner j, found one round ahead so that the partner's load is in flight
  // while the current face is solved
  auto locate = [&](int f, int &pf, int &jf) {
    int lo = 0, hi = FBS;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= f) lo = mid; else hi = mid;
    }
    pf = lo;
    jf = a.fslot[list_at(list_base(a.lseg, b0 + lo), f - pref[lo])];
  };
  int p_next = FBS, j_next = 0;
  if (f_lo + tid < f_hi) locate(f_lo + tid, p_next, j_next);
  for (int base = f_lo; base < f_hi; base += FTH) {
    const int f = base + tid;
    const bool active = f < f_hi;
    int p = FBS;  // sentinel key for idle lanes (they sit at the wave's end)
    int i = 0, j = 0;
    if (active) {
      p = p_next;
      j = j_next;
    }
    if (f + FTH < f_hi) locate(f + FTH, p_next, j_next);
    FaceState<T> fs;
    fs.skip = true;
    fs.flags = 0;
    bool defer = false;
    int Lslot = 0, Rslot = 0;
    double dtf = dt;  // this face's step
    if (active) {
      i = b0 + p;
      Lslot = i < j ? i : j;
      Rslot = i < j ? j : i;
      T hL = hdt, hR = hdt;
      face_step(a, Lslot, Rslot, dtf, hL, hR);
      FaceIn<T> Ls, Rs;
      load_side(a, Lslot, Ls);
      load_side(a, Rslot, Rs);
      // the particles' own jump (mixed path): where it is strong the face's
      // FP32 extrapolations and predictor lose accuracy even when the
      // reconstructed states have come close
      if (sizeof(T) == sizeof(float) && a.jump > 0.0f) {
        const T J = T(a.jump);
        defer = fmax(Ls.P, Rs.P) > J * fmin(Ls.P, Rs.P) ||
                fmax(Ls.rho, Rs.rho) > J * fmin(Ls.rho, Rs.rho);
      }
      face_prepare<T>(Ls, Rs, a, hL, hR, fs);
      if (LEARNED || sizeof(T) == sizeof(float)) defer = defer || hand_over<T, LEARNED>(fs, a);
    }
    if (LEARNED || sizeof(T) == sizeof(float)) {
      // queue the wave's handed-over faces with one atomic per wave, in the
      // segment of this workgroup; a face that finds the segment full is
      // solved here
      const uint64_t dmask = __ballot(defer);
      if (dmask) {
        const int seg = blockIdx.x % HARD_SEGS;
        const int leader = __ffsll((unsigned long long)dmask) - 1;
        unsigned long long base = 0;
        if (lane == leader)
          base = atomicAdd(a.hard_len + seg * HARD_SEG_STRIDE,
                           (unsigned long long)__popcll(dmask));
        base = __shfl(base, leader, 64);
        if (defer) {
          const unsigned long long below = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(dmask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)dmask, 0u));
          const unsigned long long slot = base + below;
          const unsigned long long seg_cap = (unsigned long long)(a.hard_cap / HARD_SEGS);
          if (slot < seg_cap) {
            a.hard_q[seg * (int64_t)seg_cap + (int64_t)slot] = make_int2(Lslot, Rslot);
          } else {
            defer = false;
            ++overflow;
          }
        }
      }
    }
    double c[5] = {0, 0, 0, 0, 0};
    if (active && !defer) {
      int it;
      double ps, pg;
      int br;
      face_solve<T, SCHEME, M>(fs, a, false, 0.0f, c, it, ps, pg, br);
#pragma unroll
      for (int q = 0; q < 5; ++q) c[q] *= dtf;
      if (SCHEME == MFM_SCHEME_MFV && a.gwork) add_gwork(a, Lslot, Rslot, c[0]);
      const double sgn = (i < j) ? -1.0 : 1.0;  // the left (lower) side loses c
#pragma unroll
      for (int q = 0; q < 5; ++q) c[q] *= sgn;
      const bool inb = (j >= b0) && (j < b0 + nb);
      if (inb) {
#pragma unroll
        for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q)
          atomicAdd(&acc[q][j - b0], -c[q]);
      } else {
        // the partner belongs to another block: its share goes to HBM
#pragma unroll
        for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q)
          unsafeAtomicAdd(&a.dq_ext[(int64_t)q * n + j], -c[q]);
      }
      {
        ++nfaces;
        iters_sum += it;
        vac += (fs.flags & F_VACUUM) ? 1 : 0;
        pos += (fs.flags & F_POSITIVITY) ? 1 : 0;
        maxit += (fs.flags & F_MAXIT) ? 1 : 0;
        fb += (fs.flags & F_FALLBACK) ? 1 : 0;
        if (a.dump) {
          const bool rec = !fs.skip && !(fs.flags & F_VACUUM);
          const unsigned long long slot = wave_slot(a.dump_count, rec, lane);
          if (rec && slot < (unsigned long long)a.dump_cap) {
            float x[mlp::NIN];
            features_of<T>(fs, pg, br, x);
            float *r = a.dump + slot * 8;
#pragma unroll
            for (int k = 0; k < mlp::NIN; ++k) r[k] = x[k];
            r[6] = logf((float)(ps / pg));
            r[7] = (float)it;
          }
        }
      }
    }
    if (active && !defer) {
#pragma unroll
      for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q) atomicAdd(&acc[q][p], c[q]);
    }
    if (defer) ++nfaces;  // counted here, solved in the second pass
  }
  __syncthreads();
  for (int t = tid; t < nb; t += FTH) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (slice == 0 && !a.R.rung) {
        a.dQ[(int64_t)q * n + b0 + t] = acc[q][t];
      } else if (acc[q][t] != 0.0) {
        // the other slices of the block add theirs through dq_ext; on a
        // sub-step of individual steps dq_ext is dQ itself, where the sums
        // of a particle's whole step accumulate
        unsafeAtomicAdd(&a.dq_ext[(int64_t)q * n + b0 + t], acc[q][t]);
      }
    }
  }
  count_add(a.counters + C_FACES, nfaces);
  count_add(a.counters + C_RIEMANN_ITERS, iters_sum);
  count_add(a.counters + C_VACUUM, vac);
  count_add(a.counters + C_POSITIVITY, pos);
  count_add(a.counters + C_RIEMANN_MAXIT, maxit);
  count_add(a.counters + C_GUESS_FALLBACK, fb);
  count_add(a.counters + C_HARD_OVERFLOW, overflow);
}

// One side of a face in FP64 for the second pass.  The mixed path's record is
// FP32: the particle's own values come from the FP64 particle arrays instead,
// B and the gradients (computed in FP32) are widened.
template <bool F32REC>
__device__ __forceinline__ void load_side64(const FluxArgs &a, int i, FaceIn<double> &s) {
  if (!F32REC) {
    load_side(a, i, s);
    return;
  }
  const float4 *r = reinterpret_cast<const float4 *>(a.rec) + (int64_t)i * (F_STRIDE / 4);
  float f[F_STRIDE];
#pragma unroll
  for (int k = 2; k < F_STRIDE / 4; ++k) {
    const float4 q = r[k];
    f[4 * k] = q.x; f[4 * k + 1] = q.y; f[4 * k + 2] = q.z; f[4 * k + 3] = q.w;
  }
  static_assert(F_B == 8, "B and the gradients start at the third float4 of the record");
  if (a.R.rung) {
    const double4 p = a.pos[i];  // the position of this sub-step
    s.x = p.x; s.y = p.y; s.z = p.z;
  } else {
    s.x = a.x[i]; s.y = a.y[i]; s.z = a.z[i];
  }
  s.ih = 1.0 / a.H[i];
  s.V = a.V[i];
  s.rho = a.rho[i];
  s.irho = 1.0 / s.rho;
  s.v[0] = a.vx[i]; s.v[1] = a.vy[i]; s.v[2] = a.vz[i];
  s.P = a.P[i];
#pragma unroll
  for (int k = 0; k < 6; ++k) s.B[k] = f[F_B + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) s.G[k] = f[F_G + k];
}

// Second pass of the flux loop: the handed-over faces, one per lane, in FP64
// (and, with the learned guess, the network's starting value for those that
// pass its gate).  Both sides receive their share through FP64 atomics into
// dq_ext, which is folded into dQ after this pass.  The queue length is read
// on the device; the grid strides over it.
//
// With the learned guess the network's weights and vectors are first copied
// to LDS.  A short queue (the usual case: well under 1% of the faces) leaves
// the pass bound by the latency of a wavefront's work; a wavefront then
// takes 16 faces (lanes 0..15), so that the network runs on a single 16-row
// tile and four times as many wavefronts share the queue.  A long queue
// (more than four rounds of the grid at 16 faces per wavefront) is taken 64
// faces per wavefront, the network on its four tiles in turn.
template <bool F32REC, int SCHEME, int M, bool LEARNED>
__global__ void __launch_bounds__(FTH) hard_faces_k(FluxArgs a) {
  if (a.counters[C_STEP_SKIP]) return;  // the density pass was rejected
  constexpr int FTW = FTH / 64;  // wavefronts per workgroup
  __shared__ uint16_t mlp_act[LEARNED ? FTW * 16 * mlp::AST : 1];
  __shared__ __align__(16) uint16_t mlp_w[LEARNED ? mlp::NT : 1];
  __shared__ float mlp_v[LEARNED ? mlp::NVEC : 1];
  __shared__ int64_t seg_off[HARD_SEGS + 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // the segments laid end to end: face g of the pass is entry g - seg_off[s]
  // of the segment s with seg_off[s] <= g < seg_off[s + 1]
  const int64_t seg_cap = a.hard_cap / HARD_SEGS;
  if (tid < HARD_SEGS) {
    const unsigned long long len = a.hard_len[tid * HARD_SEG_STRIDE];
    seg_off[tid + 1] = (int64_t)(len < (unsigned long long)seg_cap ? len
                                                                    : (unsigned long long)seg_cap);
  }
  __syncthreads();
  if (tid == 0) {
    seg_off[0] = 0;
    for (int s = 0; s < HARD_SEGS; ++s) seg_off[s + 1] += seg_off[s];
  }
  __syncthreads();
  const int64_t nq = seg_off[HARD_SEGS];
  // faces per wave: 16 while that takes at most four rounds of the grid
  const int fpw = (LEARNED && nq <= 4 * (int64_t)gridDim.x * FTW * 16) ? 16 : 64;
  const int fpb = FTW * fpw;  // faces per workgroup and round
  mlp::Vecs vecs{};
  if (LEARNED) {
    if ((int64_t)blockIdx.x * fpb >= nq) return;  // no face for this workgroup
    vecs = mlp::stage_net(a.net, mlp_w, mlp_v, tid, FTH);
    __syncthreads();
  }
  const double dt = a.dt[0] * a.inv_a;  // the step times 1/a (comoving)
  const double hdt = 0.5 * dt;
  const int64_t n = a.n;
  int64_t nfaces = 0, iters_sum = 0, vac = 0, pos = 0, maxit = 0, fb = 0;
  for (int64_t base = (int64_t)blockIdx.x * fpb; base < nq; base += (int64_t)gridDim.x * fpb) {
    const int64_t g = base + wid * fpw + lane;
    const bool active = lane < fpw && g < nq;
    FaceState<double> fs;
    fs.skip = true;
    fs.flags = 0;
    int L = 0, R = 0;
    double dtf = dt;
    if (active) {
      int s = 0;  // the segment holding g: a binary search over the offsets
#pragma unroll
      for (int step = HARD_SEGS / 2; step > 0; step >>= 1)
        if (seg_off[s + step] <= g) s += step;
      const int2 q = a.hard_q[s * seg_cap + (g - seg_off[s])];
      L = q.x;
      R = q.y;
      double hL = hdt, hR = hdt;
      face_step(a, L, R, dtf, hL, hR);
      FaceIn<double> Ls, Rs;
      load_side64<F32REC>(a, L, Ls);
      load_side64<F32REC>(a, R, Rs);
      face_prepare<double>(Ls, Rs, a, hL, hR, fs);
    }
    bool use_net = false;
    float y = 0.f;
    if (LEARNED) {
      // a wavefront holding a face that passes the gate evaluates the
      // network on all its faces (wave-uniform branch)
      float x[mlp::NIN];
      bool gated = false;
      if (active && !fs.skip) {
        int br0;
        const double p0 = floored_guess<double, M>(a.G, fs.SL, fs.SR, br0);
        features_of<double>(fs, p0, br0, x);
        gated = mlp::needs_guess(x);
      }
      if (__ballot(gated)) {
        uint16_t *tile = mlp_act + wid * 16 * mlp::AST;
        float yw;
        if (fpw == 16) {
          if (lane < 16) mlp::put_input(tile, lane, gated ? x : nullptr, vecs.norm);
          yw = mlp::forward_rows(tile, mlp_w, vecs, lane);
        } else {
          yw = mlp::forward_wave(tile, gated ? x : nullptr, mlp_w, vecs, lane);
        }
        use_net = gated;
        y = yw;
      }
    }
    if (active) {
      double c[5];
      int it;
      double ps, pg;
      int br;
      face_solve<double, SCHEME, M>(fs, a, use_net, y, c, it, ps, pg, br);
#pragma unroll
      for (int q = (SCHEME == MFM_SCHEME_MFM ? 1 : 0); q < 5; ++q) {
        unsafeAtomicAdd(&a.dq_ext[(int64_t)q * n + L], -dtf * c[q]);
        unsafeAtomicAdd(&a.dq_ext[(int64_t)q * n + R], dtf * c[q]);
      }
      if (SCHEME == MFM_SCHEME_MFV && a.gwork) add_gwork(a, L, R, dtf * c[0]);
      ++nfaces;
      iters_sum += it;
      vac += (fs.flags & F_VACUUM) ? 1 : 0;
      pos += (fs.flags & F_POSITIVITY) ? 1 : 0;
      maxit += (fs.flags & F_MAXIT) ? 1 : 0;
      fb += (fs.flags & F_FALLBACK) ? 1 : 0;
      if (a.dump) {
        const bool rec = !fs.skip && !(fs.flags & F_VACUUM);
        const unsigned long long slot = wave_slot(a.dump_count, rec, lane);
        if (rec && slot < (unsigned long long)a.dump_cap) {
          float x[mlp::NIN];
          features_of<double>(fs, pg, br, x);
          float *r = a.dump + slot * 8;
#pragma unroll
          for (int k = 0; k < mlp::NIN; ++k) r[k] = x[k];
          r[6] = logf((float)(ps / pg));
          r[7] = (float)it;
        }
      }
    }
  }
  count_add(a.counters + C_HARD_FACES, nfaces);
  count_add(a.counters + C_RIEMANN_ITERS, iters_sum);
  count_add(a.counters + C_VACUUM, vac);
  count_add(a.counters + C_POSITIVITY, pos);
  count_add(a.counters + C_RIEMANN_MAXIT, maxit);
  count_add(a.counters + C_GUESS_FALLBACK, fb);
}

// dq_ext (and the second pass's queue length) is cleared before the flux
// loop and folded into dQ after it (on a sub-step of individual steps only
// the queue length: the shares go straight into dQ).
__global__ void zero_f64_k(double *v, int64_t m, unsigned long long *queue_len,
                           const int64_t *counters, double *w, int64_t mw) {
  if (counters[C_STEP_SKIP]) return;
  if (blockIdx.x == 0 && threadIdx.x < HARD_SEGS) queue_len[threadIdx.x * HARD_SEG_STRIDE] = 0ull;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x)
    v[k] = 0.0;
  if (w)
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < mw;
         k += (int64_t)gridDim.x * blockDim.x)
      w[k] = 0.0;
}
__global__ void fold_f64_k(double *dst, const double *src, int64_t m, const int64_t *counters) {
  if (counters[C_STEP_SKIP]) return;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] += src[k];
}

template <typename T, int SCHEME, bool LEARNED>
void launch_m(const FluxArgs &a, int m, int nb, hipStream_t st) {
  if (m == 5)
    fluxes_k<T, SCHEME, 5, LEARNED><<<nb, FTH, 0, st>>>(a);
  else if (m == 7)
    fluxes_k<T, SCHEME, 7, LEARNED><<<nb, FTH, 0, st>>>(a);
  else
    fluxes_k<T, SCHEME, 0, LEARNED><<<nb, FTH, 0, st>>>(a);
}

template <typename T, bool LEARNED>
void launch_t(const FluxArgs &a, int scheme, int m, int nb, hipStream_t st) {
  if (scheme == MFM_SCHEME_MFM)
    launch_m<T, MFM_SCHEME_MFM, LEARNED>(a, m, nb, st);
  else
    launch_m<T, MFM_SCHEME_MFV, LEARNED>(a, m, nb, st);
}

template <bool F32REC, int SCHEME, bool LEARNED>
void launch_hard_m(const FluxArgs &a, int m, int nb, hipStream_t st) {
  if (m == 5)
    hard_faces_k<F32REC, SCHEME, 5, LEARNED><<<nb, FTH, 0, st>>>(a);
  else if (m == 7)
    hard_faces_k<F32REC, SCHEME, 7, LEARNED><<<nb, FTH, 0, st>>>(a);
  else
    hard_faces_k<F32REC, SCHEME, 0, LEARNED><<<nb, FTH, 0, st>>>(a);
}

template <bool F32REC, bool LEARNED>
void launch_hard(const FluxArgs &a, int scheme, int m, int nb, hipStream_t st) {
  if (scheme == MFM_SCHEME_MFM)
    launch_hard_m<F32REC, MFM_SCHEME_MFM, LEARNED>(a, m, nb, st);
  else
    launch_hard_m<F32REC, MFM_SCHEME_MFV, LEARNED>(a, m, nb, st);
}

template <typename T>
Gas<T> make_gas(double g) {
  Gas<T> G;
  G.gamma = T(g);
  G.g1 = T((g - 1.0) / (2.0 * g));
  G.g2 = T((g + 1.0) / (2.0 * g));
  G.g3 = T(2.0 * g / (g - 1.0));
  G.g4 = T(2.0 / (g - 1.0));
  G.g5 = T(2.0 / (g + 1.0));
  G.g6 = T((g - 1.0) / (g + 1.0));
  G.g7 = T(0.5 * (g - 1.0));
  G.inv_gm1 = T(1.0 / (g - 1.0));
  G.sg5 = T(sqrt(2.0 / (g + 1.0)));
  return G;
}

}  // namespace

hipError_t launch_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  FluxArgs a;
  a.n = pp->n;
  a.rec = ctx->rec;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.fslot = ctx->fslot;
  a.lseg = ctx->lseg;
  a.fcnt = ctx->fcnt;
  a.dt = dt_dev;
  a.dQ = pp->dQ;
  for (int k = 0; k < 3; ++k) {
    a.box[k] = ctx->p.box[k];
    a.half[k] = 0.5 * ctx->p.box[k];
  }
  const double g = ctx->p.gamma;
  a.G = make_gas<double>(g);
  a.Gf = make_gas<float>(g);
  // root path when 1/g1 = 2 gamma / (gamma - 1) is an integer m (gamma = m/(m-2))
  const double mm = 2.0 * g / (g - 1.0);
  const int mi = (int)(mm + 0.5);
  const int m = (mi >= 3 && mi <= 16 && fabs(mm - mi) < 1e-12 * mm) ? mi : 0;
  a.psi1 = ctx->p.psi1;
  a.psi2 = ctx->p.psi2;
  a.rtol = ctx->p.riemann_tol;
  a.rtol_f = 1e-6f;  // FP32 Newton tolerance of the mixed path (the FP64 check follows)
  a.rmaxit = ctx->p.riemann_maxit;
  a.limiter = ctx->p.limiter;
  a.counters = ctx->counters;
  a.dump = ctx->dump;
  a.dump_cap = ctx->dump_cap;
  a.dump_count = ctx->dump_count;
  // individual steps: every share goes straight into dQ, which holds the
  // sums of the whole base step (nothing to clear or fold per sub-step)
  a.dq_ext = ctx->rungs.rung ? pp->dQ : ctx->dq_ext;
  a.hard_q = ctx->hard_q;
  a.hard_cap = ctx->hard_cap;
  a.hard_len = ctx->hard_len;
  a.jump = (float)ctx->p.mixed_jump;
  a.x = pp->x; a.y = pp->y; a.z = pp->z; a.H = pp->H; a.V = pp->V; a.rho = pp->rho;
  a.vx = pp->vx; a.vy = pp->vy; a.vz = pp->vz; a.P = pp->P;
  a.inv_a = ctx->inv_a;
  a.gwork = (pp->accel && ctx->p.scheme == MFM_SCHEME_MFV) ? ctx->gwork : nullptr;
  a.R = ctx->rungs;
  const bool learned = ctx->p.guess == MFM_GUESS_LEARNED;
  const bool mixed = ctx->p.precision == MFM_MIXED;
  if (learned) mlp_net_of(ctx->mlp_state, &a.net);
  a.gate_p = learned ? 1.9f : 0.0f;
  a.gate_du = learned ? 0.24f : 0.0f;
  // a set of few blocks (under FLUX_WG_TARGET) splits each block's faces
  // over several workgroups so that the chip fills; a sub-step of individual
  // steps keeps one workgroup per block (most of them have no face to solve)
  const int nblk = blocks_for(pp->n, FBS);
  a.split = ctx->rungs.rung ? 1 : std::max(1, std::min(FLUX_MAX_SPLIT, FLUX_WG_TARGET / nblk));
  const int nb = nblk * a.split;
  const int64_t m5 = 5 * pp->n;
  const int fb = (int)std::min<int64_t>(blocks_for(m5, 256), 8192);
  const int ev_all = stage_begin(ctx, 4);
  zero_f64_k<<<ctx->rungs.rung ? 1 : fb, 256, 0, ctx->stream>>>(ctx->rungs.rung ? nullptr : ctx->dq_ext,
                                          ctx->rungs.rung ? 0 : m5, a.hard_len, ctx->counters,
                                          a.gwork, 3 * pp->n);
  const int ev_main = stage_begin(ctx, 6);
  if (mixed) {
    launch_t<float, false>(a, ctx->p.scheme, m, nb, ctx->stream);  // learned: a.gate_*
  } else {
    if (learned)
      launch_t<double, true>(a, ctx->p.scheme, m, nb, ctx->stream);
    else
      launch_t<double, false>(a, ctx->p.scheme, m, nb, ctx->stream);
  }
  stage_end(ctx, ev_main);
  if (mixed || learned) {
    // the second pass strides over the queue with a grid of its own (its
    // length is known only on the device); an empty queue ends it at once
    const int hb = 2048;
    const int ev_hard = stage_begin(ctx, 7);
    if (mixed) {
      if (learned) launch_hard<true, true>(a, ctx->p.scheme, m, hb, ctx->stream);
      else launch_hard<true, false>(a, ctx->p.scheme, m, hb, ctx->stream);
    } else {
      launch_hard<false, true>(a, ctx->p.scheme, m, hb, ctx->stream);
    }
    stage_end(ctx, ev_hard);
  }
  if (!ctx->rungs.rung)
    fold_f64_k<<<fb, 256, 0, ctx->stream>>>(pp->dQ, ctx->dq_ext, m5, ctx->counters);
  stage_end(ctx, ev_all);
  return hipGetLastError();
}
