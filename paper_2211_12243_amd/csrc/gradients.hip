// gradients.hip -- loops (2) and (4) of the scheme: the renormalised
// (Lanson-Vila) gradients with the conditioned slope limiter (sec. 2.3.3 and
// 2.3.6) and the CFL time step (sec. 2.3.10), then the global minimum step.
//
// One lane per particle over its candidate list.  Each neighbour (r < H_i)
// is gathered as one 128-byte record written by the density loop.  Pass one
// accumulates E_i, the five gradient sums, the neighbour extrema and the
// signal velocity, and records the faces this particle will evaluate in the
// flux loop; B_i = E_i^-1 is the cofactor inverse; pass two finds the extreme
// face extrapolations for the limiter.  The particle's flux record is written
// packed: 256 bytes in FP64 (positions included), 128 bytes in the mixed
// path (FP32; positions stay FP64 in the separate position array).
//
// Precision.  T = double is the FP64 path.  T = float is the mixed path: the
// separation is formed in FP64 and rounded, every pair term and sum is FP32;
// an E_i whose FP32 condition number exceeds MIXED_FP64_NCOND is inverted
// in FP64 (and the gradients formed with that inverse), as are the outputs
// kept in FP64 arrays.
#include "mfm_internal.h"
#include "lanes.h"

namespace {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 1024;
constexpr double PI = 3.14159265358979323846;
constexpr float MIXED_FP64_NCOND = 10.0f;
// Face slots leave through a ring of RING planes per wavefront in LDS: a
// lane appends at its own rate, and a plane is stored (64 consecutive
// particles, one 256-byte write) once every lane has passed it.  A lone
// 4-byte store per lane into separate planes cost a full sector of HBM
// write each (measured 1.6 GB written per launch instead of 0.8).
constexpr int RING = 16;
constexpr int RSTEP = 4;  // list entries between two looks at the ring's fill

struct GradArgs {
  int64_t n;
  const double *gin;
  const double *H;      // converged support radii (SoA: 16 particles per cache line)
  // (x, y, z, H) per particle: this pass's positions (on a sub-step of
  // individual steps, every particle's at that time)
  const double4 *pos;
  const int32_t *cand, *cand_cnt;  // candidates with r >= H_i
  const float *rest_r2;             // their r^2, rounded to FP32
  const int32_t *gl, *gl_cnt;
  const int64_t *lseg;  // list blocks of the chunks (list_at)
  double *B, *grad, *ncond, *dt_i, *rec;
  int32_t *fslot, *fcnt;
  double box[3], half[3];
  double ncond_max, c_cfl;
  int limiter;
  int64_t *counters;
  const double *m;  // masses, for E_kin^max
  double *ekm;      // E_kin^max = max_j m_i |v_j - v_i|^2 / 2 (null: not wanted)
  int32_t *grad_q;  // mixed path: particles whose E is redone in FP64 (grad_fix_k)
  const uint8_t *act;  // individual steps: 1 for the particles whose step begins (null: all)
};

template <typename T>
__device__ __forceinline__ T spline_wt(T q) {
  if (q < T(0.5)) return T(1) + q * q * (T(6) * q - T(6));
  if (q < T(1)) {
    const T t = T(1) - q;
    return T(2) * t * t * t;
  }
  return T(0);
}

// Inverse of a symmetric 3x3 (xx,xy,xz,yy,yz,zz) by cofactors; returns the determinant.
template <typename T>
__device__ __forceinline__ T sym_inv(const T e[6], T b[6]) {
  T cf[6];
  cf[0] = e[3] * e[5] - e[4] * e[4];
  cf[1] = e[2] * e[4] - e[1] * e[5];
  cf[2] = e[1] * e[4] - e[2] * e[3];
  cf[3] = e[0] * e[5] - e[2] * e[2];
  cf[4] = e[1] * e[2] - e[0] * e[4];
  cf[5] = e[0] * e[3] - e[1] * e[1];
  const T det = e[0] * cf[0] + e[1] * cf[1] + e[2] * cf[2];
#pragma unroll
  for (int k = 0; k < 6; ++k) b[k] = cf[k] / det;
  return det;
}

template <typename T>
__device__ __forceinline__ T sym_frob(const T a[6]) {
  return sqrt(a[0] * a[0] + a[3] * a[3] + a[5] * a[5] +
              T(2) * (a[1] * a[1] + a[2] * a[2] + a[4] * a[4]));
}

template <typename T>
__device__ __forceinline__ void sym_apply(const T b[6], const T s[3], T g[3]) {
  g[0] = b[0] * s[0] + b[1] * s[1] + b[2] * s[2];
  g[1] = b[1] * s[0] + b[3] * s[1] + b[4] * s[2];
  g[2] = b[2] * s[0] + b[4] * s[1] + b[5] * s[2];
}

// What the first loop gathers of one neighbour's record: the FP64 position
// and velocity and, on the mixed path, the FP32 tail (V, rho, P, c); on the
// FP64 path the FP64 values.  The velocity stays FP64 on the mixed path for
// the same reason as the position: a bulk flow much faster than the
// velocity differences across the kernel would leave those differences to
// the rounding of FP32 copies.
template <typename T> struct NbRec;
template <> struct NbRec<float> {
  double x, y, z, vx, vy, vz;
  float4 f0;
  __device__ __forceinline__ void load(const double *gj) {
    x = gj[GIN_X]; y = gj[GIN_Y]; z = gj[GIN_Z];
    vx = gj[GIN_VX]; vy = gj[GIN_VY]; vz = gj[GIN_VZ];
    f0 = *reinterpret_cast<const float4 *>(gj + GIN_F32);
  }
  __device__ __forceinline__ void values(double q[5], float &v, float &c) const {
    v = f0.x;
    q[0] = f0.y; q[1] = vx; q[2] = vy; q[3] = vz; q[4] = f0.z;
    c = f0.w;
  }
};
template <> struct NbRec<double> {
  double x, y, z, v, q[5], c;
  __device__ __forceinline__ void load(const double *gj) {
    x = gj[GIN_X]; y = gj[GIN_Y]; z = gj[GIN_Z];
    v = gj[GIN_V];
    q[0] = gj[GIN_RHO]; q[1] = gj[GIN_VX]; q[2] = gj[GIN_VY]; q[3] = gj[GIN_VZ]; q[4] = gj[GIN_P];
    c = gj[GIN_C];
  }
  __device__ __forceinline__ void values(double qo[5], double &vo, double &co) const {
    vo = v;
#pragma unroll
    for (int k = 0; k < 5; ++k) qo[k] = q[k];
    co = c;
  }
};

// A neighbour's record.  On a sub-step of individual steps (RUNG) its
// position comes from pos, where the sub-step start has put every particle
// at that time (gin keeps the position of the particle's last density pass).
template <bool RUNG, typename T>
__device__ __forceinline__ void load_nb(NbRec<T> &nb, const GradArgs &a, int64_t j) {
  nb.load(a.gin + j * GIN_STRIDE);
  if (RUNG) {
    const double4 p = a.pos[j];
    nb.x = p.x;
    nb.y = p.y;
    nb.z = p.z;
  }
}

template <typename T, bool RUNG>
__global__ void __launch_bounds__(BS) gradients_k(GradArgs a) {
  if (a.counters[C_STEP_SKIP]) return;  // the density pass was rejected
  __shared__ int32_t s_ring[BS / 64][RING][64];
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = a.n;
  int64_t pairs = 0, singular = 0, inv64 = 0;
  // every lane runs the loops below (the ring's plane bookkeeping is a
  // wavefront reduction); a lane past the end works on particle 0 and
  // writes nothing
  // a particle in mid-step (individual steps) keeps its gradients and has no
  // faces of its own: its faces are solved by the particles whose step begins
  const bool live = i < n && (!a.act || a.act[i]);
  if (i < n && !live) a.fcnt[i] = 0;
  // on a sub-step most wavefronts hold no such particle: they are done
  if (a.act && !__ballot(live)) return;
  const int64_t lb = list_base(a.lseg, live ? i : 0);
  {
    const double *gi = a.gin + (live ? i : 0) * GIN_STRIDE;
    const double xi = gi[GIN_X], yi = gi[GIN_Y], zi = gi[GIN_Z], hi = gi[GIN_H];
    const double h2 = hi * hi;
    const T ih = T(1.0 / hi), wnorm = T(8.0 / (PI * hi * h2));
    // the primitives stay FP64 so that differences and extrema are exact before
    // the FP32 pair arithmetic of the mixed path
    const double q64[5] = {gi[GIN_RHO], gi[GIN_VX], gi[GIN_VY], gi[GIN_VZ], gi[GIN_P]};
    const T qi[5] = {T(q64[0]), T(q64[1]), T(q64[2]), T(q64[3]), T(q64[4])};
    const T ci = T(gi[GIN_C]);
    T e[6] = {0, 0, 0, 0, 0, 0};
    T s[5][3];
    double qmax[5], qmin[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s[q][0] = s[q][1] = s[q][2] = T(0);
      qmax[q] = qmin[q] = q64[q];
    }
    T vsig = T(0);
    double dv2max = 0.0;  // max_j |v_j - v_i|^2 over the gather set (E_kin^max)
    int nf = 0;
    // the face ring: planes [0, flushed) are stored; a lane's face number nf
    // >= flushed sits in slot nf % RING, one below flushed (a lane that fell
    // behind a forced store) goes straight to HBM
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    int flushed = 0;
    auto put_face = [&](int j) {
      if (nf >= flushed)
        s_ring[wv][nf % RING][ln] = j;
      else
        a.fslot[list_at(lb, nf)] = j;
      ++nf;
    };
    auto store_plane = [&](int p) {
      if (live && nf > p) a.fslot[list_at(lb, p)] = s_ring[wv][p % RING][ln];
    };
    // before RSTEP list entries (at most one face each per lane): keep every
    // slot they may take inside the ring
    auto make_room = [&]() {
      const int hi = lanes::wave_max_i32(nf);
      while (hi + RSTEP > flushed + RING) store_plane(flushed++);
    };
    // after it: store the planes every lane has passed
    auto store_done = [&]() {
      const int lo = lanes::wave_min_i32(live ? nf : 0x7fffffff);
      while (flushed < lo) store_plane(flushed++);
    };
    // faces of the flux loop: r < max(H_i, H_j); one evaluation per face
    // inside a block, one per side across blocks.
    // (1) the gather set r < H_i (the density loop's compact list, in
    // candidate order): every member is also a face
    const int gc = live ? a.gl_cnt[i] : 0;
    const int gmax = lanes::wave_max_i32(gc);
    // the first loop runs two entries ahead for the list index and one ahead
    // for the neighbour's record, so that a gather is in flight while the
    // previous entry is summed; the others load their next entry one
    // iteration ahead
    int jn = gc > 0 ? a.gl[list_at(lb, 0)] : 0;
    int jn2 = gc > 1 ? a.gl[list_at(lb, 1)] : 0;
    NbRec<T> nb;
    bool nact = true;  // on a sub-step: the next neighbour's active flag, with its record
    if (gc > 0) {
      load_nb<RUNG>(nb, a, jn);
      if (RUNG) nact = a.act[jn] != 0;
    }
    for (int k = 0; k < gmax; ++k) {
      if (k % RSTEP == 0) make_room();
      if (k < gc) {
        const int j = jn;
        const NbRec<T> cur = nb;
        const bool jact = nact;
        if (k + 1 < gc) {
          jn = jn2;
          load_nb<RUNG>(nb, a, jn);
          if (RUNG) nact = a.act[jn] != 0;
          if (k + 2 < gc) jn2 = a.gl[list_at(lb, k + 2)];
        }
        if (emit_face((int)i, j) || (RUNG && !jact)) put_face(j);
        ++pairs;
        const double e0 = min_image(cur.x - xi, a.box[0], a.half[0]);
        const double e1 = min_image(cur.y - yi, a.box[1], a.half[1]);
        const double e2 = min_image(cur.z - zi, a.box[2], a.half[2]);
        const double r2 = e0 * e0 + e1 * e1 + e2 * e2;
        // neighbour values: FP64 on the FP64 path; on the mixed path their FP32
        // copies (half the bytes through the cache; the separation stays FP64)
        double qj[5];
        T vj, cj;
        cur.values(qj, vj, cj);
        {
          const double w0 = qj[1] - q64[1], w1 = qj[2] - q64[2], w2 = qj[3] - q64[3];
          dv2max = fmax(dv2max, w0 * w0 + w1 * w1 + w2 * w2);
        }
        if (r2 != 0.0) {
          const T d0 = T(e0), d1 = T(e1), d2 = T(e2);
          const T r = T(sqrt(r2));
          const T wv = vj * wnorm * spline_wt<T>(r * ih);
          e[0] += wv * d0 * d0;
          e[1] += wv * d0 * d1;
          e[2] += wv * d0 * d2;
          e[3] += wv * d1 * d1;
          e[4] += wv * d1 * d2;
          e[5] += wv * d2 * d2;
          T dq[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            dq[q] = T(qj[q] - q64[q]);
            const T df = wv * dq[q];
            s[q][0] += df * d0;
            s[q][1] += df * d1;
            s[q][2] += df * d2;
            qmax[q] = fmax(qmax[q], qj[q]);
            qmin[q] = fmin(qmin[q], qj[q]);
          }
          // signal velocity: x_i - x_j = -d
          const T proj = (d0 * dq[1] + d1 * dq[2] + d2 * dq[3]) / r;
          vsig = fmax(vsig, ci + cj - fmin(T(0), proj));
        }
      }
      if (k % RSTEP == RSTEP - 1) store_done();
    }
    // (2) faces with H_i <= r < H_j, from the other candidates (r >= H_i).
    // Their r^2 is stored in FP32 (relative error <= 2^-24): a neighbour
    // clearly inside or outside H_j is decided from it, one within a band of
    // 2^-22 around H_j^2 from the exact FP64 r^2 of the positions.
    const int cnt = live ? a.cand_cnt[i] : 0;
    const int cmax = lanes::wave_max_i32(cnt);
    // the list entry two ahead, the neighbour's H (and on a sub-step its
    // active flag) one ahead, so that no load is waited for in the
    // iteration that issues it
    int cj = cnt > 0 ? a.cand[list_at(lb, 0)] : 0;
    float cr = cnt > 0 ? a.rest_r2[list_at(lb, 0)] : 0.0f;
    int cj2 = cnt > 1 ? a.cand[list_at(lb, 1)] : 0;
    float cr2 = cnt > 1 ? a.rest_r2[list_at(lb, 1)] : 0.0f;
    double ch = cnt > 0 ? a.H[cj] : 0.0;
    bool cact = RUNG && cnt > 0 ? a.act[cj] != 0 : true;
    for (int k = 0; k < cmax; ++k) {
      if (k % RSTEP == 0) make_room();
      if (k < cnt) {
        const int j = cj;
        const double r2f = (double)cr;
        const double hj = ch;
        const bool jact = cact;
        if (k + 1 < cnt) {
          cj = cj2;
          cr = cr2;
          ch = a.H[cj];
          if (RUNG) cact = a.act[cj] != 0;
          if (k + 2 < cnt) {
            cj2 = a.cand[list_at(lb, k + 2)];
            cr2 = a.rest_r2[list_at(lb, k + 2)];
          }
        }
        const double hj2 = hj * hj;
        bool in = r2f < hj2 * (1.0 - 0x1p-22) && r2f > 1e-30;
        if (!in && !(r2f > hj2 * (1.0 + 0x1p-22) && r2f > 1e-30)) {
          const double4 pj = a.pos[j];
          const double e0 = min_image(pj.x - xi, a.box[0], a.half[0]);
          const double e1 = min_image(pj.y - yi, a.box[1], a.half[1]);
          const double e2 = min_image(pj.z - zi, a.box[2], a.half[2]);
          in = e0 * e0 + e1 * e1 + e2 * e2 < hj2;
        }
        if (in && (emit_face((int)i, j) || (RUNG && !jact))) put_face(j);
      }
      if (k % RSTEP == RSTEP - 1) store_done();
    }
    for (const int top = lanes::wave_max_i32(nf); flushed < top;) store_plane(flushed++);
    T b[6];
    T det = sym_inv<T>(e, b);
    T nc = sym_frob<T>(b) * sym_frob<T>(e) / T(3);
    T g[5][3];
    double b64[6];
    if (sizeof(T) == sizeof(float) && !(nc <= T(MIXED_FP64_NCOND))) {
      // ill-conditioned E in the mixed path: invert it in FP64
      double e64[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) e64[k] = (double)e[k];
      const double det64 = sym_inv<double>(e64, b64);
      det = T(det64);
      nc = T(sym_frob<double>(b64) * sym_frob<double>(e64) / 3.0);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double s64[3] = {(double)s[q][0], (double)s[q][1], (double)s[q][2]}, g64[3];
        sym_apply<double>(b64, s64, g64);
        g[q][0] = T(g64[0]);
        g[q][1] = T(g64[1]);
        g[q][2] = T(g64[2]);
      }
      if (live) ++inv64;
    } else {
#pragma unroll
      for (int q = 0; q < 5; ++q) sym_apply<T>(b, s[q], g[q]);
#pragma unroll
      for (int k = 0; k < 6; ++k) b64[k] = (double)b[k];
    }
    if (live && (!(det != T(0)) || !isfinite(det))) ++singular;
    if (sizeof(T) == sizeof(float)) {
      // an ill-conditioned E: FP32 sums leave B, the gradients and the
      // limiter to rounding amplified by the condition number; grad_fix_k
      // redoes the particle in FP64 after this launch
      const bool redo = live && !(nc <= T(MIXED_FP64_NCOND));
      const uint64_t m = __ballot(redo);
      int base = 0;
      if (m && (threadIdx.x & 63) == 0)
        base = (int)atomicAdd((unsigned long long *)(a.counters + C_GRAD_QUEUE),
                              (unsigned long long)__popcll(m));
      base = __shfl(base, 0, 64);
      if (redo) {
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        a.grad_q[base + rank] = (int32_t)i;
      }
    }
    T alpha[5] = {T(1), T(1), T(1), T(1), T(1)};
    if (a.limiter & MFM_LIMIT_BJ) {
      T dmax[5] = {0, 0, 0, 0, 0}, dmin[5] = {0, 0, 0, 0, 0};
      int bn = gc > 1 ? a.gl[list_at(lb, 1)] : 0;
      double4 pn = gc > 0 ? a.pos[a.gl[list_at(lb, 0)]] : make_double4(0, 0, 0, 0);
      for (int k = 0; k < gc; ++k) {
        const double4 pj = pn;
        if (k + 1 < gc) {
          pn = a.pos[bn];
          if (k + 2 < gc) bn = a.gl[list_at(lb, k + 2)];
        }
        const T d0 = T(min_image(pj.x - xi, a.box[0], a.half[0]));
        const T d1 = T(min_image(pj.y - yi, a.box[1], a.half[1]));
        const T d2 = T(min_image(pj.z - zi, a.box[2], a.half[2]));
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const T ex = T(0.5) * (g[q][0] * d0 + g[q][1] * d1 + g[q][2] * d2);
          dmax[q] = fmax(dmax[q], ex);
          dmin[q] = fmin(dmin[q], ex);
        }
      }
      T t = (T(a.ncond_max) - nc) / (T(a.ncond_max) - T(1));
      t = t > T(0) ? (t < T(1) ? t : T(1)) : T(0);
      const T beta = T(1) + t;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        T rp = T(__builtin_huge_val()), rm = T(__builtin_huge_val());
        if (dmax[q] > T(0)) rp = T(qmax[q] - q64[q]) / dmax[q];
        if (dmin[q] < T(0)) rm = T(q64[q] - qmin[q]) / (-dmin[q]);
        alpha[q] = fmin(T(1), beta * fmin(rp, rm));
      }
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a.B[k * n + i] = b64[k];
      if (sizeof(T) == sizeof(double)) {
        double *rec = a.rec + i * R_STRIDE;
        rec[R_X] = xi;
        rec[R_Y] = yi;
        rec[R_Z] = zi;
        rec[R_IH] = (double)ih;
        rec[R_V] = gi[GIN_V];
        rec[R_RHO] = q64[0];
        rec[R_IRHO] = 1.0 / q64[0];
        rec[R_VX] = q64[1];
        rec[R_VY] = q64[2];
        rec[R_VZ] = q64[3];
        rec[R_P] = q64[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) rec[R_B + k] = b64[k];
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double v = (double)(alpha[q] * g[q][k]);
            a.grad[(3 * q + k) * n + i] = v;
            rec[R_G + 3 * q + k] = v;
          }
      } else {
        float *rec = reinterpret_cast<float *>(a.rec) + i * F_STRIDE;
        rec[F_IH] = (float)ih;
        rec[F_V] = (float)gi[GIN_V];
        rec[F_RHO] = (float)qi[0];
        rec[F_IRHO] = (float)(1.0 / q64[0]);
        rec[F_VX] = (float)qi[1];
        rec[F_VY] = (float)qi[2];
        rec[F_VZ] = (float)qi[3];
        rec[F_P] = (float)qi[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) rec[F_B + k] = (float)b64[k];
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const float v = (float)(alpha[q] * g[q][k]);
            a.grad[(3 * q + k) * n + i] = (double)v;
            rec[F_G + 3 * q + k] = v;
          }
        rec[F_STRIDE - 3] = rec[F_STRIDE - 2] = rec[F_STRIDE - 1] = 0.0f;
      }
      a.ncond[i] = (double)nc;
      if (a.ekm) a.ekm[i] = 0.5 * a.m[i] * dv2max;
      a.dt_i[i] = vsig > T(0) ? a.c_cfl * hi / (double)vsig : __builtin_huge_val();
      a.fcnt[i] = nf;
    }
  }
  count_add(a.counters + C_GRAD_PAIRS, pairs);
  count_add(a.counters + C_SINGULAR_E, singular);
  count_add(a.counters + C_FP64_INVERSE, inv64);
}

// The mixed path's FP64 redo of the particles gradients_k queued: E, the
// gradient sums, B = E^-1, the limiter and the flux record's B and
// gradients, all in FP64 from the FP64 neighbour records (one wavefront per
// particle, lanes over its gather set).  The face lists, the signal velocity
// and the rest of the record stay as gradients_k wrote them.
__global__ void __launch_bounds__(64) grad_fix_k(GradArgs a) {
  if (a.counters[C_STEP_SKIP]) return;
  const int64_t count = a.counters[C_GRAD_QUEUE];
  const int lane = threadIdx.x;
  const int64_t n = a.n;
  for (int64_t qn = blockIdx.x; qn < count; qn += gridDim.x) {
    const int64_t i = a.grad_q[qn];
    const double *gi = a.gin + i * GIN_STRIDE;
    const double xi = gi[GIN_X], yi = gi[GIN_Y], zi = gi[GIN_Z], hi = gi[GIN_H];
    const double ih = 1.0 / hi, wnorm = 8.0 / (PI * hi * hi * hi);
    const double q64[5] = {gi[GIN_RHO], gi[GIN_VX], gi[GIN_VY], gi[GIN_VZ], gi[GIN_P]};
    const int gc = a.gl_cnt[i];
    const int64_t lb = list_base(a.lseg, i);
    double e[6] = {0, 0, 0, 0, 0, 0}, s[5][3], qmax[5], qmin[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      s[q][0] = s[q][1] = s[q][2] = 0.0;
      qmax[q] = qmin[q] = q64[q];
    }
    // a neighbour's separation: its position from pos on a sub-step of
    // individual steps (see load_nb), else from its record
    auto sep = [&](int64_t j, double d[3]) {
      double p[3];
      if (a.act) {
        const double4 q = a.pos[j];
        p[0] = q.x; p[1] = q.y; p[2] = q.z;
      } else {
        const double *gj = a.gin + j * GIN_STRIDE;
        p[0] = gj[GIN_X]; p[1] = gj[GIN_Y]; p[2] = gj[GIN_Z];
      }
      d[0] = min_image(p[0] - xi, a.box[0], a.half[0]);
      d[1] = min_image(p[1] - yi, a.box[1], a.half[1]);
      d[2] = min_image(p[2] - zi, a.box[2], a.half[2]);
    };
    for (int k = lane; k < gc; k += 64) {
      const int64_t j = a.gl[list_at(lb, k)];
      const double *gj = a.gin + j * GIN_STRIDE;
      double d[3];
      sep(j, d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 == 0.0) continue;
      const double wv = gj[GIN_V] * wnorm * spline_wt<double>(sqrt(r2) * ih);
      e[0] += wv * d[0] * d[0];
      e[1] += wv * d[0] * d[1];
      e[2] += wv * d[0] * d[2];
      e[3] += wv * d[1] * d[1];
      e[4] += wv * d[1] * d[2];
      e[5] += wv * d[2] * d[2];
      const double qj[5] = {gj[GIN_RHO], gj[GIN_VX], gj[GIN_VY], gj[GIN_VZ], gj[GIN_P]};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double df = wv * (qj[q] - q64[q]);
        s[q][0] += df * d[0];
        s[q][1] += df * d[1];
        s[q][2] += df * d[2];
        qmax[q] = fmax(qmax[q], qj[q]);
        qmin[q] = fmin(qmin[q], qj[q]);
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = wave_sum_f64(e[k]);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s[q][k] = wave_sum_f64(s[q][k]);
      qmax[q] = wave_max_f64(qmax[q]);
      qmin[q] = wave_min_f64(qmin[q]);
    }
    double b[6], g[5][3];
    sym_inv<double>(e, b);
    const double nc = sym_frob<double>(b) * sym_frob<double>(e) / 3.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) sym_apply<double>(b, s[q], g[q]);
    double alpha[5] = {1, 1, 1, 1, 1};
    if (a.limiter & MFM_LIMIT_BJ) {
      double dmax[5] = {0, 0, 0, 0, 0}, dmin[5] = {0, 0, 0, 0, 0};
      for (int k = lane; k < gc; k += 64) {
        double d[3];
        sep(a.gl[list_at(lb, k)], d);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const double ex = 0.5 * (g[q][0] * d[0] + g[q][1] * d[1] + g[q][2] * d[2]);
          dmax[q] = fmax(dmax[q], ex);
          dmin[q] = fmin(dmin[q], ex);
        }
      }
      double t = (a.ncond_max - nc) / (a.ncond_max - 1.0);
      t = t > 0.0 ? (t < 1.0 ? t : 1.0) : 0.0;
      const double beta = 1.0 + t;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        dmax[q] = wave_max_f64(dmax[q]);
        dmin[q] = wave_min_f64(dmin[q]);
        double rp = __builtin_huge_val(), rm = __builtin_huge_val();
        if (dmax[q] > 0.0) rp = (qmax[q] - q64[q]) / dmax[q];
        if (dmin[q] < 0.0) rm = (q64[q] - qmin[q]) / (-dmin[q]);
        alpha[q] = fmin(1.0, beta * fmin(rp, rm));
      }
    }
    if (lane == 0) {
      float *rec = reinterpret_cast<float *>(a.rec) + i * F_STRIDE;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        a.B[k * n + i] = b[k];
        rec[F_B + k] = (float)b[k];
      }
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double v = alpha[q] * g[q][k];
          a.grad[(3 * q + k) * n + i] = v;
          rec[F_G + 3 * q + k] = (float)v;
        }
      a.ncond[i] = nc;
    }
  }
}

__global__ void min_partial_k(const double *__restrict__ v, int64_t n, double *partial,
                              const int64_t *counters) {
  if (counters[C_STEP_SKIP]) return;
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
  if (counters[C_STEP_SKIP]) return;
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
  a.rest_r2 = ctx->rest_r2;
  a.gl = ctx->gl;
  a.lseg = ctx->lseg;
  a.gl_cnt = ctx->gl_cnt;
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
  a.m = pp->m;
  a.ekm = ctx->p.entropy_switch ? ctx->ekm : nullptr;
  a.grad_q = ctx->grad_q;
  a.act = ctx->rungs.rung ? ctx->rungs.act : nullptr;
  if (ctx->p.precision == MFM_MIXED) {
    hipError_t e = hipMemsetAsync(ctx->counters + C_GRAD_QUEUE, 0, sizeof(int64_t), ctx->stream);
    if (e != hipSuccess) return e;
    if (a.act)
      gradients_k<float, true><<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
    else
      gradients_k<float, false><<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
    // one wavefront per queued particle, the queue's length read on the device
    grad_fix_k<<<1024, 64, 0, ctx->stream>>>(a);
  } else {
    if (a.act)
      gradients_k<double, true><<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
    else
      gradients_k<double, false><<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
  }
  min_partial_k<<<RED_BLOCKS, BS, 0, ctx->stream>>>(pp->dt_i, pp->n, ctx->red, ctx->counters);
  dt_final_k<<<1, BS, 0, ctx->stream>>>(ctx->red, RED_BLOCKS, dt_max, dt_dev, ctx->counters);
  return hipGetLastError();
}
