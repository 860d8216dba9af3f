// density.hip -- loop (1) of the scheme: smoothing length and number density
// (sec. 2.3.2 and 2.3.5), plus the one neighbour search of the step.
//
// cand_tree_k: for every particle, the candidates with
// r < cell_margin * max(H_i, H_j), both H at the build, found by a walk of the
// bucket tree (cells.hip), as (index, r^2) in the k-major list (list_at).
// The density loop bounds each H by cell_margin times its value at the build
// (else the pass is redone), so every pair closer than max(H_i, H_j) of the
// step is in the list, and the list is a superset of every neighbour set the
// step uses, however unequal the H.
//
// density_k solves, for each particle,
//   g(H) = (32/3) sum_j w(r_ij / H) - N_NGB = 0
// ((4 pi / 3) H^3 omega^-1 = N_NGB with omega^-1 = sum_j W(r_ij, H)) by Newton
// steps kept inside a bisection bracket (0, cell_margin H_build) over its
// candidate r^2.  The solve ends on a small Newton step, so H is the root to
// roundoff.  Reaching the bracket's end is flagged and the pass is redone
// with larger candidate radii.  Then the number density, the unweighted E~ of the condition-number
// check (with N_NGB boosts), the primitives and the packed 128-byte record
// the gradient loop gathers.  It leaves two lists, both in candidate order:
//   gl                the gather set r < H_i (the gradient loop's pairs);
//   cand / rest_r2    the other candidates, r >= H_i, with r^2 in FP32, where
//                     the gradient loop finds the faces with H_i <= r < H_j.
#include "mfm_internal.h"
#include "lanes.h"

namespace {

constexpr int BS = 256;
constexpr double PI = 3.14159265358979323846;

struct CandArgs {
  int64_t n;
  const double4 *pos;
  const int64_t *lseg;  // list blocks of the chunks (list_at)
  int32_t *ncand;       // out: each particle's candidate count (the next plan's input)
  int count_only;       // record ncand only; write no list
  const uint8_t *act;   // individual steps: 1 for the particles whose step begins (null: all)
  int32_t *cand;
  double *cand_r2;
  int32_t *cand_cnt;
  int64_t *counters;
  int csplit;           // workgroups per bucket (1, or BUCKET / TCH: small set, sub-step)
  // a sub-step's list pass: the chunks holding an active particle
  // (C_CHUNK_QUEUE of them; csplit = BUCKET / TCH); null: every chunk
  const int32_t *chunk_q;
};

// The neighbour search: one wavefront per bucket of BUCKET consecutive
// particles, taken in chunks of TCH (on a set of few buckets, one wavefront
// per chunk, so that the chip fills).  For a chunk, the wavefront walks the
// bucket tree breadth first: a node is opened when its box comes closer to
// the chunk's box than the larger of the two candidate radii (each
// cell_margin times the largest H at the build inside), which every pair
// with r < cell_margin max(H_i, H_j) satisfies; 64 children are tested at a
// time and the accepted ones compacted with a ballot, so the accepted
// buckets come out in index order.  Runs of consecutive buckets become
// particle ranges.  The lanes then load those candidates (coalesced ranges,
// SLOTS per lane) and keep them in registers, and take the chunk's particles
// one at a time: each lane tests its candidates against the particle (a
// uniform load), and the matches are compacted with a ballot into that
// particle's list, staged in LDS.  The lists leave as k-major planes: each
// plane of a chunk is a run of consecutive particles.
// Against a uniform grid whose cells must hold the largest H of the set, the
// walk keeps each chunk's candidates to its own radius and its neighbours',
// whatever the spread of H (the paper's bucket search, sec. 2.2.3).
// Shape of the pair loop (measured on the grid search at 128^3, search +
// density ms): SLOTS 6 / LCAP 64, 1.48 + 1.58; SLOTS 6 / LCAP 48, 1.20 +
// 1.61; SLOTS 8 / LCAP 48, 1.17 + 1.62; LCAP 32, 1.39-1.42 + 1.63.  The LDS a
// workgroup holds sets how many wavefronts a CU runs: fewer staged entries
// per particle buy occupancy at the price of more direct stores.
constexpr int SLOTS = 4;   // candidates per lane per round: 256 per wavefront
constexpr int TCH = LCH;   // particles per chunk: one list chunk
static_assert(BUCKET % TCH == 0, "a bucket holds whole chunks");
constexpr int LCAP = 48;   // list entries per particle staged in LDS (more are stored directly)
constexpr int MAXF = 256;  // accepted nodes of one tree level per chunk
constexpr int TSUB = 4;    // particles per sub-chunk of a spread chunk (cells.hip marks them)
constexpr int SEARCH_WG_TARGET = 4096;  // buckets below which each chunk has its own workgroup

// A wave-uniform value moved to scalar registers (lane 0's copy).
__device__ __forceinline__ double uniform_f64(double v) {
  const int2 w = *reinterpret_cast<const int2 *>(&v);
  int2 r;
  r.x = __builtin_amdgcn_readfirstlane(w.x);
  r.y = __builtin_amdgcn_readfirstlane(w.y);
  return *reinterpret_cast<const double *>(&r);
}

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) cand_tree_k(CandArgs a, Tree g) {
  __shared__ int32_t s_idx[TCH][LCAP];
  __shared__ double s_r2[TCH][LCAP];
  __shared__ int s_f[2][MAXF];   // accepted nodes of the current and next level
  __shared__ int s_cand[64 * SLOTS];  // filtered candidates of a round
  __shared__ int s_cnt[TCH];
  const int lane = threadIdx.x;
  const int64_t n = a.n;
  int64_t overflow = 0;
  // a planned pool that does not fit leaves every chunk without room (and
  // the pass fails as a list overflow)
  const bool no_room = a.count_only || a.counters[C_LIST_POOL] != 0;
  const int nbuckets = (int)((n + BUCKET - 1) / BUCKET);
  // one bucket per workgroup on a full pass (one chunk per workgroup on a
  // set of few buckets, csplit > 1); on the sub-steps of individual time
  // steps a capped grid strides over the chunks
  // work item w: chunk w % csplit of bucket w / csplit (with csplit =
  // BUCKET / TCH, w is the chunk's index); a queue lists the items to take
  const int64_t nwork = a.chunk_q ? a.counters[C_CHUNK_QUEUE] : (int64_t)nbuckets * a.csplit;
  for (int64_t q = a.chunk_q ? (int64_t)blockIdx.x : (int64_t)xcd_block(blockIdx.x, gridDim.x);
       q < nwork; q += gridDim.x) {
    const int w = a.chunk_q ? a.chunk_q[q] : (int)q;
    const int bucket = w / a.csplit;
    const int own_x = bucket * BUCKET;
    const int own_y = (int)min((int64_t)BUCKET, n - own_x);
    // the tree build marked the chunks of this bucket that spread over a box
    // much wider than their particles' radii (where the sorted order jumps,
    // in sparse gas): those are searched TSUB particles at a time, since a
    // smaller box accepts far fewer candidates
    const int spread = (int)g.node[((int64_t)g.lev_off[0] + bucket) * TNODE + TNODE_SPREAD];
    for (int c0 = (w % a.csplit) * TCH; c0 < own_y; c0 += a.csplit * TCH) {
      const int T16 = min(TCH, own_y - c0);
      if (a.act && !__ballot(lane < T16 && a.act[own_x + c0 + lane])) continue;
      const int step = (spread >> (c0 / TCH)) & 1 ? TSUB : TCH;
      for (int t0 = c0; t0 < c0 + T16; t0 += step) {
        const int T = min(step, c0 + T16 - t0);
        // on individual steps, only chunks with a particle whose step begins
        // need lists (wave-uniform)
        if (a.act && !__ballot(lane < T && a.act[own_x + t0 + lane])) continue;
        const int64_t chunk = (own_x + t0) / LCH;
        const int64_t cbase = no_room ? 0 : a.lseg[chunk];
        const int cap = no_room ? 0 : (int)((a.lseg[chunk + 1] - cbase) / LCH);
        // the list base of the first particle here (list_at: particle i of a
        // chunk at block offset i mod LCH)
        const int64_t seg0 = cbase + (own_x + t0) % LCH;
        // lane t holds particle t of the chunk and the length of its list; the
        // loop below broadcasts both
        int tcnt = 0;
        double tx = 0.0, ty = 0.0, tz = 0.0, tq = 0.0, th = 0.0;
        const double4 p0 = a.pos[own_x + t0];
        double blo[3] = {p0.x, p0.y, p0.z}, bhi[3] = {p0.x, p0.y, p0.z};
        if (lane < T) {
          const double4 pt = a.pos[own_x + t0 + lane];
          tx = pt.x; ty = pt.y; tz = pt.z;
          th = g.hfac * pt.w;
          tq = th * th;  // squared radius of the particle's own H
          blo[0] = bhi[0] = tx;
          blo[1] = bhi[1] = ty;
          blo[2] = bhi[2] = tz;
        }
        // the chunk's box and radius
        // (wave-uniform: held in scalar registers)
        double bc[3], bh[3];
    #pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double lo = lanes::wave_min_f64(blo[k]), hi = lanes::wave_max_f64(bhi[k]);
          bc[k] = uniform_f64(0.5 * (lo + hi));
          bh[k] = uniform_f64(0.5 * (hi - lo));
        }
        const double Rc = uniform_f64(lanes::wave_max_f64(th));
        // a node is opened when its box and the chunk's are closer than the
        // larger radius (raised by 1e-12 so that rounding in the box distance
        // cannot drop a pair at the edge)
        auto opens = [&](const double *nd) {
          double gap2 = 0.0;
    #pragma unroll
          for (int k = 0; k < 3; ++k) {
            double d = fabs(0.5 * (nd[k] + nd[3 + k]) - bc[k]);
            d = fmin(d, g.box[k] - d);  // periodic images of the centres
            const double gk = fmax(0.0, d - 0.5 * (nd[3 + k] - nd[k]) - bh[k]);
            gap2 += gk * gk;
          }
          const double R = fmax(Rc, nd[6]) * (1.0 + 1e-12);
          return gap2 < R * R;
        };
        // breadth-first walk from the top node.  When a level would accept more
        // nodes than the LDS holds (a chunk of wide particles), the walk stops
        // above it and the buckets under the accepted nodes are tested one by
        // one below.
        int cur = 0, nf = 1, lev_stop = 0;
        if (lane == 0) s_f[0][0] = 0;
        __syncthreads();
        for (int lev = g.nlev - 1; lev > 0; --lev) {
          const int cl = lev - 1, cnt_c = g.lev_cnt[cl];
          const double *nodes = g.node + (int64_t)g.lev_off[cl] * TNODE;
          int nn = 0;
          const int total = nf * TREE_FANOUT;
          for (int u0 = 0; u0 < total; u0 += 64) {
            const int u = u0 + lane;
            bool open = false;
            int child = 0;
            if (u < total) {
              child = s_f[cur][u / TREE_FANOUT] * TREE_FANOUT + u % TREE_FANOUT;
              if (child < cnt_c) open = opens(nodes + (int64_t)child * TNODE);
            }
            const uint64_t m = __ballot(open);
            const int k = nn + lanes_below(m);
            if (open && k < MAXF) s_f[cur ^ 1][k] = child;
            nn += __popcll(m);
          }
          __syncthreads();
          if (nn > MAXF) {  // wave-uniform
            lev_stop = lev;
            break;
          }
          cur ^= 1;
          nf = nn;
        }
        // the accepted buckets in index order: the frontier's nodes, each
        // expanded to the buckets under it when the walk stopped early
        // (64 at a time across the lanes; bmask holds the accepted ones of the
        // last 64, from bbase)
        const int span = 3 * lev_stop;  // TREE_FANOUT = 2^3 nodes per level
        const int64_t nb0 = g.lev_cnt[0];
        int q = 0;
        int64_t bk = 0, bend = 0, bbase = 0;
        uint64_t bmask = 0;
        auto next_bucket = [&]() -> int {
          if (span == 0) return q < nf ? s_f[cur][q++] : -1;  // accepted by the walk
          for (;;) {
            if (bmask) {
              const int t = __ffsll((unsigned long long)bmask) - 1;
              bmask &= bmask - 1;
              return (int)(bbase + t);
            }
            if (bk >= bend) {
              if (q >= nf) return -1;
              const int64_t v = s_f[cur][q++];
              bk = v << span;
              bend = min((v + 1) << span, nb0);
              continue;
            }
            const int64_t b = bk + lane;
            const bool ok = b < bend && opens(g.node + ((int64_t)g.lev_off[0] + b) * TNODE);
            bmask = __ballot(ok);
            bbase = bk;
            bk += 64;
          }
        };
        // the accepted buckets' particles, filtered by their distance from the
        // chunk's box (every pair partner is within the larger radius of that
        // box), compacted into s_cand a round at a time
        for (bool more = true; more;) {
          int nsel = 0;
          bool far = false;
          while (nsel <= 64 * (SLOTS - 1)) {
            const int bkt = next_bucket();
            if (bkt < 0) {
              more = false;
              break;
            }
            const int j = bkt * BUCKET + lane;
            bool keep = false;
            if (j < n) {
              const double4 pj = a.pos[j];
              const double pk[3] = {pj.x, pj.y, pj.z};
              double gap2 = 0.0;
              bool wrap = false;
    #pragma unroll
              for (int k = 0; k < 3; ++k) {
                double d = fabs(pk[k] - bc[k]);
                // a candidate whose separation from some particle of the chunk
                // may need the periodic image
                wrap = wrap || d + bh[k] > g.half[k];
                d = fmin(d, g.box[k] - d);
                const double gk = fmax(0.0, d - bh[k]);
                gap2 += gk * gk;
              }
              const double R = fmax(Rc, g.hfac * pj.w) * (1.0 + 1e-12);
              keep = gap2 < R * R;
              far = far || (keep && wrap);
            }
            const uint64_t m = __ballot(keep);
            if (keep) s_cand[nsel + lanes_below(m)] = j;
            nsel += __popcll(m);
          }
          if (nsel == 0) break;  // wave-uniform: nothing left
          __syncthreads();
          // slots holding at least one candidate (the rest are neither loaded
          // nor tested)
          const int nsl = (nsel + 63) / 64;
          double px[SLOTS], py[SLOTS], pz[SLOTS], pq[SLOTS];
          int jj[SLOTS];
    #pragma unroll
          for (int s = 0; s < SLOTS; ++s) {
            if (s >= nsl) break;
            const int c = s * 64 + lane;
            // an empty lane: never the particle itself, and its distance
            // overflows to +inf, which fails every test
            jj[s] = -1;
            px[s] = py[s] = pz[s] = 1e300;
            pq[s] = 0.0;
            if (c < nsel) {
              const int j = s_cand[c];
              const double4 pj = a.pos[j];
              jj[s] = j;
              px[s] = pj.x;
              py[s] = pj.y;
              pz[s] = pj.z;
              pq[s] = (g.hfac * pj.w) * (g.hfac * pj.w);
            }
          }
          // the particles of the chunk against the candidates in registers; a
          // round with a candidate that may sit across the periodic boundary
          // takes the minimum image, any other the plain difference (the same
          // value there)
          auto test_chunk = [&](auto wrap) {
          constexpr bool WRAP = decltype(wrap)::value;
          for (int t = 0; t < T; ++t) {
            const int ti = own_x + t0 + t;
            const double ptx = lanes::read_f64(tx, t), pty = lanes::read_f64(ty, t),
                         ptz = lanes::read_f64(tz, t), ptq = lanes::read_f64(tq, t);
            int base = __builtin_amdgcn_readlane(tcnt, t);
    #pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
              if (s >= nsl) break;
              double ex = px[s] - ptx, ey = py[s] - pty, ez = pz[s] - ptz;
              if (WRAP) {
                ex = min_image(ex, g.box[0], g.half[0]);
                ey = min_image(ey, g.box[1], g.half[1]);
                ez = min_image(ez, g.box[2], g.half[2]);
              }
              const double r2 = ex * ex + ey * ey + ez * ez;
              // r2 < max(ptq, pq) as two compares, the particle's own radius by
              // the integer order of the bit patterns (the same order for the
              // non-negative values here, +inf included) so that the compiler
              // keeps them apart, and one lane mask per compare: no branch and
              // no per-slot canonicalisation of the operands
              const bool na = r2 < pq[s];
              const bool nt = __double_as_longlong(r2) < __double_as_longlong(ptq);
              const bool other = jj[s] != ti;
              const bool hit = (na | nt) & other;
              const uint64_t m =
                  (__builtin_amdgcn_ballot_w64(na) | __builtin_amdgcn_ballot_w64(nt)) &
                  __builtin_amdgcn_ballot_w64(other);
              const int k = base + lanes_below(m);
              const int nb = base + __popcll(m);
              if (nb <= LCAP) {  // wave-uniform: every hit of the slot is staged
                if (hit) {
                  s_idx[t][k] = jj[s];
                  s_r2[t][k] = r2;
                }
              } else if (hit) {
                if (k < LCAP) {
                  s_idx[t][k] = jj[s];
                  s_r2[t][k] = r2;
                } else if (k < cap) {
                  const int64_t at = list_at(seg0 + t, k);
                  a.cand[at] = jj[s];
                  a.cand_r2[at] = r2;
                }
              }
              base = nb;
            }
            tcnt = lane == t ? base : tcnt;
          }
          };
          if (__ballot(far))
            test_chunk(std::true_type{});
          else
            test_chunk(std::false_type{});
          __syncthreads();
        }
        if (lane < TCH) s_cnt[lane] = tcnt;
        __syncthreads();
        // the chunk's staged lists, plane by plane:
        // lane -> (plane kk + lane / TCH, particle lane % TCH)
        int mine = lane < T ? min(s_cnt[lane], min(LCAP, cap)) : 0;
        const int kmax = lanes::wave_max_i32(mine);
        const int tl = lane % TCH;
        const int lim = tl < T ? min(s_cnt[tl], min(LCAP, cap)) : 0;
        for (int kk = 0; kk < kmax; kk += 64 / TCH) {
          const int k = kk + lane / TCH;
          if (k < lim) {
            const int64_t at = list_at(seg0 + tl, k);
            a.cand[at] = s_idx[tl][k];
            a.cand_r2[at] = s_r2[tl][k];
          }
        }
        if (lane < T) a.ncand[own_x + t0 + lane] = s_cnt[lane];
        if (lane < T && !a.count_only) {
          const int c = s_cnt[lane];
          a.cand_cnt[own_x + t0 + lane] = min(c, cap);
          overflow += c > cap ? 1 : 0;
        }
        __syncthreads();
      }
    }
  }
  count_add(a.counters + C_PASS_LIST, overflow);
}

struct DensityArgs {
  int64_t n;
  const double4 *pos;
  const double *m, *vx, *vy, *vz;
  double *U;
  double *H, *V, *rho, *P, *c, *ncond;
  double *S;              // entropy switch: extensive entropy (null when off)
  const int32_t *emode;   // 1: the pressure comes from S
  double *gin;  // GIN_STRIDE doubles per particle
  int32_t *cand, *cand_cnt;
  const double *cand_r2;
  float *rest_r2;
  int32_t *gl, *gl_cnt;
  const int64_t *lseg;    // list blocks of the chunks (list_at)
  const uint8_t *act;     // individual steps: 1 for the particles whose step begins (null: all)
  int32_t *long_q;        // particles whose list density_k cannot hold (C_LONG_QUEUE of them)
  double gamma, n_ngb, ncond_max, ngb_boost, h_tol;
  int h_maxit, max_boosts;
  int64_t *counters;
};

// The density loop: DT particles per wavefront, DG = 64 / DT lanes per
// particle, each lane holding DM entries of the particle's list (entries
// sub, sub + DG, ...) in registers, so one particle's list of up to
// DCAP = DG * DM entries is read from HBM once for all its Newton passes.
// Measured at 2.1M particles: with about 84 candidates each (an earlier, wider
// candidate radius), DM = 12 (161 VGPRs, 3 waves per SIMD) 1.74 ms, DM = 16
// (194 VGPRs, 2 waves) 2.30 ms, 4 particles per wavefront with 16 lanes
// each 2.5-2.7 ms; with about 40 (the pair radius), DM = 12 1.25 ms, DM = 10
// 1.20, DM = 8 at 3 waves 1.18, DM = 8 held to 128 VGPRs for 4 waves 1.15.
// Longer lists go to density_wave_k.
constexpr int DT = 8;
constexpr int DG = 64 / DT;
constexpr int DM = 8;
constexpr int DCAP = DG * DM;
static_assert(LCH % DT == 0, "a wavefront's particles share one list chunk");

// Sum over the G lanes of an aligned group, as a butterfly: lane pairs
// 1 apart, then 2 apart, then the other quad.  Every lane gets the same bits,
// since each pairwise sum is formed from the same two operands.  For G = 8
// the exchanges are DPP moves (quad permutations, then the half-row mirror,
// whose partner lane already holds the other quad's sum) instead of LDS
// permutes.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(G == 1 || G == 8, "group sums are built for 1 or 8 lanes");
  if constexpr (G == 8) {
    v += lanes::dpp_f64<lanes::QUAD_XOR1>(v);        // partner lane ^ 1
    v += lanes::dpp_f64<lanes::QUAD_XOR2>(v);        // partner lane ^ 2
    v += lanes::dpp_f64<lanes::ROW_HALF_MIRROR>(v);  // lane 7 - l of its 8
  }
  return v;
}

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

struct HSolve {
  double h;        // the root (the list split uses it)
  double h_store;  // what is written as H: the root, or a start value for a coarser grid
  double winv, nc;
  int noconv, boosts, fails, overflow;
};

// The smoothing-length solve of one particle from the start value h, inside
// the bracket (0, hcap): hcap = min(cell side, cell_margin * H at the build).
//   sums(h, ih, s, ds):  s = sum w(q), ds = sum q w'(q) over the list entries
//                        with r < h (q = r / h, ih = 1 / h);
//   esums(h, ih, ws, e): ws = sum w(q) and the unweighted E~ = sum w(q) d d^T.
// The particle itself (w(0) = 1) is added here.  Both must return the same
// value in every lane that calls them together.
template <typename Sums, typename ESums>
__device__ __forceinline__ HSolve newton_h(const DensityArgs &a, double hcap, double h, Sums sums,
                                           ESums esums) {
  HSolve r{};
  const double cover = hcap;
  const double qtol = fmax(a.h_tol, 1e-2 * sqrt(a.h_tol));
  double target = a.n_ngb;
  double s_last = 1.0;
  for (int b = 0;; ++b) {
    double lo = 0.0, hi = cover;
    if (!(h > lo && h < hi)) h = 0.5 * hi;
    bool conv = false;
    for (int it = 0; it < a.h_maxit; ++it) {
      const double ih = 1.0 / h;
      double s, ds;
      sums(h, ih, s, ds);
      s += 1.0;
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
      // stop on a small Newton step only (never on a bisection step).  In the
      // quadratic regime the error after a step of relative size d is of
      // order d^2, so a step below qtol = 1e-2 sqrt(h_tol) already leaves H
      // at the root to far below h_tol: the pass that would only confirm it
      // is skipped
      if (fabs(hn - h) <= qtol * hn) {
        h = hn;
        conv = true;
        break;
      }
      if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
      h = hn;
    }
    if (!conv) ++r.noconv;
    // number density at the solution and the unweighted E~ of the check
    const double h2 = h * h;
    double ws, e[6];
    esums(h, 1.0 / h, ws, e);
    ws += 1.0;
    r.winv = 8.0 / (PI * h * h2) * ws;
    r.nc = cond3(e);  // the kernel's normalisation drops out of the condition number
    if (!(r.nc > a.ncond_max)) break;
    if (b == a.max_boosts) {
      ++r.fails;
      break;
    }
    target *= a.ngb_boost;
    ++r.boosts;
  }
  r.h = h;
  r.h_store = h;
  if (h >= cover * (1.0 - 1e-12)) {
    // the root lies beyond half the box or grew by more than cell_margin
    // since the build: this pass is redone with candidate radii from an
    // estimate of the root (at fixed number density the neighbour number
    // grows as H^3; 15% more for a density that falls outwards), written as
    // the start value
    r.overflow = 1;
    r.h_store = cover * cbrt(target / fmax((32.0 / 3.0) * s_last, 1.0)) * 1.15;
  }
  return r;
}

// r: the pair's distance, sqrt(r^2)
__device__ __forceinline__ void add_pair(double &s, double &ds, double r, double ih) {
  const double q = r * ih;
  s += spline_w(q);
  ds += spline_qdw(q);
}

__device__ __forceinline__ void add_e(double &ws, double e[6], double r, double ih,
                                      double4 pj, double4 pi, const Tree &g) {
  const double w = spline_w(r * ih);
  ws += w;
  if (r > 0.0) {
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

// Upper end of a particle's bracket (pi.w: its H at the build).
__device__ __forceinline__ double hcap_of(const Tree &g, double4 pi) {
  return pi.w > 0.0 ? fmin(g.side_min, g.hfac * pi.w) : g.side_min;
}

// H, the number density, the primitives and the gradient loop's record of particle i.
__device__ __forceinline__ void finish_particle(const DensityArgs &a, int64_t i, const HSolve &r) {
  const double h = r.h_store;
  const double V = 1.0 / r.winv;
  const double rho = a.m[i] / V;
  double P = (a.gamma - 1.0) * a.U[i] / V;
  if (a.S) {
    // the entropy switch (sec. 2.3.7): a particle the last close of the step
    // put in the entropy branch takes P = (S / m) rho^gamma and the U that
    // gives it; every other particle resets S from its U
    if (a.emode[i]) {
      P = a.S[i] / a.m[i] * pow(rho, a.gamma);
      a.U[i] = P * V / (a.gamma - 1.0);
    } else {
      a.S[i] = a.m[i] * P / pow(rho, a.gamma);
    }
  }
  const double cs = sqrt(a.gamma * P / rho);
  a.H[i] = h;
  a.V[i] = V;
  a.rho[i] = rho;
  a.P[i] = P;
  a.c[i] = cs;
  a.ncond[i] = r.nc;
  const double4 pi = a.pos[i];
  const double vx = a.vx[i], vy = a.vy[i], vz = a.vz[i];
  double4 *gr = reinterpret_cast<double4 *>(a.gin + i * GIN_STRIDE);
  gr[0] = make_double4(pi.x, pi.y, pi.z, h);
  gr[1] = make_double4(V, rho, vx, vy);
  gr[2] = make_double4(vz, P, cs, 0.0);
  float4 *gf = reinterpret_cast<float4 *>(a.gin + i * GIN_STRIDE + GIN_F32);
  gf[0] = make_float4((float)V, (float)rho, (float)P, (float)cs);
  // the record's last 16 bytes are unused: written too, so that no 32-byte
  // sector of it is left partly written
  static_assert(GIN_F32 + 4 == GIN_STRIDE, "the FP32 copies end 16 bytes before the record");
  gf[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// One wavefront per DT consecutive particles.  A particle's candidate list is
// loaded once into the registers of its DG lanes; every Newton pass and the
// final pass run from there (group sums by lane exchange).  The list is then
// split at r = H_i, in candidate order: the gather set goes to gl, the rest
// (index and FP32 r^2) back into cand / rest_r2.  Both are staged in LDS and
// leave as k-major planes of DT consecutive particles.  A list longer than
// DCAP is left whole, marked gl_cnt = -1 and queued for density_wave_k.
struct DensityStage {
  int32_t (*s_i)[DT];  // gather set from the front, rest indices from the back
  float (*s_f)[DT];    // rest r^2
  int *s_gn, *s_rn;
};
struct PassCounts {
  int64_t noconv = 0, boosts = 0, fails = 0, overflow = 0;
};

__device__ __forceinline__ void density_group(const DensityArgs &a, const Tree &g, int64_t grp,
                                              const DensityStage &st, PassCounts &pc) {
  const int lane = threadIdx.x;
  const int gt = lane / DG, sub = lane % DG;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t gmask = ((1ull << DG) - 1ull) << (gt * DG);
  const int64_t n = a.n;
  auto s_i = st.s_i;
  auto s_f = st.s_f;
  int *s_gn = st.s_gn, *s_rn = st.s_rn;
  const int64_t i0 = grp * DT;
  const int64_t i = i0 + gt;
  // a particle in mid-step (individual steps) keeps its H and lists
  const bool valid = i < n && (!a.act || a.act[i]);
  if (a.act && !__ballot(valid)) return;  // wave-uniform: nothing to do
  const int cnt = valid ? a.cand_cnt[i] : 0;
  const int64_t lb = valid ? list_base(a.lseg, i) : 0;
  if (valid && cnt <= DCAP) {
    // the distances r (not r^2): the square root is taken once here, not at
    // every Newton pass, and membership is r < h as in the kernel's support
    double rs[DM];
    int jr[DM];
#pragma unroll
    for (int m = 0; m < DM; ++m) {
      const int k = sub + DG * m;
      rs[m] = __builtin_huge_val();  // beyond the list: never inside any H
      jr[m] = 0;
      if (k < cnt) {
        rs[m] = sqrt(a.cand_r2[list_at(lb, k)]);
        jr[m] = a.cand[list_at(lb, k)];
      }
    }
    const double4 pi = a.pos[i];
    auto sums = [&](double h, double ih, double &s, double &ds) {
      s = 0.0;
      ds = 0.0;
#pragma unroll
      for (int m = 0; m < DM; ++m)
        if (rs[m] < h) add_pair(s, ds, rs[m], ih);
      s = group_sum<DG>(s);
      ds = group_sum<DG>(ds);
    };
    auto esums = [&](double h, double ih, double &ws, double e[6]) {
      ws = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) e[q] = 0.0;
#pragma unroll
      for (int m = 0; m < DM; ++m)
        if (rs[m] < h) add_e(ws, e, rs[m], ih, a.pos[jr[m]], pi, g);
      ws = group_sum<DG>(ws);
#pragma unroll
      for (int q = 0; q < 6; ++q) e[q] = group_sum<DG>(e[q]);
    };
    const HSolve r = newton_h(a, hcap_of(g, pi), a.H[i], sums, esums);
    int gn = 0, rn = 0;
#pragma unroll
    for (int m = 0; m < DM; ++m) {
      const bool in = sub + DG * m < cnt;
      const bool near = in && rs[m] < r.h;
      const bool far = in && !near;
      const uint64_t mn = __ballot(near) & gmask, mf = __ballot(far) & gmask;
      if (near) s_i[gn + __popcll(mn & below)][gt] = jr[m];
      if (far) {
        const int p = rn + __popcll(mf & below);
        s_i[DCAP - 1 - p][gt] = jr[m];
        s_f[p][gt] = (float)(rs[m] * rs[m]);  // within an FP32 rounding of r^2
      }
      gn += __popcll(mn);
      rn += __popcll(mf);
    }
    if (sub == 0) {
      s_gn[gt] = gn;
      s_rn[gt] = rn;
      finish_particle(a, i, r);
      pc.noconv += r.noconv;
      pc.boosts += r.boosts;
      pc.fails += r.fails;
      pc.overflow += r.overflow;
    }
  } else if (valid && sub == 0) {
    s_gn[gt] = -1;  // left whole in cand for density_wave_k
    s_rn[gt] = -1;
    const unsigned long long slot =
        atomicAdd(reinterpret_cast<unsigned long long *>(a.counters + C_LONG_QUEUE), 1ull);
    a.long_q[slot] = (int32_t)i;
  }
  __syncthreads();
  // the staged lists, plane by plane: lane -> (plane kk + lane / DT, particle lane % DT)
  const int tl = lane % DT;
  const int64_t pl = i0 + tl;
  const bool own = pl < n && (!a.act || a.act[pl]) && s_gn[tl] >= 0;
  const int glim = own ? s_gn[tl] : 0;
  const int rlim = own ? s_rn[tl] : 0;
  const int kmax = lanes::wave_max_i32(max(glim, rlim));
  const int64_t pb = pl < n ? list_base(a.lseg, pl) : 0;
  for (int kk = 0; kk < kmax; kk += 64 / DT) {
    const int k = kk + lane / DT;
    if (k < glim) a.gl[list_at(pb, k)] = s_i[k][tl];
    if (k < rlim) {
      a.cand[list_at(pb, k)] = s_i[DCAP - 1 - k][tl];
      a.rest_r2[list_at(pb, k)] = s_f[k][tl];
    }
  }
  if (lane < DT && pl < n && (!a.act || a.act[pl])) {
    a.gl_cnt[pl] = own ? glim : -1;
    if (own) a.cand_cnt[pl] = rlim;
  }
  __syncthreads();  // the staging arrays may be reused by another group
}

// One group of DT particles per workgroup (a full pass).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) density_k(DensityArgs a, Tree g) {
  __shared__ int32_t s_i[DCAP][DT];
  __shared__ float s_f[DCAP][DT];
  __shared__ int s_gn[DT], s_rn[DT];
  // a search whose lists overflowed leaves the pass to be redone: nothing
  // here may change the state
  if (a.counters[C_PASS_LIST] != 0) return;
  PassCounts pc;
  density_group(a, g, xcd_block(blockIdx.x, gridDim.x), DensityStage{s_i, s_f, s_gn, s_rn}, pc);
  count_add(a.counters + C_PASS_NOCONV, pc.noconv);
  count_add(a.counters + C_PASS_BOOSTS, pc.boosts);
  count_add(a.counters + C_PASS_FAIL, pc.fails);
  count_add(a.counters + C_CELL_OVERFLOW, pc.overflow);
}

// The sub-steps of individual time steps, where few particles are active:
// every particle whose step begins is queued for density_wave_k, whose 64
// lanes per particle shorten the serial chain of loads and Newton passes
// that the few busy wavefronts of an 8-lane group would run.
__global__ void __launch_bounds__(BS) queue_active_k(DensityArgs a) {
  if (a.counters[C_PASS_LIST] != 0) return;  // as in density_k
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool on = i < a.n && a.act[i];
  const uint64_t m = __ballot(on);
  if (!m) return;  // wave-uniform
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if ((int)(threadIdx.x & 63) == leader)
    base = atomicAdd(reinterpret_cast<unsigned long long *>(a.counters + C_LONG_QUEUE),
                     (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  if (on) a.long_q[base + lanes_below(m)] = (int32_t)i;
}

// The lists density_k could not hold (queued, gl_cnt = -1): one wavefront
// per particle, its lanes taking the list entries k = lane, lane + 64, ...
// from HBM on every pass (sums by wavefront butterflies, wave_sum_f64: every
// lane gets the same bits, so all take the same branches), then the split in
// candidate order, 64 entries at a time (an entry moves only to a slot at or
// before its own, after the whole chunk has been read).  The grid strides
// over the queue, whose length is read on the device.
__global__ void __launch_bounds__(BS) density_wave_k(DensityArgs a, Tree g) {
  if (a.counters[C_PASS_LIST] != 0) return;  // as in density_k
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (BS / 64);
  const int64_t nq = a.counters[C_LONG_QUEUE];
  const uint64_t below = (1ull << lane) - 1ull;
  int64_t noconv = 0, boosts = 0, fails = 0, overflow = 0;
  for (int64_t q = wave; q < nq; q += nwaves) {
    const int64_t i = a.long_q[q];
    const int cnt = a.cand_cnt[i];
    const int64_t lb = list_base(a.lseg, i);
    const double4 pi = a.pos[i];
    auto sums = [&](double h, double ih, double &s, double &ds) {
      s = 0.0;
      ds = 0.0;
      for (int k = lane; k < cnt; k += 64) {
        const double r = sqrt(a.cand_r2[list_at(lb, k)]);
        if (r < h) add_pair(s, ds, r, ih);
      }
      s = wave_sum_f64(s);
      ds = wave_sum_f64(ds);
    };
    auto esums = [&](double h, double ih, double &ws, double e[6]) {
      ws = 0.0;
      for (int m = 0; m < 6; ++m) e[m] = 0.0;
      for (int k = lane; k < cnt; k += 64) {
        const double r = sqrt(a.cand_r2[list_at(lb, k)]);
        if (r < h) add_e(ws, e, r, ih, a.pos[a.cand[list_at(lb, k)]], pi, g);
      }
      ws = wave_sum_f64(ws);
      for (int m = 0; m < 6; ++m) e[m] = wave_sum_f64(e[m]);
    };
    const HSolve r = newton_h(a, hcap_of(g, pi), a.H[i], sums, esums);
    int gn = 0, rn = 0;
    for (int base = 0; base < cnt; base += 64) {
      const int k = base + lane;
      const bool in = k < cnt;
      const double r2 = in ? a.cand_r2[list_at(lb, k)] : 0.0;
      const int j = in ? a.cand[list_at(lb, k)] : 0;
      const bool near = in && sqrt(r2) < r.h;
      const bool far = in && !near;
      const uint64_t mn = __ballot(near), mf = __ballot(far);
      if (near) a.gl[list_at(lb, gn + __popcll(mn & below))] = j;
      if (far) {
        const int p = rn + __popcll(mf & below);
        a.cand[list_at(lb, p)] = j;
        a.rest_r2[list_at(lb, p)] = (float)r2;
      }
      gn += __popcll(mn);
      rn += __popcll(mf);
    }
    if (lane == 0) {
      a.gl_cnt[i] = gn;
      a.cand_cnt[i] = rn;
      finish_particle(a, i, r);
      noconv += r.noconv;
      boosts += r.boosts;
      fails += r.fails;
      overflow += r.overflow;
    }
  }
  count_add(a.counters + C_PASS_NOCONV, noconv);
  count_add(a.counters + C_PASS_BOOSTS, boosts);
  count_add(a.counters + C_PASS_FAIL, fails);
  count_add(a.counters + C_CELL_OVERFLOW, overflow);
}

__global__ void validate_k(int64_t *c) {
  if (threadIdx.x != 0) return;
  if (c[C_PASS_LIST] > 0 || c[C_CELL_OVERFLOW] > 0) {
    c[C_STEP_SKIP] = 1;
    if (c[C_CELL_OVERFLOW] > 0) c[C_CELL_REBUILDS] += 1;
    c[C_LIST_OVERFLOW] += c[C_PASS_LIST];
    return;
  }
  c[C_STEP_SKIP] = 0;
  c[C_H_NOCONV] += c[C_PASS_NOCONV];
  c[C_NCOND_BOOSTS] += c[C_PASS_BOOSTS];
  c[C_NCOND_FAIL] += c[C_PASS_FAIL];
}

// The planned capacity of each chunk: the longest candidate list its
// particles had in the last search (the counts move with the particles
// through the sort), an eighth more and 4 (positions and H drift between
// searches), times LCH.  The entry past the last chunk is 0, so that the
// scan ends with the total.
// A sub-step's list pass: the chunks (LCH consecutive particles, one
// 16-lane row of a wavefront) holding a particle whose step begins are
// queued, one atomic per wavefront.
__global__ void __launch_bounds__(BS) queue_chunks_k(int64_t n, const uint8_t *__restrict__ act,
                                                     int32_t *chunk_q, int64_t *counters) {
  static_assert(LCH == 16 && BUCKET % 64 == 0, "four chunks to a wavefront");
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const uint64_t m = __ballot(i < n && act[i]);
  // lane 16 r stands for row r: is any of its 16 particles active
  const bool head = lane % LCH == 0 && ((m >> lane) & 0xFFFFull) != 0;
  const uint64_t hm = __ballot(head);
  if (!hm) return;  // wave-uniform
  const int leader = __ffsll((unsigned long long)hm) - 1;
  unsigned long long base = 0;
  if (lane == leader)
    base = atomicAdd(reinterpret_cast<unsigned long long *>(counters + C_CHUNK_QUEUE),
                     (unsigned long long)__popcll(hm));
  base = __shfl(base, leader, 64);
  if (head) chunk_q[base + lanes_below(hm)] = (int32_t)(i / LCH);
}

__global__ void plan_k(int64_t n, int64_t nch, const int32_t *__restrict__ ncand, int64_t *cap) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > nch) return;
  int64_t k = 0;
  if (c < nch) {
    int l = 0;
    for (int64_t i = c * LCH; i < min(n, (c + 1) * LCH); ++i) l = max(l, ncand[i]);
    k = (int64_t)l + l / 8 + 4;
  }
  cap[c] = k * LCH;
}

__global__ void pool_check_k(const int64_t *__restrict__ lseg, int64_t nch, int64_t pool,
                             int64_t *counters) {
  if (threadIdx.x == 0) {
    counters[C_LIST_POOL] = lseg[nch] > pool ? 1 : 0;
    counters[C_LONG_QUEUE] = 0;  // the density loop that follows fills the queue
    counters[C_CHUNK_QUEUE] = 0;  // and a sub-step's list pass its chunk queue
  }
}

}  // namespace

hipError_t launch_plan_lists(mfm_ctx *ctx, int64_t n) {
  const int64_t nch = list_chunks(n);
  plan_k<<<blocks_for(nch + 1, BS), BS, 0, ctx->stream>>>(n, nch, ctx->ncand, ctx->lcap);
  hipError_t e = scan_exclusive_i64(ctx->stream, ctx->lcap, ctx->lseg, nch + 1, ctx->scan64);
  if (e != hipSuccess) return e;
  pool_check_k<<<1, 64, 0, ctx->stream>>>(ctx->lseg, nch, (int64_t)ctx->pool, ctx->counters);
  return hipGetLastError();
}

hipError_t launch_validate(mfm_ctx *ctx) {
  validate_k<<<1, 64, 0, ctx->stream>>>(ctx->counters);
  return hipGetLastError();
}

hipError_t launch_candidates(mfm_ctx *ctx, const mfm_particles *pp, bool count_only) {
  CandArgs a;
  a.n = pp->n;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.lseg = ctx->lseg;
  a.ncand = ctx->ncand;
  a.count_only = count_only ? 1 : 0;
  a.act = ctx->rungs.rung ? ctx->rungs.act : nullptr;
  a.cand = ctx->cand;
  a.cand_r2 = ctx->cand_r2;
  a.cand_cnt = ctx->cand_cnt;
  a.counters = ctx->counters;
  const int64_t buckets = ctx->tree.lev_cnt[0];
  // under SEARCH_WG_TARGET buckets, and on the sub-steps of individual
  // steps (few chunks, scattered, need lists), each chunk gets a workgroup
  // of its own; on a sub-step a capped grid strides over the chunks
  a.csplit = (a.act || buckets < SEARCH_WG_TARGET) ? BUCKET / TCH : 1;
  // a sub-step's list pass takes the chunks with an active particle from a
  // queue (in the gradient loop's queue buffer, unused until that loop; the
  // counting pass, rare on a sub-step, strides over every chunk)
  a.chunk_q = nullptr;
  if (a.act && !count_only) {
    queue_chunks_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(pp->n, a.act, ctx->grad_q,
                                                                   ctx->counters);
    a.chunk_q = ctx->grad_q;
  }
  const int64_t grid = a.act ? std::min<int64_t>(buckets * a.csplit, 8192) : buckets * a.csplit;
  cand_tree_k<<<(unsigned)grid, 64, 0, ctx->stream>>>(a, ctx->tree);
  return hipGetLastError();
}

hipError_t launch_density(mfm_ctx *ctx, const mfm_particles *pp) {
  DensityArgs a;
  a.n = pp->n;
  a.pos = reinterpret_cast<const double4 *>(ctx->pos4);
  a.m = pp->m; a.U = pp->U; a.vx = pp->vx; a.vy = pp->vy; a.vz = pp->vz;
  a.H = pp->H; a.V = pp->V; a.rho = pp->rho; a.P = pp->P; a.c = pp->c; a.ncond = pp->ncond;
  a.S = ctx->p.entropy_switch ? pp->S : nullptr;
  a.emode = pp->emode;
  a.gin = ctx->gin;
  a.cand = ctx->cand;
  a.cand_cnt = ctx->cand_cnt;
  a.cand_r2 = ctx->cand_r2;
  a.rest_r2 = ctx->rest_r2;
  a.gl = ctx->gl;
  a.gl_cnt = ctx->gl_cnt;
  a.lseg = ctx->lseg;
  a.act = ctx->rungs.rung ? ctx->rungs.act : nullptr;
  a.gamma = ctx->p.gamma;
  a.n_ngb = ctx->p.n_ngb;
  a.ncond_max = ctx->p.ncond_max;
  a.ngb_boost = ctx->p.ngb_boost;
  a.h_tol = ctx->p.h_tol;
  a.h_maxit = ctx->p.h_maxit;
  a.max_boosts = ctx->p.max_boosts;
  a.counters = ctx->counters;
  a.long_q = ctx->grad_q;  // the gradient loop's queue, unused until that loop
  const int64_t groups = (pp->n + DT - 1) / DT;
  if (a.act)
    queue_active_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(a);
  else
    density_k<<<(unsigned)groups, 64, 0, ctx->stream>>>(a, ctx->tree);
  density_wave_k<<<2048, BS, 0, ctx->stream>>>(a, ctx->tree);
  return hipGetLastError();
}
