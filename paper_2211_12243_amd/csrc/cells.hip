// cells.hip -- the particle order and the neighbour-search tree: Morton
// (Z-order) keys of the particles' positions, a stable radix sort by them,
// the in-place permutation of the state arrays, and the bucket tree.
//
// The paper reorders its particle array so that the particles of a tree node
// are contiguous (sec. 2.2.1) and searches neighbours per bucket of particles
// (sec. 2.2.3).  Here the keys carry KEY_BITS bits per axis, fine enough that
// the sorted array follows a Z-order curve through the particles even where
// they cluster; buckets are runs of BUCKET consecutive particles, and a tree
// over them (TREE_FANOUT consecutive nodes per parent) carries each node's
// bounding box and largest candidate radius.  The search (density.hip) walks
// that tree per chunk of a bucket, so a particle's candidates follow its own
// H and its neighbours', not the largest H of the set.
#include "mfm_internal.h"
#include "lanes.h"

namespace {

constexpr int BS = 256;

// Exclusive scan, 1024 elements per block (4 per thread), block totals out.
template <typename T>
__global__ void scan_block_k(const T *in, T *out, int64_t n, T *block_sums) {
  __shared__ T s[BS];
  int64_t base = blockIdx.x * (int64_t)(4 * BS) + 4 * threadIdx.x;
  T v[4];
  T t = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    t += v[k];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    T add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  T run = s[threadIdx.x] - t;  // exclusive prefix of this thread
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == BS - 1) block_sums[blockIdx.x] = s[BS - 1];
}

template <typename T>
__global__ void scan_add_k(T *out, int64_t n, const T *block_offsets) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_offsets[i / (4 * BS)];
}

// In place is allowed (in == out); tmp holds the block sums of every level.
template <typename T>
hipError_t scan_exclusive_t(hipStream_t st, const T *in, T *out, int64_t n, T *tmp) {
  int64_t nb = (n + 4 * BS - 1) / (4 * BS);
  scan_block_k<T><<<(int)nb, BS, 0, st>>>(in, out, n, tmp);
  if (nb > 1) {
    hipError_t e = scan_exclusive_t<T>(st, tmp, tmp, nb, tmp + nb);
    if (e != hipSuccess) return e;
    scan_add_k<T><<<blocks_for(n, BS), BS, 0, st>>>(out, n, tmp);
  }
  return hipGetLastError();
}

hipError_t scan_exclusive(hipStream_t st, const int32_t *in, int32_t *out, int64_t n,
                          int32_t *tmp) {
  return scan_exclusive_t<int32_t>(st, in, out, n, tmp);
}

// Lanes of the wavefront whose 8-bit digit equals this lane's, among the
// live ones (every lane must take part).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool live) {
  uint64_t m = __ballot(live);
#pragma unroll
  for (int b = 0; b < RADIX_BITS; ++b) {
    const uint64_t t = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? t : ~t;
  }
  return m;
}

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Morton key of each particle (bits per axis of its place in the box) and
// its slot, the value the sort carries.
__global__ void key_k(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                      const double *__restrict__ z, double sx, double sy, double sz, int bits,
                      uint32_t *key, int32_t *val) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int top = (1 << bits) - 1;
  auto q = [top](double v, double s) {
    const int c = (int)(v * s);
    return c < 0 ? 0 : (c > top ? top : c);
  };
  key[i] = morton3(q(x[i], sx), q(y[i], sy), q(z[i], sz));
  val[i] = (int32_t)i;
}

// One pass of the least-significant-digit radix sort: each workgroup counts
// the digits of its tile (SORT_TILE consecutive items) into hist, digit-major
// (hist[d * nb + b]), so that an exclusive scan of hist gives every
// workgroup's first output slot for every digit.
__global__ void __launch_bounds__(SORT_BS) radix_hist_k(int64_t n, const uint32_t *__restrict__ key,
                                                        int shift, int nb, int32_t *hist) {
  __shared__ int32_t s[RADIX];
  const int t = threadIdx.x;
  s[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const int64_t i = base + r * SORT_BS + t;
    if (base + r * SORT_BS >= n) break;  // uniform
    const bool live = i < n;
    const uint32_t d = live ? (key[i] >> shift) & (RADIX - 1) : 0u;
    const uint64_t m = match_digit(d, live);
    if (live && lanes_below(m) == 0) atomicAdd(&s[d], __popcll(m));
  }
  __syncthreads();
  hist[(int64_t)t * nb + blockIdx.x] = s[t];
}

// The scatter of the same pass.  The tile goes round by round (SORT_BS
// items), wavefront by wavefront, lane by lane: an item's slot is its
// workgroup's first slot for the digit, plus the items of that digit in the
// earlier rounds, the earlier wavefronts of the round and the lower lanes.
// Equal digits keep their order, so the sort is stable and the result does
// not depend on scheduling.
__global__ void __launch_bounds__(SORT_BS) radix_scatter_k(
    int64_t n, const uint32_t *__restrict__ key, const int32_t *__restrict__ val, int shift, int nb,
    const int32_t *__restrict__ first, uint32_t *key_out, int32_t *val_out) {
  constexpr int NW = SORT_BS / 64;
  __shared__ int32_t s_base[RADIX];
  __shared__ int32_t s_w[NW][RADIX];
  const int t = threadIdx.x, w = t >> 6;
  s_base[t] = first[(int64_t)t * nb + blockIdx.x];
#pragma unroll
  for (int q = 0; q < NW; ++q) s_w[q][t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
  for (int r = 0; r < SORT_ITEMS; ++r) {
    if (base + r * SORT_BS >= n) break;  // uniform
    const int64_t i = base + r * SORT_BS + t;
    const bool live = i < n;
    uint32_t k = 0u, d = 0u;
    int32_t v = 0;
    if (live) {
      k = key[i];
      v = val[i];
      d = (k >> shift) & (RADIX - 1);
    }
    const uint64_t m = match_digit(d, live);
    const int below = lanes_below(m);
    if (live && below == 0) s_w[w][d] = __popcll(m);
    __syncthreads();
    if (live) {
      int at = s_base[d] + below;
      for (int q = 0; q < w; ++q) at += s_w[q][d];
      key_out[at] = k;
      val_out[at] = v;
    }
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      tot += s_w[q][t];
      s_w[q][t] = 0;
    }
    s_base[t] += tot;
    __syncthreads();
  }
}

// Level 0 of the tree: one wavefront per bucket reduces the bounding box and
// the largest H (at the build) of its particles.
__global__ void __launch_bounds__(64) leaf_box_k(int64_t n, const double4 *__restrict__ pos4,
                                                 double hfac, double *node) {
  const int64_t b = blockIdx.x;
  const int64_t i = b * BUCKET + threadIdx.x;
  const bool live = i < n;
  const double4 p = pos4[live ? i : b * BUCKET];  // a bucket has at least one particle
  double lo[3] = {p.x, p.y, p.z}, hi[3] = {p.x, p.y, p.z}, h = live ? p.w : 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = lanes::wave_min_f64(lo[k]);
    hi[k] = lanes::wave_max_f64(hi[k]);
  }
  h = lanes::wave_max_f64(h);
  // each chunk of LCH lanes: its box's half-diagonal against its particles'
  // mean search radius (the spread flag the search reads); a lane past the
  // end takes the last particle, which lies in the same chunk
  const double4 pl = pos4[live ? i : n - 1];
  double clo[3] = {pl.x, pl.y, pl.z}, chi[3] = {pl.x, pl.y, pl.z}, r = live ? hfac * pl.w : 0.0;
  double cnt = live ? 1.0 : 0.0;
  static_assert(LCH == 16, "a chunk is one 16-lane DPP row");
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    clo[k] = lanes::row_min_f64(clo[k]);
    chi[k] = lanes::row_max_f64(chi[k]);
  }
  r = lanes::row_sum_f64(r);
  cnt = lanes::row_sum_f64(cnt);
  double diag2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) diag2 += (chi[k] - clo[k]) * (chi[k] - clo[k]);
  const double rmean = cnt > 0.0 ? r / cnt : 0.0;
  const bool spread = live && diag2 > 4.0 * SPREAD_RATIO * SPREAD_RATIO * rmean * rmean;
  const uint64_t sm = __ballot(spread && (threadIdx.x % LCH) == 0);
  int mask = 0;
  for (int c = 0; c < BUCKET / LCH; ++c) mask |= ((sm >> (c * LCH)) & 1ull) ? 1 << c : 0;
  if (threadIdx.x < TNODE) {
    const double v[TNODE] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], hfac * h, (double)mask};
    node[b * TNODE + threadIdx.x] = v[threadIdx.x];
  }
}

// Level l + 1 from level l: each node the union of its children's boxes and
// the largest of their radii.
__global__ void inner_box_k(const double *__restrict__ child, int nchild, double *parent,
                            int nparent) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nparent) return;
  double v[TNODE];
  const int c0 = k * TREE_FANOUT, c1 = min(c0 + TREE_FANOUT, nchild);
#pragma unroll
  for (int q = 0; q < TNODE; ++q) v[q] = child[(int64_t)c0 * TNODE + q];
  for (int c = c0 + 1; c < c1; ++c) {
    const double *w = child + (int64_t)c * TNODE;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      v[q] = fmin(v[q], w[q]);
      v[3 + q] = fmax(v[3 + q], w[3 + q]);
    }
    v[6] = fmax(v[6], w[6]);
  }
#pragma unroll
  for (int q = 0; q < TNODE; ++q) parent[(int64_t)k * TNODE + q] = v[q];
}

// The state arrays the permutation moves: the ten FP64 fields, the labels,
// the optional source-term arrays (entropy, the three acceleration
// components, the entropy-mode flags; absent ones are null) and the
// candidate counts of the last search (the next list plan's input).
struct Fields {
  double *f[10];
  int64_t *id;
  double *x[4];
  int32_t *emode;
  int32_t *ncand;
  int32_t *rung;  // rungs given by the caller of mfm_step_rungs (null: none)
};

__global__ void gather_k(int64_t n, Fields fs, const int32_t *__restrict__ order, double *tmp,
                         int64_t *perm) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  int32_t o = order[k];
#pragma unroll
  for (int f = 0; f < 10; ++f) tmp[f * n + k] = fs.f[f][o];
  if (fs.id) ((int64_t *)(tmp + 10 * n))[k] = fs.id[o];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (fs.x[e]) tmp[(11 + e) * n + k] = fs.x[e][o];
  if (fs.emode) ((int32_t *)(tmp + 15 * n))[k] = fs.emode[o];
  ((int32_t *)(tmp + 15 * n))[n + k] = fs.ncand[o];
  if (fs.rung) ((int32_t *)(tmp + 16 * n))[k] = fs.rung[o];
  if (perm) perm[k] = o;
}

__global__ void writeback_k(int64_t n, Fields fs, const double *__restrict__ tmp,
                            double4 *pos4) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int f = 0; f < 10; ++f) fs.f[f][k] = tmp[f * n + k];
  if (fs.id) fs.id[k] = ((const int64_t *)(tmp + 10 * n))[k];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (fs.x[e]) fs.x[e][k] = tmp[(11 + e) * n + k];
  if (fs.emode) fs.emode[k] = ((const int32_t *)(tmp + 15 * n))[k];
  fs.ncand[k] = ((const int32_t *)(tmp + 15 * n))[n + k];
  if (fs.rung) fs.rung[k] = ((const int32_t *)(tmp + 16 * n))[k];
  pos4[k] = make_double4(tmp[k], tmp[n + k], tmp[2 * n + k], tmp[9 * n + k]);
}

}  // namespace

hipError_t scan_exclusive_i64(hipStream_t st, const int64_t *in, int64_t *out, int64_t n,
                              int64_t *tmp) {
  return scan_exclusive_t<int64_t>(st, in, out, n, tmp);
}

hipError_t launch_build_cells(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm) {
  hipStream_t st = ctx->stream;
  const int64_t n = pp->n;
  const Tree &g = ctx->tree;
  // small sets take coarser keys and half the passes (their cost is the
  // launches); both pass counts are even, so the sorted slots end in
  // ctx->order, and the second buffers are the front of the gather buffer
  const int bits = n <= SMALL_SORT ? SMALL_KEY_BITS : KEY_BITS;
  const int passes = (3 * bits + RADIX_BITS - 1) / RADIX_BITS;
  const double scale = (double)(1 << bits);
  key_k<<<blocks_for(n, BS), BS, 0, st>>>(n, pp->x, pp->y, pp->z, scale / g.box[0],
                                          scale / g.box[1], scale / g.box[2], bits, ctx->code,
                                          ctx->order);
  uint32_t *ka = ctx->code, *kb = reinterpret_cast<uint32_t *>(ctx->tmp);
  int32_t *va = ctx->order, *vb = reinterpret_cast<int32_t *>(ctx->tmp) + n;
  const int nb = blocks_for(n, SORT_TILE);
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RADIX_BITS;
    radix_hist_k<<<nb, SORT_BS, 0, st>>>(n, ka, shift, nb, ctx->hist);
    hipError_t e = scan_exclusive(st, ctx->hist, ctx->hist, (int64_t)RADIX * nb, ctx->scan_tmp);
    if (e != hipSuccess) return e;
    radix_scatter_k<<<nb, SORT_BS, 0, st>>>(n, ka, va, shift, nb, ctx->hist, kb, vb);
    uint32_t *tk = ka;
    ka = kb;
    kb = tk;
    int32_t *tv = va;
    va = vb;
    vb = tv;
  }
  Fields fs;
  double *src[10] = {pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz, pp->m, pp->E, pp->U, pp->H};
  for (int f = 0; f < 10; ++f) fs.f[f] = src[f];
  fs.id = pp->id;
  fs.x[0] = pp->S;
  for (int e = 0; e < 3; ++e) fs.x[1 + e] = pp->accel ? pp->accel + (int64_t)e * n : nullptr;
  fs.emode = pp->emode;
  fs.ncand = ctx->ncand;
  fs.rung = ctx->rung_perm;
  gather_k<<<blocks_for(n, BS), BS, 0, st>>>(n, fs, ctx->order, ctx->tmp, perm);
  writeback_k<<<blocks_for(n, BS), BS, 0, st>>>(n, fs, ctx->tmp,
                                                reinterpret_cast<double4 *>(ctx->pos4));
  // the tree over the sorted particles
  return launch_tree(ctx, n);
}

namespace {

// pos4 = (x, y, z, H) of the particles in their present order
__global__ void pos4_k(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ z, const double *__restrict__ H,
                       double4 *pos4) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) pos4[i] = make_double4(x[i], y[i], z[i], H[i]);
}

}  // namespace

hipError_t launch_refresh_cells(mfm_ctx *ctx, const mfm_particles *pp) {
  pos4_k<<<blocks_for(pp->n, BS), BS, 0, ctx->stream>>>(
      pp->n, pp->x, pp->y, pp->z, pp->H, reinterpret_cast<double4 *>(ctx->pos4));
  return launch_tree(ctx, pp->n);
}

hipError_t launch_tree(mfm_ctx *ctx, int64_t n) {
  hipStream_t st = ctx->stream;
  const Tree &g = ctx->tree;
  leaf_box_k<<<g.lev_cnt[0], 64, 0, st>>>(n, reinterpret_cast<const double4 *>(ctx->pos4),
                                           g.hfac, ctx->tnode + (int64_t)g.lev_off[0] * TNODE);
  for (int l = 1; l < g.nlev; ++l)
    inner_box_k<<<blocks_for(g.lev_cnt[l], 64), 64, 0, st>>>(
        ctx->tnode + (int64_t)g.lev_off[l - 1] * TNODE, g.lev_cnt[l - 1],
        ctx->tnode + (int64_t)g.lev_off[l] * TNODE, g.lev_cnt[l]);
  return hipGetLastError();
}
