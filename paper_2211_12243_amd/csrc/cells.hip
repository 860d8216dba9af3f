// cells.hip -- neighbour-cell build: Morton order of cells, counting sort of
// the particles into it, and the in-place permutation of the state arrays.
//
// The paper reorders its particle array so that the particles of a tree node
// are contiguous (sec. 2.2.1) and searches neighbours per bucket of particles
// (sec. 2.2.3).  Here the buckets are cells of a uniform periodic grid whose
// side is at least the largest support radius, laid out along a Z-order curve,
// so every pair closer than max(H_i, H_j) is found in the 27 cells around a
// particle's own, and a 64-lane wavefront of consecutive particles touches a
// compact set of cells.
#include "mfm_internal.h"

namespace {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 1024;

__global__ void fill_i32_k(int32_t *a, int64_t n, int32_t v) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    a[k] = v;
}

__global__ void max_partial_k(const double *__restrict__ v, int64_t n, double *partial) {
  __shared__ double s[BS / 64];
  double m = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, v[k]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BS / 64; ++w) m = fmax(m, s[w]);
    partial[blockIdx.x] = m;
  }
}

__global__ void max_final_k(const double *partial, int np, double *out) {
  __shared__ double s[BS / 64];
  double m = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) m = fmax(m, partial[k]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BS / 64; ++w) m = fmax(m, s[w]);
    out[0] = m;
  }
}

// Runs of equal keys among the lanes of a wavefront (every lane must take
// part): whether this lane starts a run, the run's length (valid at its
// start) and the lane that starts this lane's run.  The particles arrive in
// last step's cell order, so runs are long and one atomic per run replaces
// one per particle.
__device__ __forceinline__ void key_runs(uint32_t key, int lane, bool &head, int &len,
                                         int &head_lane) {
  const uint32_t prev = __shfl_up(key, 1, 64);
  head = lane == 0 || prev != key;
  const uint64_t hm = __ballot(head);
  const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0..lane (all 64 bits at lane 63)
  const uint64_t after = hm & ~upto;
  len = (after ? __ffsll((unsigned long long)after) - 1 : 64) - lane;
  head_lane = 63 - __clzll(hm & upto);
}

constexpr uint32_t NO_KEY = 0xffffffffu;  // lanes past the end (no cell has this code)

// Morton code of each particle's cell and the per-cell histogram.
__global__ void cell_code_k(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, CellGrid g, uint32_t *code,
                            int32_t *count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool live = i < n;
  uint32_t c = NO_KEY;
  if (live) {
    const int cx = cell_coord(x[i], g.inv[0], g.nc[0]);
    const int cy = cell_coord(y[i], g.inv[1], g.nc[1]);
    const int cz = cell_coord(z[i], g.inv[2], g.nc[2]);
    c = morton3(cx, cy, cz);
    code[i] = c;
  }
  bool head;
  int len, hl;
  key_runs(c, lane, head, len, hl);
  if (live && head) atomicAdd(count + c, len);
}

// Exclusive scan, 1024 elements per block (4 per thread), block totals out.
__global__ void scan_block_k(const int32_t *in, int32_t *out, int64_t n, int32_t *block_sums) {
  __shared__ int32_t s[BS];
  int64_t base = blockIdx.x * (int64_t)(4 * BS) + 4 * threadIdx.x;
  int32_t v[4];
  int32_t t = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    t += v[k];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    int32_t add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = s[threadIdx.x] - t;  // exclusive prefix of this thread
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == BS - 1) block_sums[blockIdx.x] = s[BS - 1];
}

__global__ void scan_add_k(int32_t *out, int64_t n, const int32_t *block_offsets) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_offsets[i / (4 * BS)];
}

hipError_t scan_exclusive(hipStream_t st, const int32_t *in, int32_t *out, int64_t n,
                          int32_t *tmp) {
  int64_t nb = (n + 4 * BS - 1) / (4 * BS);
  scan_block_k<<<(int)nb, BS, 0, st>>>(in, out, n, tmp);
  if (nb > 1) {
    hipError_t e = scan_exclusive(st, tmp, tmp, nb, tmp + nb);
    if (e != hipSuccess) return e;
    scan_add_k<<<blocks_for(n, BS), BS, 0, st>>>(out, n, tmp);
  }
  return hipGetLastError();
}

__global__ void scatter_k(int64_t n, const uint32_t *__restrict__ code, int32_t *cursor,
                          int32_t *order) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool live = i < n;
  const uint32_t c = live ? code[i] : NO_KEY;
  bool head;
  int len, hl;
  key_runs(c, lane, head, len, hl);
  int base = 0;
  if (live && head) base = atomicAdd(cursor + c, len);
  base = __shfl(base, hl, 64);
  if (live) order[base + (lane - hl)] = (int32_t)i;
}

// Within a cell, order the particles by their slot before the sort, so the
// result does not depend on the order the atomics were served in.  One
// wavefront per cell (grid-stride over the cell codes): a lane holds one
// member, and its place is the number of smaller members (the slots are
// distinct).  A cell of more than 64 particles is sorted by one lane.
__global__ void cell_sort_k(int64_t ncodes, const int32_t *__restrict__ start,
                            const int32_t *__restrict__ count, int32_t *order) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; c < ncodes; c += nw) {
    const int k = count[c];  // the same in every lane: the branches below are uniform
    if (k < 2) continue;
    int32_t *a = order + start[c];
    if (k <= 64) {
      const int32_t v = lane < k ? a[lane] : 0x7fffffff;
      int rank = 0;
      for (int t = 0; t < k; ++t) rank += __builtin_amdgcn_readlane(v, t) < v ? 1 : 0;
      if (lane < k) a[rank] = v;  // every read above has completed
    } else if (lane == 0) {
      for (int s = 1; s < k; ++s) {
        int32_t v = a[s];
        int t = s - 1;
        while (t >= 0 && a[t] > v) {
          a[t + 1] = a[t];
          --t;
        }
        a[t + 1] = v;
      }
    }
  }
}

__global__ void range_k(int64_t ncodes, const int32_t *__restrict__ start,
                        const int32_t *__restrict__ count, int2 *range) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < ncodes) range[c] = make_int2(start[c], count[c]);
}

// The state arrays the permutation moves: the ten FP64 fields, the labels,
// and the optional source-term arrays (entropy, the three acceleration
// components, the entropy-mode flags); absent ones are null.
struct Fields {
  double *f[10];
  int64_t *id;
  double *x[4];
  int32_t *emode;
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
  pos4[k] = make_double4(tmp[k], tmp[n + k], tmp[2 * n + k], tmp[9 * n + k]);
}

}  // namespace

hipError_t launch_max_h(mfm_ctx *ctx, const mfm_particles *pp) {
  max_partial_k<<<RED_BLOCKS, BS, 0, ctx->stream>>>(pp->H, pp->n, ctx->red);
  max_final_k<<<1, BS, 0, ctx->stream>>>(ctx->red, RED_BLOCKS, ctx->scalars);
  return hipGetLastError();
}

hipError_t launch_build_cells(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm) {
  hipStream_t st = ctx->stream;
  const int64_t n = pp->n;
  const CellGrid &g = ctx->grid;
  int fb = (int)(ctx->ncodes / BS + 1);
  if (fb > 4096) fb = 4096;
  fill_i32_k<<<fb, BS, 0, st>>>(ctx->cell_count, ctx->ncodes, 0);
  cell_code_k<<<blocks_for(n, BS), BS, 0, st>>>(n, pp->x, pp->y, pp->z, g, ctx->code,
                                                 ctx->cell_count);
  hipError_t e = scan_exclusive(st, ctx->cell_count, ctx->cell_start, ctx->ncodes, ctx->scan_tmp);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(ctx->cursor, ctx->cell_start, ctx->ncodes * sizeof(int32_t),
                     hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  scatter_k<<<blocks_for(n, BS), BS, 0, st>>>(n, ctx->code, ctx->cursor, ctx->order);
  int sb = (int)((ctx->ncodes + BS / 64 - 1) / (BS / 64));  // one wavefront per cell code
  if (sb > 16384) sb = 16384;
  cell_sort_k<<<sb, BS, 0, st>>>(ctx->ncodes, ctx->cell_start, ctx->cell_count, ctx->order);
  range_k<<<blocks_for(ctx->ncodes, BS), BS, 0, st>>>(ctx->ncodes, ctx->cell_start,
                                                       ctx->cell_count, ctx->crange);
  Fields fs;
  double *src[10] = {pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz, pp->m, pp->E, pp->U, pp->H};
  for (int f = 0; f < 10; ++f) fs.f[f] = src[f];
  fs.id = pp->id;
  fs.x[0] = pp->S;
  for (int e = 0; e < 3; ++e) fs.x[1 + e] = pp->accel ? pp->accel + (int64_t)e * n : nullptr;
  fs.emode = pp->emode;
  gather_k<<<blocks_for(n, BS), BS, 0, st>>>(n, fs, ctx->order, ctx->tmp, perm);
  writeback_k<<<blocks_for(n, BS), BS, 0, st>>>(n, fs, ctx->tmp,
                                                reinterpret_cast<double4 *>(ctx->pos4));
  return hipGetLastError();
}
