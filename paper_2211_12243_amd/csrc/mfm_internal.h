// mfm_internal.h -- device helpers, context layout and launcher declarations
// shared by the HIP translation units of libmfm.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mfm.h"

// ---------------------------------------------------------------------------
// Device counters (int64 slots in the workspace).  The order matches the
// leading int64 fields of mfm_diag.
// ---------------------------------------------------------------------------
enum {
  C_H_NOCONV = 0,
  C_NCOND_BOOSTS,
  C_NCOND_FAIL,
  C_CELL_REBUILDS,
  C_LIST_OVERFLOW,
  C_GRAD_PAIRS,
  C_FACES,
  C_RIEMANN_ITERS,
  C_RIEMANN_MAXIT,
  C_VACUUM,
  C_POSITIVITY,
  C_NEG_MASS,
  C_SINGULAR_E,
  C_GUESS_FALLBACK,
  C_FP64_INVERSE,
  C_U_GUARD,
  C_HARD_FACES,
  C_HARD_OVERFLOW,
  C_NONFINITE,      // internal: non-finite dt or state (cleared per step)
  // the density pass in flight (cleared before each pass); its counts are
  // folded into the slots above only when the pass is accepted (a pass whose
  // H outgrew the cells is redone)
  C_CELL_OVERFLOW,  // some H reached its bracket (cell_margin H at the build, or half the box)
  C_PASS_NOCONV,
  C_PASS_BOOSTS,
  C_PASS_FAIL,
  C_PASS_LIST,      // particles whose candidate list overflowed
  C_STEP_SKIP,      // the pass is rejected: the kernels after it return at once
  C_DUMP_COUNT,     // face records appended since the dump was armed
  C_LIST_POOL,      // the planned list blocks exceed the list pool (set by each plan)
  C_GRAD_QUEUE,     // mixed path: particles queued for the gradient loop's FP64 redo
  C_RUNG_CHANGED,   // the rung limiter raised some rung in its last sweep
  C_RUNG_DEEP,      // particles whose step needs a rung beyond MFM_RUNG_MAX
  C_LONG_QUEUE,     // density loop: particles queued for the wavefront-per-particle pass
  C_CHUNK_QUEUE,    // sub-steps: 16-particle chunks with an active particle, queued for the search
  NCOUNTERS = 32
};
static_assert(C_CHUNK_QUEUE < NCOUNTERS, "every counter has its slot");

// Packed per-particle record the gradient loop gathers for each neighbour
// (written by the density loop; one 128-byte line).
enum { GIN_X = 0, GIN_Y, GIN_Z, GIN_H, GIN_V, GIN_RHO, GIN_VX, GIN_VY, GIN_VZ, GIN_P, GIN_C,
       GIN_F32 = 12,  // from here: V, rho, P, c rounded to FP32 (the mixed path's gather)
       GIN_STRIDE = 16 };

// Packed per-particle record the flux loop gathers for each face side
// (written by the gradient loop; two 128-byte lines).
enum {
  R_X = 0, R_Y, R_Z,
  R_IH = 3,     // 1 / H
  R_V = 4,      // volume
  R_RHO = 5,    // primitives rho, vx, vy, vz, P at 5..10 (with 1/rho at 6)
  R_IRHO = 6,
  R_VX = 7, R_VY = 8, R_VZ = 9, R_P = 10,
  R_B = 11,     // 6 entries of B = E^-1
  R_G = 17,     // 15 entries of the limited gradients (rho, vx, vy, vz, P) x (x, y, z)
  R_STRIDE = 32
};

// The mixed path's FP32 flux record (one 128-byte line; positions stay FP64
// in the position array).
enum {
  F_IH = 0, F_V = 1, F_RHO = 2, F_IRHO = 3, F_VX = 4, F_VY = 5, F_VZ = 6, F_P = 7,
  F_B = 8,      // 6 entries of B
  F_G = 14,     // 15 entries of the limited gradients
  F_STRIDE = 32
};

// The neighbour search's bucket tree (sec. 2.2.3: the paper searches
// neighbours per bucket of particles).  Level 0 has one node per bucket of
// BUCKET consecutive particles of the Z-ordered array; a node of level l + 1
// covers TREE_FANOUT consecutive nodes of level l; the top level has one
// node.  A node holds the bounding box of its particles and R, cell_margin
// times their largest H at the build (the largest candidate radius inside).
constexpr int BUCKET = 64;
constexpr int TREE_FANOUT = 8;
constexpr int MAX_TREE_LEVELS = 12;
constexpr int TNODE = 8;  // doubles per node: min x, y, z, max x, y, z, R, spread mask
constexpr int TNODE_SPREAD = 7;  // leaves: bit c set when chunk c of the bucket is spread
// A chunk of LCH particles is "spread" when its box's half-diagonal exceeds
// SPREAD_RATIO times its particles' mean search radius; the search takes it
// a few particles at a time.
constexpr double SPREAD_RATIO = 3.0;

// The particle order: Morton keys of KEY_BITS bits per axis (SMALL_KEY_BITS
// for sets of at most SMALL_SORT particles), sorted by a stable
// least-significant-digit radix sort of RADIX_BITS-bit digits: 4 passes, or
// 2 for the small sets (an even number, so that the result lands back in the
// primary buffers).
constexpr int KEY_BITS = 10;
constexpr int SMALL_KEY_BITS = 5;
constexpr int64_t SMALL_SORT = 1 << 16;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
static_assert((3 * KEY_BITS + RADIX_BITS - 1) / RADIX_BITS % 2 == 0 &&
                  (3 * SMALL_KEY_BITS + RADIX_BITS - 1) / RADIX_BITS % 2 == 0,
              "the sort must take an even number of passes");
constexpr int SORT_BS = RADIX;   // threads per sort workgroup (one per digit)
constexpr int SORT_ITEMS = 16;   // items per thread
constexpr int SORT_TILE = SORT_BS * SORT_ITEMS;

// Individual time steps (sec. 2.3.4, sec. 2.3.10), passed by value to the
// kernels of a sub-step.  rung == null: one global step (every particle
// active, the step from the dt argument).
struct Rungs {
  const int32_t *rung;     // each particle's rung: its step is 2^-rung dt0
  int32_t *s0;             // the sub-step at which its current step began
  const uint8_t *act;      // 1 where its step begins at this sub-step
  const double *elapsed;   // (k - s0) times the sub-step: time since its step began
  double dt0;              // the base step
  int rmax;                // the deepest rung: 2^rmax sub-steps
  int64_t k;               // this sub-step
};
// 2^-r dt, by halving (exact)
__host__ __device__ __forceinline__ double rung_step(double dt, int r) {
  for (int k = 0; k < r; ++k) dt *= 0.5;
  return dt;
}

// Geometry of the box and the tree, passed by value to kernels.
struct Tree {
  double box[3];      // periodic sides
  double half[3];     // box / 2
  double side_min;    // bound on any H: half the smallest side (minimum image)
  double hfac;        // cell_margin (times the rebuild boost): bound on H / H at the build
  const double *node; // TNODE doubles per tree node, level by level
  int nlev;           // tree levels (the top one has one node)
  int lev_off[MAX_TREE_LEVELS], lev_cnt[MAX_TREE_LEVELS];
};

constexpr int MAX_EVENT_PAIRS = 1024;  // timed launches held between two harvests

struct mfm_ctx {
  mfm_params p;
  int64_t n_max;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  // workspace carve
  uint32_t *code;      // n: Morton key of each particle
  int32_t *hist;       // RADIX per sort workgroup: digit counts, then first slots
  double *tnode;       // the bucket tree, TNODE doubles per node
  int32_t *scan_tmp;   // block sums of the scans
  int32_t *order;      // n: input slot of each sorted slot
  double *tmp;         // 17 n doubles: gather buffer of the permutation (its front
                       // doubles as the sort's second key and value buffers)
  double *pos4;        // 4 n: (x, y, z, H at the build) per particle
  int64_t *lseg;       // list_chunks(n) + 1: each chunk's first pool entry (list_at)
  int64_t *lcap;       // list_chunks(n) + 1: the planned block sizes before their scan
  int64_t *scan64;     // block sums of that scan
  int32_t *ncand;      // n: each particle's candidate count in the last search (permuted with it)
  int64_t pool;        // pool entries (list_len)
  int have_need;       // ncand holds the last search's counts for need_n particles
  int64_t need_n;
  int32_t *cand;       // pool: candidates (r < cell_margin max(H_i, H_j) at the build);
                       // after the density loop: the candidates with r >= H_i
  double *cand_r2;     // pool: their squared distances (FP64, from the search)
  float *rest_r2;      // pool: squared distances of the r >= H_i list, rounded to FP32
  int32_t *cand_cnt;   // n
  int32_t *gl;         // pool: gather set r < H_i of each particle, from the density loop
  int32_t *gl_cnt;     // n
  double *gin;         // GIN_STRIDE * n packed gradient-loop records
  int32_t *fslot;      // pool: faces each particle evaluates
  int32_t *fcnt;       // n
  double *dq_ext;      // 5 n: flux contributions to particles outside the evaluating block
                       // and of the FP64 second pass, folded into dQ after the loop
  int2 *hard_q;        // faces (lower, higher slot) queued for the flux loop's FP64 pass:
                       // HARD_SEGS segments of hard_cap / HARD_SEGS faces
  int64_t hard_cap;    // its capacity
  unsigned long long *hard_len;  // the segments' lengths (HARD_SEG_STRIDE apart)
  double *rec;         // R_STRIDE * n packed flux records
  double *ekm;         // n: E_kin^max of the entropy switch (gradient loop)
  int32_t *grad_q;     // n: particles queued for the mixed gradient loop's FP64 redo
  // individual time steps (mfm_step_rungs)
  int32_t *rung_w;     // n: rungs
  int32_t *s0_w;       // n: sub-step at which each particle's step began
  uint8_t *act_w;      // n: active flags of the current sub-step
  double *elapsed_w;   // n: time since each particle's step began
  Rungs rungs;         // rungs.rung == null outside mfm_step_rungs
  int32_t *rung_perm;  // the caller's given rungs, permuted by the build (null: none)
  double *gwork;       // 3 n: sum_j dm_ij (x_j - x_i) (flux loop, MFV with gravity)
  // comoving integration (mfm_set_cosmology)
  double inv_a, hubble_n, hubble_np1;
  double *red;         // reduction partials
  int64_t *counters;   // NCOUNTERS
  double *scalars;     // small device scalars: [0] max H, [1] dt, [2..6] conserved sums
  size_t scan_tmp_len, red_len;
  // current tree geometry
  Tree tree;
  double margin_boost;
  int overflow_streak;  // density passes in a row rejected for an outgrown H
  int have_cells, have_density, have_grad;
  int64_t n_cells_built;  // n of the particles the cells were built for
  // learned guess and face dump
  const void *mlp_state;  // network state (mfm_mlp_attach), null if none
  float *dump;            // face records (mfm_face_dump), null when off
  int64_t dump_cap;
  unsigned long long *dump_count;  // = counters + C_DUMP_COUNT
  // timing
  int timing, ev_created;
  hipEvent_t ev_pool[2 * MAX_EVENT_PAIRS];
  int ev_stage[MAX_EVENT_PAIRS];
  int ev_open[MAX_EVENT_PAIRS];
  int ev_used;
  double stage_ms[MFM_NSTAGES];
  int64_t stage_count[MFM_NSTAGES];
  int static_dev;  // 1 + the GPU whose static scratch this context uses (0: caller's workspace)
  // individual steps: pinned host copy of the counters and the event after
  // which it holds a sub-step's values (made on first use; none on a static
  // context, which reads the counters with a plain synchronising copy)
  int64_t *host_ctr;
  hipEvent_t ev_ctr;
  // mfm_step's reuse of the particle order: keep_order says the next step
  // may skip the sort (set at the end of a step, for the arrays order_x of
  // order_n particles); ev_ord time the cells, search and density stages
  // of a step (made on first use; none on a static context, which always
  // sorts), ms_sorted is that time in the step of the last sort, steps_kept
  // the steps since
  int keep_order, steps_kept, ev_ord_made;
  hipEvent_t ev_ord[2];
  float ms_sorted;
  const double *order_x;
  int64_t order_n;
  char err[512];
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Minimum-image separation along one periodic axis of side L.
__device__ __forceinline__ double min_image(double d, double L, double half) {
  if (d > half)
    d -= L;
  else if (d < -half)
    d += L;
  return d;
}

// Cubic spline shape in compact-support form: W(r, H) = 8/(pi H^3) w(r/H).
__device__ __forceinline__ double spline_w(double q) {
  if (q < 0.5) return 1.0 + q * q * (6.0 * q - 6.0);
  if (q < 1.0) {
    double t = 1.0 - q;
    return 2.0 * t * t * t;
  }
  return 0.0;
}
// q * dw/dq
__device__ __forceinline__ double spline_qdw(double q) {
  if (q < 0.5) return q * q * (18.0 * q - 12.0);
  if (q < 1.0) {
    double t = 1.0 - q;
    return -6.0 * q * t * t;
  }
  return 0.0;
}

__device__ __forceinline__ uint32_t spread_bits3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t morton3(int cx, int cy, int cz) {
  return spread_bits3((uint32_t)cx) | (spread_bits3((uint32_t)cy) << 1) |
         (spread_bits3((uint32_t)cz) << 2);
}
// 64-lane wave reductions.
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Add a per-lane count to a device counter with one atomic per wave.
__device__ __forceinline__ void count_add(int64_t *ctr, int64_t v) {
  int64_t s = wave_sum_i64(v);
  if ((threadIdx.x & 63) == 0 && s != 0) atomicAdd((unsigned long long *)ctr, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// Launchers (host side), one translation unit each.  All enqueue on ctx->stream
// and return a hipError_t.
// ---------------------------------------------------------------------------
// After a density pass: reject it (C_STEP_SKIP) if a candidate list
// overflowed or an H outgrew its bound; else fold the pass counts into the
// running counters.
hipError_t launch_validate(mfm_ctx *ctx);
hipError_t launch_build_cells(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm);
// Exclusive int64 scan (in place allowed); tmp: block sums of every level,
// scan_len(n) entries.
hipError_t scan_exclusive_i64(hipStream_t st, const int64_t *in, int64_t *out, int64_t n,
                              int64_t *tmp);
static inline size_t scan_len(int64_t n) {
  size_t len = 64;
  for (int64_t m = n; m > 1; m = (m + 1023) / 1024) len += (size_t)(m + 1023) / 1024;
  return len;
}
// The neighbour search.  count_only: record each particle's candidate count
// in ncand and write no list (the first search of a context).
hipError_t launch_candidates(mfm_ctx *ctx, const mfm_particles *pp, bool count_only);
// Plan the list blocks from ncand (plus a margin): lseg, and C_LIST_POOL when
// they exceed the pool.
hipError_t launch_plan_lists(mfm_ctx *ctx, int64_t n);
hipError_t launch_density(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_gradients(mfm_ctx *ctx, const mfm_particles *pp, double dt_max, double *dt_dev);
// Times the whole flux loop as stage 4, its first-pass kernel as stage 6 and
// its FP64 second pass as stage 7.
hipError_t launch_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev);
hipError_t launch_update(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev);
// The bucket tree over the particles' current positions (pos4), in the
// current order.
hipError_t launch_tree(mfm_ctx *ctx, int64_t n);
// pos4 from the particle arrays in their present order, then the tree (no sort)
hipError_t launch_refresh_cells(mfm_ctx *ctx, const mfm_particles *pp);
// Individual time steps: rungs from dt_i (or given), one limiter sweep over
// the face lists, the active set and predicted positions of sub-step k.
hipError_t launch_rungs_from_dt(mfm_ctx *ctx, const mfm_particles *pp, double dt0);
hipError_t launch_rung_limiter(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_rmax(mfm_ctx *ctx, int64_t n, int32_t *rmax_dev);
hipError_t launch_rung_check(mfm_ctx *ctx, int64_t n);  // given rungs: out of range -> C_RUNG_DEEP
hipError_t launch_substep_begin(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_conserved(mfm_ctx *ctx, const mfm_particles *pp);

// device pointers of a network state (mlp translation unit); net_out is an mlp::Net
const void *mlp_net_of(const void *state, void *net_out);

// timing helpers (api translation unit): stage_begin records a start event
// for the stage and returns its slot (-1 when timing is off or the pool is
// full), stage_end the matching end event; pairs may nest
int stage_begin(mfm_ctx *ctx, int stage);
void stage_end(mfm_ctx *ctx, int slot);

// The hardware hands workgroup b of a launch to XCD b % 8, and each XCD has
// its own L2.  The neighbour loops renumber their workgroups so that every XCD
// works through one contiguous range of the sorted (hence spatially compact)
// particles and its L2 keeps serving the same neighbours.  A bijection on
// [0, nb): XCD x takes nb / 8 workgroups, plus one if x < nb % 8.
constexpr int NUM_XCD = 8;

// mfm_step keeps the particle order for at most KEEP_MAX_STEPS steps
constexpr int KEEP_MAX_STEPS = 16;
__host__ __device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / NUM_XCD, r = nb % NUM_XCD, x = b % NUM_XCD;
  return x * q + (x < r ? x : r) + b / NUM_XCD;
}

static inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// Per-particle lists (candidates, gather sets, faces) live in a pool shared
// by chunks of LCH consecutive particles.  Chunk c owns the block
// [lseg[c], lseg[c + 1]): LCH * K_c entries, entry k of particle i at
// lseg[i / LCH] + k * LCH + i % LCH, so the loops read entry k of
// consecutive particles in one coalesced access.  K_c, the chunk's capacity,
// is planned from the longest candidate list the chunk had in the last
// search (plus a margin), so the pool follows the lists' real lengths, not
// the longest list of the set.
constexpr int LCH = 16;
__device__ __forceinline__ int64_t list_base(const int64_t *__restrict__ lseg, int64_t i) {
  return lseg[i / LCH] + i % LCH;
}
__host__ __device__ __forceinline__ int64_t list_at(int64_t base, int k) {
  return base + (int64_t)k * LCH;
}
static inline int64_t list_chunks(int64_t n) { return (n + LCH - 1) / LCH; }
// entries of the pool: max_list per particle slot of the chunks
static inline size_t list_len(int max_list, int64_t n) {
  return (size_t)max_list * (size_t)(list_chunks(n) * LCH);
}

// Particles per workgroup of the flux loop.  Every face is computed once, by
// the block of the particle that lists it; a partner in another block receives
// its share through FP64 global atomics (see fluxes.hip).  On a Morton-ordered
// lattice about 25% of the faces cross a 1024-particle block boundary (38% for
// 256), so larger blocks send fewer shares through HBM atomics.
constexpr int FLUX_BLOCK = 1024;

// The flux loop's FP64 second pass takes its faces from HARD_SEGS queues,
// each with its own append counter (HARD_SEG_STRIDE 8-byte words apart, on
// separate cache lines): where most faces are handed over (strong jumps
// everywhere) a single counter serialises millions of same-address atomics.
constexpr int HARD_SEGS = 32;
constexpr int HARD_SEG_STRIDE = 32;
static_assert((HARD_SEGS & (HARD_SEGS - 1)) == 0, "the second pass bisects the segments");

// Exactly one of emit(i, j), emit(j, i) holds, and about half of any
// particle's in-block faces are its own whatever its rank in the block.
__device__ __forceinline__ bool emit_face(int i, int j) {
  return ((i ^ j) & 1) ? (i < j) : (i > j);
}
