// mfm_api.hip -- the C ABI declared in include/mfm.h: parameter checks,
// workspace carving, launch order, error reporting and event timing.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "mfm_internal.h"

namespace {

constexpr size_t ALIGN = 256;

struct Layout {
  size_t code, hist, tnode, scan, lseg, lcap, scan64, ncand, order, tmp, pos4, cand, cand_r2, rest_r2,
      cand_cnt, gl, gl_cnt, gin, fslot, fcnt, dq_ext, hard_q, hard_len, rec, ekm, grad_q, rung,
      s0, act,
      elapsed, gwork, red, counters,
      scalars;
  int64_t hard_cap;
  size_t total;
  size_t scan_len;
};


size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

Layout make_layout(const mfm_params *p, int64_t n) {
  Layout L;
  // the sort's digit counts: RADIX per workgroup tile, and the block sums
  // of their scan
  const int64_t hist_len = (int64_t)RADIX * ((n + SORT_TILE - 1) / SORT_TILE);
  L.scan_len = scan_len(hist_len);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += up(bytes);
    return o;
  };
  L.code = take(4 * (size_t)n);
  L.hist = take(4 * (size_t)hist_len);
  // tree nodes: one per bucket, then each level an eighth of the last
  int64_t nodes = 0;
  for (int64_t c = (n + BUCKET - 1) / BUCKET;; c = (c + TREE_FANOUT - 1) / TREE_FANOUT) {
    nodes += c;
    if (c <= 1) break;
  }
  L.tnode = take(8 * TNODE * (size_t)nodes);
  L.scan = take(4 * L.scan_len);
  // the list blocks: one per chunk of LCH particles, planned and scanned
  const int64_t nch = list_chunks(n);
  L.lseg = take(8 * (size_t)(nch + 1));
  L.lcap = take(8 * (size_t)(nch + 1));
  L.scan64 = take(8 * scan_len(nch + 1));
  L.ncand = take(4 * (size_t)n);
  L.order = take(4 * (size_t)n);
  L.tmp = take(8 * 17 * (size_t)n);
  L.pos4 = take(32 * (size_t)n);
  L.cand = take(4 * list_len(p->max_list, n));
  L.cand_r2 = take(8 * list_len(p->max_list, n));
  L.rest_r2 = take(4 * list_len(p->max_list, n));
  L.cand_cnt = take(4 * (size_t)n);
  L.gl = take(4 * list_len(p->max_list, n));
  L.gl_cnt = take(4 * (size_t)n);
  L.gin = take(8 * (size_t)GIN_STRIDE * (size_t)n);
  L.fslot = take(4 * list_len(p->max_list, n));
  L.fcnt = take(4 * (size_t)n);
  L.dq_ext = take(8 * 5 * (size_t)n);
  // the FP64 pass's queue holds as many faces as half the face lists, in
  // HARD_SEGS equal segments
  L.hard_cap = (int64_t)(list_len(p->max_list, n) / 2) / HARD_SEGS * HARD_SEGS;
  L.hard_q = take(8 * (size_t)L.hard_cap);
  L.hard_len = take(8 * (size_t)HARD_SEGS * HARD_SEG_STRIDE);
  L.rec = take(8 * (size_t)R_STRIDE * (size_t)n);
  L.ekm = take(8 * (size_t)n);
  L.grad_q = take(4 * (size_t)n);
  L.rung = take(4 * (size_t)n);
  L.s0 = take(4 * (size_t)n);
  L.act = take((size_t)n);
  L.elapsed = take(8 * (size_t)n);
  L.gwork = take(8 * 3 * (size_t)n);
  L.red = take(8 * 5 * 1024);
  L.counters = take(8 * NCOUNTERS);
  L.scalars = take(8 * 16);
  L.total = off;
  return L;
}

int check_params(const mfm_params *p) {
  if (!p) return 0;
  if (p->scheme != MFM_SCHEME_MFV && p->scheme != MFM_SCHEME_MFM) return 0;
  if (p->precision != MFM_FP64 && p->precision != MFM_MIXED) return 0;
  if (p->guess != MFM_GUESS_PLAIN && p->guess != MFM_GUESS_LEARNED) return 0;
  if (p->limiter < 0 || p->limiter > (MFM_LIMIT_BJ | MFM_LIMIT_PAIRWISE)) return 0;
  if (!(p->gamma > 1.0)) return 0;
  if (!(p->n_ngb > 32.0 / 3.0)) return 0;
  if (!(p->ncond_max > 1.0) || !(p->ngb_boost > 1.0) || p->max_boosts < 0) return 0;
  if (!(p->h_tol > 0.0) || p->h_maxit < 1) return 0;
  if (!(p->c_cfl > 0.0)) return 0;
  if (!(p->riemann_tol > 0.0) || p->riemann_maxit < 1) return 0;
  if (p->max_list < 1 || p->max_list > 4096) return 0;
  if (!(p->cell_margin >= 1.0)) return 0;
  if (p->reserved != 0) return 0;
  if (!(p->mixed_jump == 0.0 || p->mixed_jump >= 1.0)) return 0;
  if (!(p->alpha2 >= 0.0) || !(p->alpha3 >= 0.0)) return 0;
  if (p->entropy_switch != 0 && p->entropy_switch != 1) return 0;
  for (int k = 0; k < 3; ++k)
    if (!(p->box[k] > 0.0)) return 0;
  return 1;
}

int check_parts(const mfm_ctx *ctx, const mfm_particles *pp) {
  if (!pp || pp->n <= 0 || pp->n > ctx->n_max || pp->n > 0x7fffffff) return 0;
  const void *req[] = {pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz, pp->m, pp->E, pp->U,
                       pp->H, pp->V, pp->rho, pp->P, pp->c, pp->ncond, pp->B, pp->grad,
                       pp->dQ, pp->dt_i};
  for (const void *q : req)
    if (!q) return 0;
  if (ctx->p.entropy_switch && (!pp->S || !pp->emode)) return 0;
  return 1;
}

int fail(mfm_ctx *ctx, int code, const char *msg) {
  if (ctx) snprintf(ctx->err, sizeof(ctx->err), "%s", msg);
  return code;
}

int hip_fail(mfm_ctx *ctx, hipError_t e, const char *where) {
  if (ctx) snprintf(ctx->err, sizeof(ctx->err), "%s: %s", where, hipGetErrorString(e));
  return MFM_E_HIP;
}

#define HIPCHK(ctx, expr, where)              \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

int read_counters(mfm_ctx *ctx, int64_t *host) {
  HIPCHK(ctx, hipMemcpyAsync(host, ctx->counters, sizeof(int64_t) * NCOUNTERS,
                             hipMemcpyDeviceToHost, ctx->stream),
         "read counters");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return MFM_OK;
}

// The box and the tree's level sizes, from n and the parameters alone.
int setup_tree(mfm_ctx *ctx, int64_t n) {
  Tree &g = ctx->tree;
  g.hfac = ctx->p.cell_margin * ctx->margin_boost;
  g.side_min = 1e300;
  for (int k = 0; k < 3; ++k) {
    g.box[k] = ctx->p.box[k];
    g.half[k] = 0.5 * ctx->p.box[k];
    g.side_min = fmin(g.side_min, 0.5 * ctx->p.box[k]);
  }
  g.node = ctx->tnode;
  g.nlev = 0;
  int off = 0;
  for (int64_t c = (n + BUCKET - 1) / BUCKET;; c = (c + TREE_FANOUT - 1) / TREE_FANOUT) {
    if (g.nlev == MAX_TREE_LEVELS) return fail(ctx, MFM_E_ARG, "too many particles for the tree");
    g.lev_off[g.nlev] = off;
    g.lev_cnt[g.nlev] = (int)c;
    ++g.nlev;
    off += (int)c;
    if (c <= 1) break;
  }
  return MFM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
int stage_begin(mfm_ctx *ctx, int stage) {
  if (!ctx->timing || ctx->ev_used >= MAX_EVENT_PAIRS) return -1;
  const int k = ctx->ev_used++;
  ctx->ev_stage[k] = stage;
  ctx->ev_open[k] = 1;
  hipEventRecord(ctx->ev_pool[2 * k], ctx->stream);
  return k;
}

void stage_end(mfm_ctx *ctx, int slot) {
  if (slot < 0) return;
  hipEventRecord(ctx->ev_pool[2 * slot + 1], ctx->stream);
  ctx->ev_open[slot] = 0;
}

static void harvest_events(mfm_ctx *ctx) {
  for (int k = 0; k < ctx->ev_used; ++k) {
    if (ctx->ev_open[k]) continue;
    float ms = 0.0f;
    hipEventSynchronize(ctx->ev_pool[2 * k + 1]);
    if (hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]) == hipSuccess) {
      ctx->stage_ms[ctx->ev_stage[k]] += ms;
      ctx->stage_count[ctx->ev_stage[k]] += 1;
    }
  }
  ctx->ev_used = 0;
}

extern "C" {

void mfm_default_params(mfm_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->scheme = MFM_SCHEME_MFV;
  p->precision = MFM_FP64;
  p->limiter = MFM_LIMIT_BJ | MFM_LIMIT_PAIRWISE;
  p->max_boosts = 5;
  p->h_maxit = 64;
  p->riemann_maxit = 100;
  p->guess = MFM_GUESS_PLAIN;
  p->max_list = 160;
  p->gamma = 5.0 / 3.0;
  p->n_ngb = 32.0;
  p->ncond_max = 100.0;
  p->ngb_boost = 1.2;
  p->h_tol = 1e-13;
  p->c_cfl = 0.2;
  p->psi1 = 0.5;
  p->psi2 = 0.25;
  p->riemann_tol = 1e-10;
  p->alpha1 = 0.01;
  p->box[0] = p->box[1] = p->box[2] = 1.0;
  p->cell_margin = 1.10;
  p->mixed_jump = 8.0;
  p->alpha2 = 1e-3;
  p->alpha3 = 1e-3;
  p->entropy_switch = 0;
}

size_t mfm_workspace_bytes(const mfm_params *p, int64_t n_max) {
  if (!check_params(p) || n_max <= 0) return 0;
  return make_layout(p, n_max).total;
}

}  // extern "C"

namespace {

// Fill a zeroed context: parameters, stream and the carve of its workspace;
// clear its counters.
int init_ctx(mfm_ctx *ctx, const mfm_params *p, int64_t n_max, void *workspace,
             size_t workspace_bytes, void *stream) {
  Layout L = make_layout(p, n_max);
  ctx->p = *p;
  ctx->n_max = n_max;
  ctx->stream = (hipStream_t)stream;
  ctx->ws = (char *)workspace;
  ctx->ws_bytes = workspace_bytes;
  ctx->code = (uint32_t *)(ctx->ws + L.code);
  ctx->hist = (int32_t *)(ctx->ws + L.hist);
  ctx->lseg = (int64_t *)(ctx->ws + L.lseg);
  ctx->lcap = (int64_t *)(ctx->ws + L.lcap);
  ctx->scan64 = (int64_t *)(ctx->ws + L.scan64);
  ctx->ncand = (int32_t *)(ctx->ws + L.ncand);
  ctx->pool = (int64_t)list_len(p->max_list, n_max);
  ctx->have_need = 0;
  ctx->need_n = 0;
  ctx->tnode = (double *)(ctx->ws + L.tnode);
  ctx->scan_tmp = (int32_t *)(ctx->ws + L.scan);
  ctx->order = (int32_t *)(ctx->ws + L.order);
  ctx->tmp = (double *)(ctx->ws + L.tmp);
  ctx->pos4 = (double *)(ctx->ws + L.pos4);
  ctx->cand = (int32_t *)(ctx->ws + L.cand);
  ctx->cand_r2 = (double *)(ctx->ws + L.cand_r2);
  ctx->rest_r2 = (float *)(ctx->ws + L.rest_r2);
  ctx->cand_cnt = (int32_t *)(ctx->ws + L.cand_cnt);
  ctx->gin = (double *)(ctx->ws + L.gin);
  ctx->gl = (int32_t *)(ctx->ws + L.gl);
  ctx->gl_cnt = (int32_t *)(ctx->ws + L.gl_cnt);
  ctx->fslot = (int32_t *)(ctx->ws + L.fslot);
  ctx->fcnt = (int32_t *)(ctx->ws + L.fcnt);
  ctx->dq_ext = (double *)(ctx->ws + L.dq_ext);
  ctx->hard_q = (int2 *)(ctx->ws + L.hard_q);
  ctx->hard_len = (unsigned long long *)(ctx->ws + L.hard_len);
  ctx->hard_cap = L.hard_cap;
  ctx->rec = (double *)(ctx->ws + L.rec);
  ctx->ekm = (double *)(ctx->ws + L.ekm);
  ctx->grad_q = (int32_t *)(ctx->ws + L.grad_q);
  ctx->rung_w = (int32_t *)(ctx->ws + L.rung);
  ctx->s0_w = (int32_t *)(ctx->ws + L.s0);
  ctx->act_w = (uint8_t *)(ctx->ws + L.act);
  ctx->elapsed_w = (double *)(ctx->ws + L.elapsed);
  memset(&ctx->rungs, 0, sizeof(ctx->rungs));
  ctx->rung_perm = nullptr;
  ctx->gwork = (double *)(ctx->ws + L.gwork);
  ctx->inv_a = 1.0;
  ctx->hubble_n = ctx->hubble_np1 = 0.0;
  ctx->red = (double *)(ctx->ws + L.red);
  ctx->counters = (int64_t *)(ctx->ws + L.counters);
  ctx->scalars = (double *)(ctx->ws + L.scalars);
  ctx->scan_tmp_len = L.scan_len;
  ctx->margin_boost = 1.0;
  ctx->overflow_streak = 0;
  ctx->dump_count = reinterpret_cast<unsigned long long *>(ctx->counters + C_DUMP_COUNT);
  // counters start at zero whatever the workspace held (the static scratch
  // keeps the last context's contents)
  hipError_t e = hipMemsetAsync(ctx->counters, 0, sizeof(int64_t) * NCOUNTERS, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MFM_OK : MFM_E_HIP;
}

// ---------------------------------------------------------------------------
// The workspace of mfm_create_static: a file-scope device array.  Each GPU
// holds its own copy for the life of the process; host code reaches it only
// through the device address hipGetSymbolAddress returns for that GPU (the
// array's name is a host-side stand-in).  One context per GPU may use it at
// a time; its host context lives in static storage too.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int STATIC_MAX_DEVICES = 16;
__device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];
void *scratch_dev[STATIC_MAX_DEVICES];        // device address per GPU, 0 until looked up
mfm_ctx static_ctx[STATIC_MAX_DEVICES];       // host context per GPU
int static_busy[STATIC_MAX_DEVICES];
std::mutex static_mu;

}  // namespace

extern "C" {

int mfm_create(const mfm_params *p, int64_t n_max, void *workspace, size_t workspace_bytes,
               void *stream, mfm_ctx **out) {
  if (!out) return MFM_E_ARG;
  *out = nullptr;
  if (!check_params(p) || n_max <= 0 || n_max > 0x7fffffff) return MFM_E_ARG;
  Layout L = make_layout(p, n_max);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0)
    return MFM_E_WORKSPACE;
  mfm_ctx *ctx = (mfm_ctx *)calloc(1, sizeof(mfm_ctx));
  if (!ctx) return MFM_E_ARG;
  int rc = init_ctx(ctx, p, n_max, workspace, workspace_bytes, stream);
  if (rc) {
    free(ctx);
    return rc;
  }
  *out = ctx;
  return MFM_OK;
}

size_t mfm_static_workspace_bytes(void) { return STATIC_SCRATCH_BYTES; }

int mfm_create_static(const mfm_params *p, int64_t n_max, void *stream, mfm_ctx **out) {
  if (!out) return MFM_E_ARG;
  *out = nullptr;
  if (!check_params(p) || n_max <= 0 || n_max > 0x7fffffff) return MFM_E_ARG;
  if (make_layout(p, n_max).total > STATIC_SCRATCH_BYTES) return MFM_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES)
    return MFM_E_HIP;
  std::lock_guard<std::mutex> lock(static_mu);
  if (static_busy[dev]) return MFM_E_STATE;
  if (!scratch_dev[dev]) {
    // once per GPU, with that GPU current: the device address of its copy
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MFM_E_HIP;
    scratch_dev[dev] = ptr;
  }
  mfm_ctx *ctx = &static_ctx[dev];
  memset(ctx, 0, sizeof(*ctx));
  int rc = init_ctx(ctx, p, n_max, scratch_dev[dev], STATIC_SCRATCH_BYTES, stream);
  if (rc) return rc;
  ctx->static_dev = dev + 1;
  static_busy[dev] = 1;
  *out = ctx;
  return MFM_OK;
}

int mfm_destroy(mfm_ctx *ctx) {
  if (!ctx) return MFM_E_ARG;
  hipStreamSynchronize(ctx->stream);
  if (ctx->ev_created)
    for (int q = 0; q < 2 * MAX_EVENT_PAIRS; ++q) hipEventDestroy(ctx->ev_pool[q]);
  if (ctx->ev_ord_made) {
    hipEventDestroy(ctx->ev_ord[0]);
    hipEventDestroy(ctx->ev_ord[1]);
    ctx->ev_ord_made = 0;
  }
  if (ctx->host_ctr) {
    hipEventDestroy(ctx->ev_ctr);
    hipHostFree(ctx->host_ctr);
    ctx->host_ctr = nullptr;
  }
  if (ctx->static_dev) {
    std::lock_guard<std::mutex> lock(static_mu);
    static_busy[ctx->static_dev - 1] = 0;
    ctx->static_dev = 0;
    return MFM_OK;
  }
  free(ctx);
  return MFM_OK;
}

}  // extern "C"

namespace {

// After a density pass some of whose H outgrew cell_margin times their value
// at the build: those H now hold estimates of their roots, and the next
// build's radii follow them.  A second such pass in a row widens every
// radius by a tenth as well; the widening outlives the step and decays by 2%
// per accepted pass.
void grow_margin(mfm_ctx *ctx) {
  if (++ctx->overflow_streak >= 2) ctx->margin_boost = fmin(ctx->margin_boost * 1.1, 2.0);
}
void relax_margin(mfm_ctx *ctx) {
  ctx->overflow_streak = 0;
  ctx->margin_boost = fmax(1.0, ctx->margin_boost * 0.98);
}

// Sort, permutation and tree build (no synchronisation).
int build_cells_async(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm) {
  int rc = setup_tree(ctx, pp->n);
  if (rc) return rc;
  const int ev = stage_begin(ctx, 0);
  HIPCHK(ctx, launch_build_cells(ctx, pp, perm), "cells");
  stage_end(ctx, ev);
  ctx->have_cells = 1;
  ctx->have_density = 0;
  ctx->have_grad = 0;
  ctx->n_cells_built = pp->n;
  return MFM_OK;
}

// The tree over the particles in their present order, without the sort
// (mfm_step's reuse of the last order).
int refresh_cells_async(mfm_ctx *ctx, const mfm_particles *pp) {
  int rc = setup_tree(ctx, pp->n);
  if (rc) return rc;
  const int ev = stage_begin(ctx, 0);
  HIPCHK(ctx, launch_refresh_cells(ctx, pp), "tree");
  stage_end(ctx, ev);
  ctx->have_cells = 1;
  ctx->have_density = 0;
  ctx->have_grad = 0;
  ctx->n_cells_built = pp->n;
  return MFM_OK;
}

// Neighbour search, density pass and its validation (no synchronisation).
int density_async(mfm_ctx *ctx, const mfm_particles *pp) {
  static_assert(C_STEP_SKIP - C_CELL_OVERFLOW == 5, "per-pass counters are contiguous");
  HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_CELL_OVERFLOW, 0, 6 * sizeof(int64_t),
                             ctx->stream), "clear pass counters");
  int ev = stage_begin(ctx, 1);
  // the list blocks follow the last search's list lengths; without them
  // (the first pass, or another particle count) a counting search runs first
  if (!ctx->have_need || ctx->need_n != pp->n)
    HIPCHK(ctx, launch_candidates(ctx, pp, true), "neighbour count");
  HIPCHK(ctx, launch_plan_lists(ctx, pp->n), "plan the lists");
  HIPCHK(ctx, launch_candidates(ctx, pp, false), "neighbour search");
  ctx->have_need = 1;
  ctx->need_n = pp->n;
  stage_end(ctx, ev);
  ev = stage_begin(ctx, 2);
  HIPCHK(ctx, launch_density(ctx, pp), "density");
  stage_end(ctx, ev);
  HIPCHK(ctx, launch_validate(ctx), "validate the density pass");
  return MFM_OK;
}

}  // namespace

extern "C" {

int mfm_build_cells(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm) {
  if (!ctx) return MFM_E_ARG;
  if (!check_parts(ctx, pp)) return fail(ctx, MFM_E_ARG, "invalid particle set");
  ctx->keep_order = 0;
  return build_cells_async(ctx, pp, perm);
}

int mfm_density(mfm_ctx *ctx, const mfm_particles *pp) {
  if (!ctx) return MFM_E_ARG;
  if (!check_parts(ctx, pp)) return fail(ctx, MFM_E_ARG, "invalid particle set");
  if (!ctx->have_cells || ctx->n_cells_built != pp->n)
    return fail(ctx, MFM_E_STATE, "mfm_density needs mfm_build_cells first");
  int64_t c[NCOUNTERS];
  // a chunk whose lists outgrew the blocks planned from the last search
  // leaves the state untouched and its lengths recorded: the second pass is
  // planned from them
  for (int pass = 0; pass < 2; ++pass) {
    int rc = density_async(ctx, pp);
    if (rc) return rc;
    rc = read_counters(ctx, c);
    if (rc) return rc;
    if (c[C_PASS_LIST] == 0) break;
    if (c[C_LIST_POOL])
      return fail(ctx, MFM_E_LIST, "neighbour lists exceed the list pool (raise max_list)");
  }
  if (c[C_PASS_LIST] > 0)
    return fail(ctx, MFM_E_LIST, "neighbour lists outgrew their planned blocks twice");
  if (c[C_CELL_OVERFLOW] > 0) {
    // some H reached cell_margin times its value at the build: this pass is
    // discarded (its counts too) and the next build searches wider.  The
    // density loop has written an estimate of each outgrown root as its
    // start value; a small extra margin guards against underestimates.
    grow_margin(ctx);
    ctx->have_cells = 0;
    ctx->have_need = 0;  // new radii: the next search counts its lists first
    return fail(ctx, MFM_E_CELLS, "smoothing lengths outgrew their search radii; rebuild cells");
  }
  relax_margin(ctx);
  ctx->have_density = 1;
  ctx->have_grad = 0;
  if (c[C_PASS_NOCONV] > 0)
    return fail(ctx, MFM_E_H_NOCONV, "smoothing-length solve did not converge");
  return MFM_OK;
}

int mfm_gradients(mfm_ctx *ctx, const mfm_particles *pp, double dt_max, double *dt_dev) {
  if (!ctx) return MFM_E_ARG;
  if (!check_parts(ctx, pp) || !dt_dev || !(dt_max > 0.0))
    return fail(ctx, MFM_E_ARG, "invalid arguments");
  if (!ctx->have_density || ctx->n_cells_built != pp->n)
    return fail(ctx, MFM_E_STATE, "mfm_gradients needs mfm_density first");
  const int ev = stage_begin(ctx, 3);
  HIPCHK(ctx, launch_gradients(ctx, pp, dt_max, dt_dev), "gradients");
  stage_end(ctx, ev);
  ctx->have_grad = 1;
  return MFM_OK;
}

int mfm_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  if (!ctx) return MFM_E_ARG;
  if (!check_parts(ctx, pp) || !dt_dev) return fail(ctx, MFM_E_ARG, "invalid arguments");
  if (!ctx->have_grad || ctx->n_cells_built != pp->n)
    return fail(ctx, MFM_E_STATE, "mfm_fluxes needs mfm_gradients first");
  if (ctx->p.guess == MFM_GUESS_LEARNED && !ctx->mlp_state)
    return fail(ctx, MFM_E_STATE, "learned guess requested but no network attached");
  HIPCHK(ctx, launch_fluxes(ctx, pp, dt_dev), "fluxes");
  return MFM_OK;
}

int mfm_set_cosmology(mfm_ctx *ctx, double inv_a, double hubble_n, double hubble_np1) {
  if (!ctx) return MFM_E_ARG;
  if (!(inv_a > 0.0) || !isfinite(inv_a) || !isfinite(hubble_n) || !isfinite(hubble_np1))
    return fail(ctx, MFM_E_ARG, "invalid cosmology");
  if ((hubble_n != 0.0 || hubble_np1 != 0.0) && fabs(ctx->p.gamma - 5.0 / 3.0) > 1e-12)
    return fail(ctx, MFM_E_ARG, "the Hubble update of the total energy needs gamma = 5/3");
  ctx->inv_a = inv_a;
  ctx->hubble_n = hubble_n;
  ctx->hubble_np1 = hubble_np1;
  return MFM_OK;
}

int mfm_mlp_attach(mfm_ctx *ctx, const void *state_dev) {
  if (!ctx) return MFM_E_ARG;
  ctx->mlp_state = state_dev;
  return MFM_OK;
}

int mfm_face_dump(mfm_ctx *ctx, float *records_dev, int64_t capacity) {
  if (!ctx) return MFM_E_ARG;
  if (records_dev && capacity <= 0) return fail(ctx, MFM_E_ARG, "dump capacity must be > 0");
  ctx->dump = records_dev;
  ctx->dump_cap = records_dev ? capacity : 0;
  HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_DUMP_COUNT, 0, sizeof(int64_t), ctx->stream),
         "reset dump count");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return MFM_OK;
}

int mfm_face_dump_count(mfm_ctx *ctx, int64_t *count_host) {
  if (!ctx || !count_host) return MFM_E_ARG;
  int64_t c[NCOUNTERS];
  int rc = read_counters(ctx, c);
  if (rc) return rc;
  *count_host = c[C_DUMP_COUNT] < ctx->dump_cap ? c[C_DUMP_COUNT] : ctx->dump_cap;
  return MFM_OK;
}

int mfm_update(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev) {
  if (!ctx) return MFM_E_ARG;
  if (!check_parts(ctx, pp) || !dt_dev) return fail(ctx, MFM_E_ARG, "invalid arguments");
  const int ev = stage_begin(ctx, 5);
  HIPCHK(ctx, launch_update(ctx, pp, dt_dev), "update");
  stage_end(ctx, ev);
  ctx->have_cells = 0;
  ctx->have_density = 0;
  ctx->have_grad = 0;
  return MFM_OK;
}

int mfm_step(mfm_ctx *ctx, const mfm_particles *pp, double dt_max, double *dt_host) {
  if (!ctx) return MFM_E_ARG;
  if (!dt_host) return fail(ctx, MFM_E_ARG, "dt_host is NULL");
  if (!check_parts(ctx, pp) || !(dt_max > 0.0)) return fail(ctx, MFM_E_ARG, "invalid arguments");
  if (ctx->p.guess == MFM_GUESS_LEARNED && !ctx->mlp_state)
    return fail(ctx, MFM_E_STATE, "learned guess requested but no network attached");
  // A density pass whose candidate radii or list blocks turn out too small
  // is rejected on the device; the kernels after it return at once (the
  // state is not updated), and the step is repeated with larger radii or
  // blocks.
  //
  // The particle order: the sort (and the permutation of every array) is
  // skipped while the last step left keep_order set for these arrays: the
  // tree is then built over the particles in the order the last sort gave
  // them.  Events time the cells, search and density stages of every step;
  // a step that keeps the order saves the sort but its search and density
  // loops slow down as the particles drift out of their grouping, so the
  // next step sorts again once that time reaches the one of the step of the
  // last sort, after KEEP_MAX_STEPS steps, or on a repeated attempt.  A
  // sorting step whose search first counted its lists (a first step, grown
  // radii) is no reference: the step after it sorts again.  A context on
  // the static scratch makes no events and always sorts.  The order changes only the grouping of the search,
  // never which pairs interact.
  double *dt_dev = ctx->scalars + 1;
  for (int attempt = 0; attempt < 6; ++attempt) {
    HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_NONFINITE, 0, sizeof(int64_t), ctx->stream),
           "clear step counters");
    const bool kept = attempt == 0 && ctx->keep_order && ctx->order_x == pp->x &&
                      ctx->order_n == pp->n && ctx->have_need && ctx->need_n == pp->n;
    ctx->keep_order = 0;
    if (!ctx->ev_ord_made && !ctx->static_dev) {
      if (hipEventCreate(&ctx->ev_ord[0]) == hipSuccess) {
        if (hipEventCreate(&ctx->ev_ord[1]) == hipSuccess)
          ctx->ev_ord_made = 1;
        else
          hipEventDestroy(ctx->ev_ord[0]);
      }
    }
    const bool counted = !ctx->have_need || ctx->need_n != pp->n;  // a counting search
    if (ctx->ev_ord_made) HIPCHK(ctx, hipEventRecord(ctx->ev_ord[0], ctx->stream), "event");
    int rc = kept ? refresh_cells_async(ctx, pp) : build_cells_async(ctx, pp, nullptr);
    if (rc) return rc;
    rc = density_async(ctx, pp);
    if (rc) return rc;
    if (ctx->ev_ord_made) HIPCHK(ctx, hipEventRecord(ctx->ev_ord[1], ctx->stream), "event");
    ctx->have_density = 1;
    rc = mfm_gradients(ctx, pp, dt_max, dt_dev);
    if (rc) return rc;
    rc = mfm_fluxes(ctx, pp, dt_dev);
    if (rc) return rc;
    rc = mfm_update(ctx, pp, dt_dev);
    if (rc) return rc;
    // the step's one synchronisation: counters and dt together
    int64_t c[NCOUNTERS];
    double sc[2];
    HIPCHK(ctx, hipMemcpyAsync(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost, ctx->stream),
           "read counters");
    HIPCHK(ctx, hipMemcpyAsync(sc, ctx->scalars, sizeof(sc), hipMemcpyDeviceToHost, ctx->stream),
           "read dt");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    if (c[C_STEP_SKIP]) {
      // lists longer than their planned blocks: the next attempt plans from
      // the lengths this one recorded (the same order, the same lists)
      // (on a kept order the next attempt sorts first, which may fit the pool)
      if (c[C_PASS_LIST] > 0 && c[C_LIST_POOL] && !kept)
        return fail(ctx, MFM_E_LIST, "neighbour lists exceed the list pool (raise max_list)");
      if (c[C_CELL_OVERFLOW] > 0) {
        // new start values (and radii): the next search counts its lists
        // first
        grow_margin(ctx);
        ctx->have_need = 0;
      }
      continue;
    }
    relax_margin(ctx);
    *dt_host = sc[1];
    // the order for the next step
    float ms = 0.0f;
    if (ctx->ev_ord_made &&
        hipEventElapsedTime(&ms, ctx->ev_ord[0], ctx->ev_ord[1]) == hipSuccess) {
      if (!kept) {
        ctx->ms_sorted = ms;
        ctx->steps_kept = 0;
      } else {
        ++ctx->steps_kept;
      }
      ctx->keep_order = !counted && ms <= ctx->ms_sorted && ctx->steps_kept + 1 < KEEP_MAX_STEPS;
    }
    ctx->order_x = pp->x;
    ctx->order_n = pp->n;
    if (c[C_NONFINITE] > 0) return fail(ctx, MFM_E_NONFINITE, "non-finite step or state");
    if (c[C_PASS_NOCONV] > 0)
      return fail(ctx, MFM_E_H_NOCONV, "smoothing-length solve did not converge");
    return MFM_OK;
  }
  return fail(ctx, MFM_E_CELLS, "smoothing lengths kept outgrowing their search radii");
}

}  // extern "C"

namespace {

// The device scalars the sub-step loop reads back: the counters and rmax.
int read_step_counters(mfm_ctx *ctx, int64_t *c) {
  HIPCHK(ctx, hipMemcpyAsync(c, ctx->counters, sizeof(int64_t) * NCOUNTERS,
                             hipMemcpyDeviceToHost, ctx->stream),
         "read counters");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return MFM_OK;
}

// The counters at the end of sub-step k of individual steps.  With the
// pinned copy, the start of sub-step k + 1 (when there is one) is enqueued
// before the host waits, so that the GPU runs it while the host takes the
// counters and enqueues the rest of that sub-step; *next_begun says so.  A
// rejected sub-step k is started again from its own start, which overwrites
// what that early start wrote.
int read_substep_counters(mfm_ctx *ctx, const mfm_particles *pp, int64_t *c, int64_t k,
                          int64_t nsub, bool *next_begun) {
  *next_begun = false;
  if (!ctx->host_ctr) return read_step_counters(ctx, c);
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_ctr, ctx->counters, sizeof(int64_t) * NCOUNTERS,
                             hipMemcpyDeviceToHost, ctx->stream),
         "read counters");
  HIPCHK(ctx, hipEventRecord(ctx->ev_ctr, ctx->stream), "record the counters' event");
  if (k + 1 < nsub) {
    ctx->rungs.k = k + 1;
    const hipError_t e = launch_substep_begin(ctx, pp);
    ctx->rungs.k = k;
    HIPCHK(ctx, e, "next sub-step start");
    *next_begun = true;
  }
  HIPCHK(ctx, hipEventSynchronize(ctx->ev_ctr), "synchronise");
  memcpy(c, ctx->host_ctr, sizeof(int64_t) * NCOUNTERS);
  return MFM_OK;
}

// After a rejected density pass: which retry, or the error.
int on_skip(mfm_ctx *ctx, const int64_t *c) {
  if (c[C_PASS_LIST] > 0 && c[C_LIST_POOL])
    return fail(ctx, MFM_E_LIST, "neighbour lists exceed the list pool (raise max_list)");
  if (c[C_CELL_OVERFLOW] > 0) {
    grow_margin(ctx);
    ctx->have_need = 0;
  }
  return MFM_OK;
}

// Leave the individual-step mode whatever happened.
struct RungsOff {
  mfm_ctx *ctx;
  ~RungsOff() {
    memset(&ctx->rungs, 0, sizeof(ctx->rungs));
    ctx->rung_perm = nullptr;
    ctx->have_cells = ctx->have_density = ctx->have_grad = 0;
  }
};

}  // namespace

extern "C" {

int mfm_step_rungs(mfm_ctx *ctx, const mfm_particles *pp, double dt0, int32_t *rung_io,
                   int rungs_given, int64_t *nsub_out) {
  if (!ctx) return MFM_E_ARG;
  if (nsub_out) *nsub_out = 0;
  if (!check_parts(ctx, pp) || !(dt0 > 0.0) || !isfinite(dt0) || (rungs_given && !rung_io))
    return fail(ctx, MFM_E_ARG, "invalid arguments");
  if (pp->accel || ctx->inv_a != 1.0 || ctx->hubble_n != 0.0 || ctx->hubble_np1 != 0.0 ||
      ctx->p.entropy_switch)
    return fail(ctx, MFM_E_ARG, "individual steps take no source terms and no entropy switch");
  if (ctx->p.guess == MFM_GUESS_LEARNED && !ctx->mlp_state)
    return fail(ctx, MFM_E_STATE, "learned guess requested but no network attached");
  RungsOff off{ctx};
  ctx->keep_order = 0;  // the base step sorts; the next mfm_step sorts again
  memset(&ctx->rungs, 0, sizeof(ctx->rungs));
  ctx->rung_perm = rungs_given ? rung_io : nullptr;
  const int64_t n = pp->n;
  double *dt_dev = ctx->scalars + 1;
  int32_t *rmax_dev = reinterpret_cast<int32_t *>(ctx->scalars + 8);
  int64_t c[NCOUNTERS];
  // the base step starts with every particle synchronised: the order, the
  // density and gradient loops of all of them (as mfm_step's first stages)
  bool ok = false;
  for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
    HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_NONFINITE, 0, sizeof(int64_t), ctx->stream),
           "clear step counters");
    int rc = build_cells_async(ctx, pp, nullptr);
    if (!rc) rc = density_async(ctx, pp);
    if (rc) return rc;
    int ev = stage_begin(ctx, 3);
    HIPCHK(ctx, launch_gradients(ctx, pp, dt0, dt_dev), "gradients");
    stage_end(ctx, ev);
    rc = read_step_counters(ctx, c);
    if (rc) return rc;
    if (c[C_STEP_SKIP]) {
      rc = on_skip(ctx, c);
      if (rc) return rc;
      continue;
    }
    ok = true;
  }
  if (!ok) return fail(ctx, MFM_E_CELLS, "smoothing lengths kept outgrowing their search radii");
  relax_margin(ctx);
  // rungs: from the CFL steps, with the limiter swept to its fixed point
  // over the faces of the pass above (every particle active), or given
  int32_t *rung = rungs_given ? rung_io : ctx->rung_w;
  ctx->rungs.rung = rung;
  HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_RUNG_CHANGED, 0, 2 * sizeof(int64_t), ctx->stream),
         "clear rung counters");
  if (!rungs_given) {
    HIPCHK(ctx, launch_rungs_from_dt(ctx, pp, dt0), "rungs");
    for (int sweep = 0;; ++sweep) {
      HIPCHK(ctx, hipMemsetAsync(ctx->counters + C_RUNG_CHANGED, 0, sizeof(int64_t), ctx->stream),
             "clear the limiter flag");
      HIPCHK(ctx, launch_rung_limiter(ctx, pp), "rung limiter");
      int rc = read_step_counters(ctx, c);
      if (rc) return rc;
      if (c[C_RUNG_CHANGED] == 0) break;
      if (sweep > 4 * MFM_RUNG_MAX) return fail(ctx, MFM_E_HIP, "rung limiter did not settle");
    }
    if (c[C_RUNG_DEEP] > 0)
      return fail(ctx, MFM_E_NONFINITE, "a step needs a rung beyond MFM_RUNG_MAX");
  } else {
    HIPCHK(ctx, launch_rung_check(ctx, n), "check the rungs");
    int rc = read_step_counters(ctx, c);
    if (rc) return rc;
    if (c[C_RUNG_DEEP] > 0) return fail(ctx, MFM_E_ARG, "a given rung is out of range");
  }
  HIPCHK(ctx, launch_rmax(ctx, n, rmax_dev), "deepest rung");
  int32_t rmax = 0;
  HIPCHK(ctx, hipMemcpyAsync(&rmax, rmax_dev, sizeof(rmax), hipMemcpyDeviceToHost, ctx->stream),
         "read the deepest rung");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (rmax < 0 || rmax > MFM_RUNG_MAX) return fail(ctx, MFM_E_ARG, "rung out of range");
  const int64_t nsub = (int64_t)1 << rmax;
  ctx->rungs.s0 = ctx->s0_w;
  ctx->rungs.act = ctx->act_w;
  ctx->rungs.elapsed = ctx->elapsed_w;
  ctx->rungs.dt0 = dt0;
  ctx->rungs.rmax = rmax;
  HIPCHK(ctx, hipMemsetAsync(ctx->s0_w, 0, sizeof(int32_t) * n, ctx->stream), "clear step starts");
  HIPCHK(ctx, hipMemsetAsync(pp->dQ, 0, sizeof(double) * 5 * n, ctx->stream), "clear flux sums");
  if (!ctx->host_ctr && !ctx->static_dev) {
    // the pinned counter copy of the sub-step loop (kept until mfm_destroy)
    if (hipHostMalloc((void **)&ctx->host_ctr, sizeof(int64_t) * NCOUNTERS) != hipSuccess) {
      ctx->host_ctr = nullptr;
    } else if (hipEventCreateWithFlags(&ctx->ev_ctr, hipEventDisableTiming) != hipSuccess) {
      hipHostFree(ctx->host_ctr);
      ctx->host_ctr = nullptr;
    }
  }
  bool begun = false;  // this sub-step's start was enqueued by the one before
  for (int64_t k = 0; k < nsub; ++k) {
    ctx->rungs.k = k;
    ok = false;
    for (int attempt = 0; attempt < 6 && !ok; ++attempt) {
      if (!begun) HIPCHK(ctx, launch_substep_begin(ctx, pp), "sub-step start");
      begun = false;
      if (k > 0) {
        // the particles whose step begins: tree at this sub-step's positions,
        // search, density and gradient loops
        int rc = setup_tree(ctx, n);
        if (rc) return rc;
        int ev = stage_begin(ctx, 0);
        HIPCHK(ctx, launch_tree(ctx, n), "tree");
        stage_end(ctx, ev);
        rc = density_async(ctx, pp);
        if (rc) return rc;
        ev = stage_begin(ctx, 3);
        HIPCHK(ctx, launch_gradients(ctx, pp, dt0, dt_dev), "gradients");
        stage_end(ctx, ev);
      }
      HIPCHK(ctx, launch_fluxes(ctx, pp, dt_dev), "fluxes");
      int ev = stage_begin(ctx, 5);
      HIPCHK(ctx, launch_update(ctx, pp, dt_dev), "close");
      stage_end(ctx, ev);
      int rc = read_substep_counters(ctx, pp, c, k, nsub, &begun);
      if (rc) return rc;
      if (k > 0 && c[C_STEP_SKIP]) {
        begun = false;  // sub-step k starts again from its own start
        rc = on_skip(ctx, c);
        if (rc) return rc;
        continue;
      }
      ok = true;
    }
    if (!ok) return fail(ctx, MFM_E_CELLS, "smoothing lengths kept outgrowing their search radii");
    if (k > 0) relax_margin(ctx);
    if (c[C_NONFINITE] > 0) return fail(ctx, MFM_E_NONFINITE, "non-finite step or state");
    if (c[C_PASS_NOCONV] > 0)
      return fail(ctx, MFM_E_H_NOCONV, "smoothing-length solve did not converge");
  }
  if (!rungs_given && rung_io)
    HIPCHK(ctx, hipMemcpyAsync(rung_io, ctx->rung_w, sizeof(int32_t) * n,
                               hipMemcpyDeviceToDevice, ctx->stream),
           "copy the rungs out");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (nsub_out) *nsub_out = nsub;
  return MFM_OK;
}

int mfm_diagnostics(mfm_ctx *ctx, const mfm_particles *pp, mfm_diag *out) {
  if (!ctx || !out) return MFM_E_ARG;
  memset(out, 0, sizeof(*out));
  if (pp) {
    if (!check_parts(ctx, pp)) return fail(ctx, MFM_E_ARG, "invalid particle set");
    HIPCHK(ctx, launch_conserved(ctx, pp), "conserved sums");
  }
  double sums[5] = {0, 0, 0, 0, 0};
  HIPCHK(ctx, hipMemcpyAsync(sums, ctx->scalars + 2, sizeof(sums), hipMemcpyDeviceToHost,
                             ctx->stream),
         "read sums");
  int64_t c[NCOUNTERS];
  int rc = read_counters(ctx, c);
  if (rc) return rc;
  int64_t *dst = &out->h_noconv;
  for (int k = 0; k <= C_HARD_OVERFLOW; ++k) dst[k] = c[k];
  if (pp) {
    out->mass = sums[0];
    out->px = sums[1];
    out->py = sums[2];
    out->pz = sums[3];
    out->energy = sums[4];
  }
  return MFM_OK;
}

int mfm_reset_counters(mfm_ctx *ctx) {
  if (!ctx) return MFM_E_ARG;
  HIPCHK(ctx, hipMemsetAsync(ctx->counters, 0, sizeof(int64_t) * NCOUNTERS, ctx->stream),
         "reset counters");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return MFM_OK;
}

int mfm_enable_timing(mfm_ctx *ctx, int on) {
  if (!ctx) return MFM_E_ARG;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (on && !ctx->ev_created) {
    // the events are made on first use, so that a context that is never
    // timed creates none
    for (int k = 0; k < 2 * MAX_EVENT_PAIRS; ++k) {
      hipError_t e = hipEventCreate(&ctx->ev_pool[k]);
      if (e != hipSuccess) {
        for (int q = 0; q < k; ++q) hipEventDestroy(ctx->ev_pool[q]);
        return hip_fail(ctx, e, "create timing events");
      }
    }
    ctx->ev_created = 1;
  }
  harvest_events(ctx);
  ctx->timing = on ? 1 : 0;
  for (int s = 0; s < MFM_NSTAGES; ++s) {
    ctx->stage_ms[s] = 0.0;
    ctx->stage_count[s] = 0;
  }
  return MFM_OK;
}

int mfm_kernel_times(mfm_ctx *ctx, double *ms_out, int64_t *count_out) {
  if (!ctx || !ms_out) return MFM_E_ARG;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  harvest_events(ctx);
  for (int s = 0; s < MFM_NSTAGES; ++s) {
    ms_out[s] = ctx->stage_ms[s];
    if (count_out) count_out[s] = ctx->stage_count[s];
  }
  return MFM_OK;
}

const char *mfm_strerror(int status) {
  switch (status) {
    case MFM_OK: return "ok";
    case MFM_E_ARG: return "invalid argument";
    case MFM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case MFM_E_HIP: return "HIP runtime error";
    case MFM_E_H_NOCONV: return "smoothing-length solve did not converge";
    case MFM_E_CELLS: return "smoothing lengths outgrew their search radii";
    case MFM_E_LIST: return "neighbour list capacity exceeded";
    case MFM_E_NONFINITE: return "non-finite time step or state";
    case MFM_E_STATE: return "call order violated";
    default: return "unknown status";
  }
}

const char *mfm_last_error(mfm_ctx *ctx) { return ctx ? ctx->err : "no context"; }

}  // extern "C"
