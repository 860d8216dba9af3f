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
  C_CELL_OVERFLOW,  // internal: some H reached the cell side in the last density pass
  C_NONFINITE,      // internal: non-finite dt or state
  // counts of the density pass in flight; folded into the slots above only
  // when the pass is accepted (a pass whose H outgrew the cells is redone)
  C_PASS_NOCONV,
  C_PASS_BOOSTS,
  C_PASS_FAIL,
  NCOUNTERS = 24
};

// Packed per-particle record read by the flux pass (one 256-byte line pair).
enum {
  R_X = 0, R_Y, R_Z, R_H, R_V, R_RHO, R_VX, R_VY, R_VZ, R_P,
  R_B = 10,     // 6 entries of B = E^-1
  R_G = 16,     // 15 entries of the limited gradients (rho, vx, vy, vz, P) x (x, y, z)
  R_STRIDE = 32
};

// Geometry of the cell grid, passed by value to kernels.
struct CellGrid {
  int nc[3];          // cells per axis (>= 3)
  double inv[3];      // nc / box per axis
  double box[3];      // periodic sides
  double half[3];     // box / 2
  double side_min;    // smallest cell side: every pair closer than this is in the 27-cell stencil
  const int32_t *start;  // indexed by Morton code
  const int32_t *count;  // indexed by Morton code
};

struct mfm_ctx {
  mfm_params p;
  int64_t n_max;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  // workspace carve
  uint32_t *code;      // n: Morton code of each particle's cell
  int32_t *cell_count; // ncodes_max
  int32_t *cell_start; // ncodes_max
  int32_t *cursor;     // ncodes_max
  int32_t *scan_tmp;   // block sums of the scans
  int32_t *order;      // n: input slot of each sorted slot
  double *tmp;         // 11 n doubles: gather buffer of the permutation
  int32_t *list;       // max_list * n, entry k of particle i at [k * n + i]
  int32_t *list_cnt;   // n
  double *rec;         // R_STRIDE * n packed flux records
  double *red;         // reduction partials
  int64_t *counters;   // NCOUNTERS
  double *scalars;     // small device scalars: [0] max H, [1] dt, [2..6] conserved sums
  int64_t ncodes_max;
  size_t scan_tmp_len, red_len;
  // current grid
  CellGrid grid;
  int64_t ncodes;
  int bits;
  double margin_boost;
  int have_cells, have_density, have_grad;
  int64_t n_cells_built;  // n of the particles the cells were built for
  // timing
  int timing;
  hipEvent_t ev_pool[2 * 1024];
  int ev_stage[1024];
  int ev_used;
  double stage_ms[MFM_NSTAGES];
  int64_t stage_count[MFM_NSTAGES];
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
__device__ __forceinline__ int cell_coord(double x, double inv, int nc) {
  int c = (int)(x * inv);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
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
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
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
hipError_t launch_max_h(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_build_cells(mfm_ctx *ctx, const mfm_particles *pp, int64_t *perm);
hipError_t launch_density(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_build_lists(mfm_ctx *ctx, const mfm_particles *pp);
hipError_t launch_gradients(mfm_ctx *ctx, const mfm_particles *pp, double dt_max, double *dt_dev);
hipError_t launch_fluxes(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev);
hipError_t launch_update(mfm_ctx *ctx, const mfm_particles *pp, const double *dt_dev);
hipError_t launch_conserved(mfm_ctx *ctx, const mfm_particles *pp);

// timing helpers (api translation unit)
void stage_begin(mfm_ctx *ctx, int stage);
void stage_end(mfm_ctx *ctx, int stage);

static inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }
