// lanes.h -- reductions across the lanes of a wavefront through DPP row
// operations, which move registers inside the 16-lane rows without the LDS
// traffic of ds_bpermute: two quad permutations and the two row mirrors
// leave the row's result in each of its 16 lanes; a wavefront result then
// combines one lane of each of the four rows (readlane, wave-uniform).
// min and max are exact in any order; a row sum is taken in this fixed order.
#pragma once
#include <hip/hip_runtime.h>

namespace lanes {

// DPP_CTRL values of the CDNA instruction set
constexpr int QUAD_XOR1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int QUAD_XOR2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int ROW_HALF_MIRROR = 0x141;  // lane l of each 8 reads lane 7 - l
constexpr int ROW_MIRROR = 0x140;       // lane l of each 16 reads lane 15 - l

// every lane reads a lane of its own row: the masks enable all rows and banks
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 w = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = dpp_i32<CTRL>(w.x);
  r.y = dpp_i32<CTRL>(w.y);
  return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ double read_f64(double v, int l) {
  const int2 w = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(w.x, l);
  r.y = __builtin_amdgcn_readlane(w.y, l);
  return __builtin_bit_cast(double, r);
}

template <typename F>
__device__ __forceinline__ double row_f64(double v, F op) {
  v = op(v, dpp_f64<QUAD_XOR1>(v));
  v = op(v, dpp_f64<QUAD_XOR2>(v));
  v = op(v, dpp_f64<ROW_HALF_MIRROR>(v));
  return op(v, dpp_f64<ROW_MIRROR>(v));
}

__device__ __forceinline__ double row_min_f64(double v) {
  return row_f64(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double row_max_f64(double v) {
  return row_f64(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double row_sum_f64(double v) {
  return row_f64(v, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double wave_min_f64(double v) {
  v = row_min_f64(v);
  return fmin(fmin(read_f64(v, 0), read_f64(v, 16)), fmin(read_f64(v, 32), read_f64(v, 48)));
}
__device__ __forceinline__ double wave_max_f64(double v) {
  v = row_max_f64(v);
  return fmax(fmax(read_f64(v, 0), read_f64(v, 16)), fmax(read_f64(v, 32), read_f64(v, 48)));
}

__device__ __forceinline__ int wave_max_i32(int v) {
  v = max(v, dpp_i32<QUAD_XOR1>(v));
  v = max(v, dpp_i32<QUAD_XOR2>(v));
  v = max(v, dpp_i32<ROW_HALF_MIRROR>(v));
  v = max(v, dpp_i32<ROW_MIRROR>(v));
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, dpp_i32<QUAD_XOR1>(v));
  v = min(v, dpp_i32<QUAD_XOR2>(v));
  v = min(v, dpp_i32<ROW_HALF_MIRROR>(v));
  v = min(v, dpp_i32<ROW_MIRROR>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

}  // namespace lanes
