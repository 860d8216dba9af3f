// mlp_device.h -- the Riemann-guess network on matrix cores: a 6 -> 64 -> 64
// -> 64 -> 1 perceptron with SiLU activations, BF16 operands and FP32
// accumulation on v_mfma_f32_16x16x16_bf16.  A wavefront evaluates 16 * MT
// rows (faces) at a time; activations live in LDS between layers, the BF16
// weights (18 KB, transposed so each lane's operand is one 8-byte load) are
// read through L1.
//
// Operand layout of the 16x16x16 BF16 MFMA (lane l, element e = 0..3):
//   A (16 x 16, M x K): row l % 16, column 4 (l / 16) + e
//   B (16 x 16, K x N): row 4 (l / 16) + e, column l % 16
//   D (16 x 16, M x N): row 4 (l / 16) + e, column l % 16
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlp {

constexpr int NIN = 6;    // features
constexpr int K1 = 16;    // first-layer input width padded to one MFMA K step
constexpr int HID = 64;   // hidden width
// FP32 parameter vector: W1 [K1][HID] (rows >= NIN stay zero), b1, W2 [HID][HID],
// b2, W3 [HID][HID], b3, w4 [HID], b4.
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + K1 * HID;
constexpr int OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID;
constexpr int OFF_B3 = OFF_W3 + HID * HID;
constexpr int OFF_W4 = OFF_B3 + HID;
constexpr int OFF_B4 = OFF_W4 + HID;
constexpr int NPARAM = OFF_B4 + 1;
constexpr int NPARAM_PAD = (NPARAM + 63) / 64 * 64;
// transposed BF16 weights: W1^T [HID][K1], W2^T [HID][HID], W3^T [HID][HID]
constexpr int T_W1 = 0;
constexpr int T_W2 = T_W1 + HID * K1;
constexpr int T_W3 = T_W2 + HID * HID;
constexpr int NT = T_W3 + HID * HID;
// normalisation: mean[6], std[6], y mean, y std
constexpr int NNORM = 16;

constexpr int AST = HID + 8;  // LDS activation row stride (BF16 elements)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__host__ __device__ inline uint16_t to_bf16(float f) {
  union {
    float f;
    uint32_t u;
  } v;
  v.f = f;
  uint32_t u = v.u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t h) {
  union {
    float f;
    uint32_t u;
  } v;
  v.u = ((uint32_t)h) << 16;
  return v.f;
}

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Where the network's weights live (device memory).
struct Net {
  const uint16_t *wt;   // transposed BF16 weights (T_* offsets)
  const uint16_t *wr;   // row-major BF16 copy of the parameter vector
  const float *p;       // FP32 parameters (biases, w4, b4 are read from here)
  const float *norm;
};

__device__ inline bf16x4 ld4(const uint16_t *q) {
  const uint2 v = *reinterpret_cast<const uint2 *>(q);  // 8-byte aligned
  bf16x4 r;
  r[0] = (short)(v.x & 0xffffu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xffffu);
  r[3] = (short)(v.y >> 16);
  return r;
}

// A dense layer for the wave's 16 * MT rows: out[:, :HID] = silu(in[:, :K] W + b).
// in and out may be the same buffer (each row block is read before it is
// written).  If z is given, the pre-activations are kept there (row stride zst).
template <int MT, int K>
__device__ inline void layer(const uint16_t *in, int ist, uint16_t *out, int ost,
                             const uint16_t *wt, const float *bias, float *z, int zst,
                             int lane) {
  const int r16 = lane & 15, q4 = (lane >> 4) * 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < K / 16; ++kt) {
      const bf16x4 a = ld4(in + (16 * mt + r16) * ist + 16 * kt + q4);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const bf16x4 b = ld4(wt + (16 * nt + r16) * K + 16 * kt + q4);
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = 16 * nt + r16;
      const float bn = bias[n];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = 16 * mt + q4 + e;
        const float zz = acc[nt][e] + bn;
        if (z) z[m * zst + n] = zz;
        out[m * ost + n] = to_bf16(silu(zz));
      }
    }
  }
}

// Orders this wave's LDS writes before its later LDS reads of other lanes' data.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Standardised BF16 features of row `row` (zeros when x is null).
__device__ inline void put_input(uint16_t *act, int row, const float *x, const float *norm) {
#pragma unroll
  for (int k = 0; k < NIN; ++k)
    act[row * AST + k] = x ? to_bf16((x[k] - norm[k]) / norm[NIN + k]) : (uint16_t)0;
#pragma unroll
  for (int k = NIN; k < K1; ++k) act[row * AST + k] = 0;
}

// The FP32 vectors a forward pass reads besides the BF16 weight matrices:
// the three hidden biases, the output weights and bias, the normalisation.
struct Vecs {
  const float *b1, *b2, *b3, *w4, *b4, *norm;
};
__device__ inline Vecs vecs_of(const Net &net) {
  return Vecs{net.p + OFF_B1, net.p + OFF_B2, net.p + OFF_B3, net.p + OFF_W4, net.p + OFF_B4,
              net.norm};
}
constexpr int NVEC = 4 * HID + 1 + NNORM;  // floats of an LDS copy of the vectors

// Copies a network's BF16 weights (w, NT elements, 16-byte aligned) and FP32
// vectors (v, NVEC floats) into LDS; every thread of the workgroup takes
// part (tid of nth), and a workgroup barrier must follow before they are
// read.  Returns the vectors' LDS addresses.
__device__ inline Vecs stage_net(const Net &net, uint16_t *w, float *v, int tid, int nth) {
  const uint4 *src = reinterpret_cast<const uint4 *>(net.wt);
  uint4 *dst = reinterpret_cast<uint4 *>(w);
  for (int k = tid; k < NT / 8; k += nth) dst[k] = src[k];
  const Vecs g = vecs_of(net);
  for (int k = tid; k < NVEC; k += nth) {
    float x;
    if (k < 4 * HID) {
      const int q = k / HID, e = k % HID;
      x = (q == 0 ? g.b1 : q == 1 ? g.b2 : q == 2 ? g.b3 : g.w4)[e];
    } else if (k == 4 * HID) {
      x = g.b4[0];
    } else {
      x = g.norm[k - 4 * HID - 1];
    }
    v[k] = x;
  }
  return Vecs{v, v + HID, v + 2 * HID, v + 3 * HID, v + 4 * HID, v + 4 * HID + 1};
}

// Forward pass of one 16-row tile held in act (row stride AST), in place,
// with the weights wt and vectors v.  Every lane returns the unstandardised
// output of row lane % 16.
__device__ inline float forward_rows(uint16_t *act, const uint16_t *wt, const Vecs &v, int lane) {
  wave_lds_sync();
  layer<1, K1>(act, AST, act, AST, wt + T_W1, v.b1, nullptr, 0, lane);
  wave_lds_sync();
  layer<1, HID>(act, AST, act, AST, wt + T_W2, v.b2, nullptr, 0, lane);
  wave_lds_sync();
  layer<1, HID>(act, AST, act, AST, wt + T_W3, v.b3, nullptr, 0, lane);
  wave_lds_sync();
  // output layer in FP32: lanes l, l+16, l+32, l+48 each sum 16 of the 64 terms
  const int r = lane & 15, k0 = (lane >> 4) * 16;
  float y = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) y += from_bf16(act[r * AST + k0 + k]) * v.w4[k0 + k];
  y += __shfl_xor(y, 16, 64);
  y += __shfl_xor(y, 32, 64);
  y += v.b4[0];
  wave_lds_sync();  // the tile is free for the wave's next rows
  return v.norm[2 * NIN] + v.norm[2 * NIN + 1] * y;
}

// Forward pass of one 16-row tile with the network's own (global) weights.
__device__ inline float forward_tile(uint16_t *act, const Net &net, int lane) {
  return forward_rows(act, net.wt, vecs_of(net), lane);
}

// Forward pass for the 64 rows of a wave, one tile at a time through a
// 16-row buffer; lane l supplies row l (x null: a zero row) and gets its output.
__device__ inline float forward_wave(uint16_t *tile, const float *x, const uint16_t *wt,
                                     const Vecs &v, int lane) {
  float y = 0.f;
  for (int mt = 0; mt < 4; ++mt) {
    if ((lane >> 4) == mt) put_input(tile, lane & 15, x, v.norm);
    const float yt = forward_rows(tile, wt, v, lane);
    if ((lane >> 4) == mt) y = yt;
  }
  return y;
}
__device__ inline float forward_wave(uint16_t *tile, const float *x, const Net &net, int lane) {
  return forward_wave(tile, x, net.wt, vecs_of(net), lane);
}

// Faces whose plain starting value is least accurate -- a pressure ratio
// above 2 (where the plain guess leaves the primitive-variable estimate) or a
// normal velocity jump above half the mean sound speed.  Only these faces
// are given to the network.
constexpr float GATE_LOG_P = 0.69314718f;   // ln 2
constexpr float GATE_DU = 0.40546511f;      // slog(0.5) = ln 1.5
__device__ __host__ inline bool needs_guess(const float x[NIN]) {
  return fabsf(x[1]) > GATE_LOG_P || fabsf(x[2]) > GATE_DU;
}

// Which estimate the plain starting value p0 is (Toro's adaptive choice).
enum GuessBranch { GUESS_PV = 0, GUESS_TR = 1, GUESS_TS = 2 };

// Learned-guess features of a face's Riemann problem: the density and
// pressure ratios, the normal velocity jump over the mean sound speed, and
// the plain starting value p0 with the estimate it came from.  p* depends on
// the states only through the first three (and gamma); p0 and its branch tell
// the network where the error it predicts, ln(p*/p0), jumps.
__device__ inline void face_features(float rL, float pL, float rR, float pR, float du, float cL,
                                     float cR, float p0, int branch, float x[NIN]) {
  const float v = du / (0.5f * (cL + cR));
  x[0] = logf(rL / rR);
  x[1] = logf(pL / pR);
  x[2] = copysignf(log1pf(fabsf(v)), v);
  x[3] = logf(p0 / (0.5f * (pL + pR)));
  x[4] = branch == GUESS_TR ? 1.0f : 0.0f;
  x[5] = branch == GUESS_TS ? 1.0f : 0.0f;
}

}  // namespace mlp
