// mlp.hip -- training and inference of the Riemann-guess network (see
// mlp_device.h): forward and backward passes on BF16 MFMA with FP32
// accumulation, Adam on an FP32 master copy, prediction.
//
// The network predicts y = ln(p* / p0) of a face's Riemann problem, the error
// of the plain starting value p0 (Toro's adaptive choice), from six
// dimensionless features of its left and right states; the flux loop starts
// the exact Newton iteration (which always finishes the solve) from p0 e^y.  Training rows are the face records the flux loop dumps
// (mfm_face_dump): 8 floats per face, the raw features, the target and the
// plain guess's iteration count.
#include "mfm_internal.h"
#include "mlp_device.h"

using namespace mlp;

namespace {

constexpr int TR = 32;        // training rows per workgroup (two 16-row MFMA tiles)
constexpr int TMT = TR / 16;
constexpr int ZST = HID + 4;  // FP32 pre-activation row stride

struct State {
  float *params, *m, *v, *grad, *norm, *loss;
  uint16_t *wbf;   // row-major BF16 copy of params
  uint16_t *wbt;   // transposed BF16 weights
};

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

State carve(void *base) {
  char *p = (char *)base;
  State s;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *q = p + off;
    off += up256(bytes);
    return q;
  };
  s.params = (float *)take(4 * NPARAM_PAD);
  s.m = (float *)take(4 * NPARAM_PAD);
  s.v = (float *)take(4 * NPARAM_PAD);
  s.grad = (float *)take(4 * NPARAM_PAD);
  s.norm = (float *)take(4 * NNORM);
  s.loss = (float *)take(4 * 16);
  s.wbf = (uint16_t *)take(2 * NPARAM_PAD);
  s.wbt = (uint16_t *)take(2 * NT);
  return s;
}

size_t state_bytes() {
  return up256(4 * NPARAM_PAD) * 4 + up256(4 * NNORM) + up256(4 * 16) + up256(2 * NPARAM_PAD) +
         up256(2 * NT);
}

__host__ __device__ inline Net net_of(const State &s) {
  Net n;
  n.wt = s.wbt;
  n.wr = s.wbf;
  n.p = s.params;
  n.norm = s.norm;
  return n;
}

// Weight gradient dW[k][n] += sum_m A[m][k] dZ[m][n] over the TR rows, k < 16 KT,
// added to the global FP32 gradient g (row stride HID).
template <int KT>
__device__ inline void weight_grad(const uint16_t *A, const uint16_t *dZ, float *g, int lane) {
  const int r16 = lane & 15, q4 = (lane >> 4) * 4;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int mt = 0; mt < TMT; ++mt) {
        bf16x4 a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[e] = (short)A[(16 * mt + q4 + e) * AST + 16 * kt + r16];
          b[e] = (short)dZ[(16 * mt + q4 + e) * AST + 16 * nt + r16];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) atomicAdd(g + (16 * kt + q4 + e) * HID + 16 * nt + r16, acc[e]);
    }
  }
}

// dZprev[m][k] = (sum_n dZ[m][n] W[k][n]) silu'(Zprev[m][k]); W row-major in global memory.
__device__ inline void back_layer(const uint16_t *dZ, const uint16_t *w, const float *zprev,
                                  uint16_t *dzprev, int lane) {
  const int r16 = lane & 15, q4 = (lane >> 4) * 4;
#pragma unroll
  for (int mt = 0; mt < TMT; ++mt) {
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const bf16x4 a = ld4(dZ + (16 * mt + r16) * AST + 16 * nt + q4);
        const bf16x4 b = ld4(w + (16 * kt + r16) * HID + 16 * nt + q4);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
      const int k = 16 * kt + r16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = 16 * mt + q4 + e;
        dzprev[m * AST + k] = to_bf16(acc[e] * dsilu(zprev[m * ZST + k]));
      }
    }
  }
}

// Column sums of a [TR][HID] BF16 buffer added to the global gradient.
__device__ inline void bias_grad(const uint16_t *dZ, float *g, int lane) {
  float s = 0.f;
  for (int m = 0; m < TR; ++m) s += from_bf16(dZ[m * AST + lane]);
  atomicAdd(g + lane, s);
}

struct TrainSmem {
  uint16_t x[TR * AST];
  uint16_t a1[TR * AST], a2[TR * AST], a3[TR * AST];
  uint16_t dza[TR * AST], dzb[TR * AST];
  float z1[TR * ZST], z2[TR * ZST], z3[TR * ZST];
  float dy[TR];
};

// One wavefront per workgroup and TR rows each: forward, loss, backward; the
// gradients of the mean squared error over the n rows are added to s.grad.
__global__ void __launch_bounds__(64) mlp_backward_k(State s, const float *rows, int64_t n,
                                                     int64_t stride) {
  __shared__ TrainSmem S;
  const int lane = threadIdx.x;
  const Net net = net_of(s);
  const int64_t row = (int64_t)blockIdx.x * TR + lane;
  const bool valid = lane < TR && row < n;
  float t = 0.f;
  if (lane < TR) {
    float x[NIN] = {0, 0, 0, 0, 0, 0};
    if (valid) {
      for (int k = 0; k < NIN; ++k) x[k] = rows[row * stride + k];
      t = rows[row * stride + NIN];
    }
    put_input(S.x, lane, valid ? x : nullptr, s.norm);
  }
  __syncthreads();
  layer<TMT, K1>(S.x, AST, S.a1, AST, net.wt + T_W1, s.params + OFF_B1, S.z1, ZST, lane);
  __syncthreads();
  layer<TMT, HID>(S.a1, AST, S.a2, AST, net.wt + T_W2, s.params + OFF_B2, S.z2, ZST, lane);
  __syncthreads();
  layer<TMT, HID>(S.a2, AST, S.a3, AST, net.wt + T_W3, s.params + OFF_B3, S.z3, ZST, lane);
  __syncthreads();
  float err = 0.f;
  if (lane < TR) {
    float y = s.params[OFF_B4];
    for (int k = 0; k < HID; ++k) y += from_bf16(S.a3[lane * AST + k]) * s.params[OFF_W4 + k];
    const float ts = (t - s.norm[2 * NIN]) / s.norm[2 * NIN + 1];
    err = valid ? y - ts : 0.f;
    S.dy[lane] = 2.0f * err / (float)n;
  }
  float l2 = err * err;
  for (int o = 32; o > 0; o >>= 1) l2 += __shfl_xor(l2, o, 64);
  if (lane == 0) atomicAdd(s.loss, l2 / (float)n);
  __syncthreads();
  // output layer: dw4, db4 and dZ3 = dy w4 silu'(Z3)
  {
    float g = 0.f;
    for (int m = 0; m < TR; ++m) g += from_bf16(S.a3[m * AST + lane]) * S.dy[m];
    atomicAdd(s.grad + OFF_W4 + lane, g);
    float d = lane < TR ? S.dy[lane] : 0.f;
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if (lane == 0) atomicAdd(s.grad + OFF_B4, d);
    if (lane < TR)
      for (int k = 0; k < HID; ++k)
        S.dza[lane * AST + k] =
            to_bf16(S.dy[lane] * s.params[OFF_W4 + k] * dsilu(S.z3[lane * ZST + k]));
  }
  __syncthreads();
  bias_grad(S.dza, s.grad + OFF_B3, lane);
  weight_grad<4>(S.a2, S.dza, s.grad + OFF_W3, lane);
  back_layer(S.dza, net.wr + OFF_W3, S.z2, S.dzb, lane);
  __syncthreads();
  bias_grad(S.dzb, s.grad + OFF_B2, lane);
  weight_grad<4>(S.a1, S.dzb, s.grad + OFF_W2, lane);
  back_layer(S.dzb, net.wr + OFF_W2, S.z1, S.dza, lane);
  __syncthreads();
  bias_grad(S.dza, s.grad + OFF_B1, lane);
  weight_grad<1>(S.x, S.dza, s.grad + OFF_W1, lane);
}

__global__ void zero_k(float *a, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    a[k] = 0.f;
}

// BF16 copies (row-major and transposed) of the FP32 parameters.
__global__ void refresh_bf16_k(State s) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NPARAM) s.wbf[k] = to_bf16(s.params[k]);
  if (k < K1 * HID) {  // W1 [k1][n] -> W1^T [n][k1]
    const int r = k / HID, c = k % HID;
    s.wbt[T_W1 + c * K1 + r] = to_bf16(s.params[OFF_W1 + k]);
  }
  if (k < HID * HID) {
    const int r = k / HID, c = k % HID;
    s.wbt[T_W2 + c * HID + r] = to_bf16(s.params[OFF_W2 + k]);
    s.wbt[T_W3 + c * HID + r] = to_bf16(s.params[OFF_W3 + k]);
  }
}

__global__ void adam_k(State s, float lr, float b1, float b2, float eps, int t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NPARAM) return;
  const float g = s.grad[k];
  const float m = b1 * s.m[k] + (1.f - b1) * g;
  const float v = b2 * s.v[k] + (1.f - b2) * g * g;
  s.m[k] = m;
  s.v[k] = v;
  const float mh = m / (1.f - powf(b1, (float)t));
  const float vh = v / (1.f - powf(b2, (float)t));
  s.params[k] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void __launch_bounds__(64) mlp_predict_k(State s, const float *rows, int64_t n,
                                                    int64_t stride, float *y) {
  __shared__ uint16_t tile[16 * AST];
  const int lane = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * 64 + lane;
  float x[NIN] = {0, 0, 0, 0, 0, 0};
  if (row < n)
    for (int k = 0; k < NIN; ++k) x[k] = rows[row * stride + k];
  const float out = forward_wave(tile, row < n ? x : nullptr, net_of(s), lane);
  if (row < n) y[row] = out;
}

int hipret(hipError_t e) { return e == hipSuccess ? MFM_OK : MFM_E_HIP; }

}  // namespace

const void *mlp_net_of(const void *state, void *net_out) {
  State s = carve((void *)state);
  *reinterpret_cast<Net *>(net_out) = net_of(s);
  return net_out;
}

extern "C" {

size_t mfm_mlp_state_bytes(void) { return state_bytes(); }

int mfm_mlp_param_count(void) { return NPARAM; }

int mfm_mlp_init(void *state, const float *params_host, const float *norm_host, void *stream) {
  if (!state || !params_host || !norm_host) return MFM_E_ARG;
  for (int k = 0; k < NIN; ++k)
    if (!(norm_host[NIN + k] > 0.f)) return MFM_E_ARG;
  if (!(norm_host[2 * NIN + 1] > 0.f)) return MFM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  State s = carve(state);
  hipError_t e = hipMemsetAsync(state, 0, state_bytes(), st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.params, params_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.norm, norm_host, sizeof(float) * NNORM, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return MFM_E_HIP;
  refresh_bf16_k<<<(NPARAM + 255) / 256, 256, 0, st>>>(s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return hipret(e);
}

int mfm_mlp_backward(void *state, const float *rows_dev, int64_t n, int64_t stride,
                     float *loss_host, void *stream) {
  if (!state || !rows_dev || n <= 0 || stride < NIN + 1) return MFM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  State s = carve(state);
  zero_k<<<64, 256, 0, st>>>(s.grad, NPARAM_PAD);
  zero_k<<<1, 64, 0, st>>>(s.loss, 16);
  mlp_backward_k<<<(int)((n + TR - 1) / TR), 64, 0, st>>>(s, rows_dev, n, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return MFM_E_HIP;
  if (loss_host) {
    e = hipMemcpyAsync(loss_host, s.loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  return hipret(e);
}

int mfm_mlp_adam(void *state, float lr, int step, void *stream) {
  if (!state || step < 1 || !(lr >= 0.f)) return MFM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  State s = carve(state);
  adam_k<<<(NPARAM + 255) / 256, 256, 0, st>>>(s, lr, 0.9f, 0.999f, 1e-8f, step);
  refresh_bf16_k<<<(NPARAM + 255) / 256, 256, 0, st>>>(s);
  return hipret(hipGetLastError());
}

int mfm_mlp_train_step(void *state, const float *rows_dev, int64_t n, int64_t stride, float lr,
                       int step, float *loss_host, void *stream) {
  int rc = mfm_mlp_backward(state, rows_dev, n, stride, nullptr, stream);
  if (rc == MFM_OK) rc = mfm_mlp_adam(state, lr, step, stream);
  if (rc == MFM_OK && loss_host) {
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(loss_host, carve(state).loss, sizeof(float),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    rc = hipret(e);
  }
  return rc;
}

int mfm_mlp_predict(const void *state, const float *rows_dev, int64_t n, int64_t stride,
                    float *y_dev, void *stream) {
  if (!state || !rows_dev || !y_dev || n <= 0 || stride < NIN) return MFM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  mlp_predict_k<<<(int)((n + 63) / 64), 64, 0, st>>>(carve((void *)state), rows_dev, n, stride,
                                                      y_dev);
  return hipret(hipGetLastError());
}

int mfm_mlp_get(const void *state, float *params_host, float *grad_host, void *stream) {
  if (!state) return MFM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  State s = carve((void *)state);
  hipError_t e = hipSuccess;
  if (params_host)
    e = hipMemcpyAsync(params_host, s.params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && grad_host)
    e = hipMemcpyAsync(grad_host, s.grad, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return hipret(e);
}

}  // extern "C"
