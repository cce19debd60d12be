// Cost-model MLP (12 -> 64 -> 64 -> 3, ReLU, FP32): forward, backward and Adam.
//
// The network predicts, from features of a pending update batch, the log running time of
// the incremental and of the recompute path of an algorithm and the log2 scale of the
// initial slab count.  It is tiny (5,187 parameters), so plain FP32 FMAs are used: the
// weights sit in LDS and one thread evaluates one sample.  Weight gradients are written
// without atomics (one thread per weight sums over the minibatch), so a training step is
// deterministic.  Adam follows Kingma and Ba (ICLR 2015) with bias correction.
#include <algorithm>
#include <mutex>

#include "mk_internal.h"

using namespace mk;

namespace {

constexpr int kIn = MK_MLP_IN, kHid = MK_MLP_HIDDEN, kOut = MK_MLP_OUT;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;
static_assert(kParams == MK_MLP_PARAMS, "parameter count");

__device__ inline void load_params(const float* __restrict__ p, float* lds) {
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) lds[i] = p[i];
  __syncthreads();
}

// h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 (one sample per thread).
__device__ inline void forward_one(const float* P, const float* x, float* h1, float* h2, float* y) {
#pragma unroll 4
  for (int j = 0; j < kHid; ++j) {
    float a = P[oB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a = fmaf(P[oW1 + j * kIn + i], x[i], a);
    h1[j] = a > 0.f ? a : 0.f;
  }
#pragma unroll 2
  for (int j = 0; j < kHid; ++j) {
    float a = P[oB2 + j];
#pragma unroll 8
    for (int i = 0; i < kHid; ++i) a = fmaf(P[oW2 + j * kHid + i], h1[i], a);
    h2[j] = a > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int k = 0; k < kOut; ++k) {
    float a = P[oB3 + k];
#pragma unroll 8
    for (int i = 0; i < kHid; ++i) a = fmaf(P[oW3 + k * kHid + i], h2[i], a);
    y[k] = a;
  }
}

__global__ void __launch_bounds__(kBlock) k_mlp_forward(const float* __restrict__ params,
                                                        const float* __restrict__ X, uint32_t n,
                                                        float* __restrict__ Y) {
  __shared__ float P[kParams];
  load_params(params, P);
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kIn], h1[kHid], h2[kHid], y[kOut];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = X[(uint64_t)s * kIn + i];
  forward_one(P, x, h1, h2, y);
#pragma unroll
  for (int k = 0; k < kOut; ++k) Y[(uint64_t)s * kOut + k] = y[k];
}

// Per sample: forward, then the output and hidden-layer error terms of the masked mean
// squared error L = sum_{s,k} m_sk (y_sk - t_sk)^2 / sum m.  Stores H1, H2 (activations)
// and D1, D2, DY (error terms) for the weight-gradient pass, and the squared errors.
__global__ void __launch_bounds__(kBlock) k_mlp_backward_samples(
    const float* __restrict__ params, const float* __restrict__ X, const float* __restrict__ T,
    const float* __restrict__ M, uint32_t n, const double* __restrict__ count, float* __restrict__ H1,
    float* __restrict__ H2, float* __restrict__ D1, float* __restrict__ D2, float* __restrict__ DY,
    double* __restrict__ loss) {
  __shared__ float P[kParams];
  __shared__ double part[kBlock / 64];
  load_params(params, P);
  const float inv_count = (float)(1.0 / *count);
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  double se = 0.0;
  if (s < n) {
    float x[kIn], h1[kHid], h2[kHid], y[kOut], dy[kOut], d2[kHid];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = X[(uint64_t)s * kIn + i];
    forward_one(P, x, h1, h2, y);
#pragma unroll
    for (int k = 0; k < kOut; ++k) {
      const float m = M[(uint64_t)s * kOut + k];
      const float e = y[k] - T[(uint64_t)s * kOut + k];
      dy[k] = 2.f * m * e * inv_count;
      se += (double)m * e * e;
      DY[(uint64_t)s * kOut + k] = dy[k];
    }
    for (int j = 0; j < kHid; ++j) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < kOut; ++k) a = fmaf(P[oW3 + k * kHid + j], dy[k], a);
      d2[j] = h2[j] > 0.f ? a : 0.f;
      D2[(uint64_t)s * kHid + j] = d2[j];
      H2[(uint64_t)s * kHid + j] = h2[j];
    }
    for (int i = 0; i < kHid; ++i) {
      float a = 0.f;
#pragma unroll 8
      for (int j = 0; j < kHid; ++j) a = fmaf(P[oW2 + j * kHid + i], d2[j], a);
      D1[(uint64_t)s * kHid + i] = h1[i] > 0.f ? a : 0.f;
      H1[(uint64_t)s * kHid + i] = h1[i];
    }
  }
  for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = se;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < kBlock / 64; ++i) t += part[i];
    if (t != 0.0) atomicAdd(loss, t);
  }
}

// One thread per parameter: the weight gradient is a sum over the minibatch of
// (error term of the output unit) x (input of the layer), the bias gradient the sum of
// the error terms.
__global__ void __launch_bounds__(kBlock) k_mlp_weight_grads(
    const float* __restrict__ X, const float* __restrict__ H1, const float* __restrict__ H2,
    const float* __restrict__ D1, const float* __restrict__ D2, const float* __restrict__ DY,
    uint32_t n, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float* err;
  const float* in;
  int es, is, j, i;  // error row stride / index, input row stride / index (-1: bias)
  if (p < oB1) {
    err = D1; es = kHid; j = (p - oW1) / kIn; in = X; is = kIn; i = (p - oW1) % kIn;
  } else if (p < oW2) {
    err = D1; es = kHid; j = p - oB1; in = nullptr; is = 0; i = -1;
  } else if (p < oB2) {
    err = D2; es = kHid; j = (p - oW2) / kHid; in = H1; is = kHid; i = (p - oW2) % kHid;
  } else if (p < oW3) {
    err = D2; es = kHid; j = p - oB2; in = nullptr; is = 0; i = -1;
  } else if (p < oB3) {
    err = DY; es = kOut; j = (p - oW3) / kHid; in = H2; is = kHid; i = (p - oW3) % kHid;
  } else {
    err = DY; es = kOut; j = p - oB3; in = nullptr; is = 0; i = -1;
  }
  float acc = 0.f;
  for (uint32_t s = 0; s < n; ++s) {
    const float e = err[(uint64_t)s * es + j];
    acc = i < 0 ? acc + e : fmaf(e, in[(uint64_t)s * is + i], acc);
  }
  grad[p] = acc;
}

// Number of supervised outputs (sum of the mask), and a zeroed loss accumulator.
__global__ void __launch_bounds__(kBlock) k_mlp_mask_count(const float* __restrict__ M, uint32_t n,
                                                           double* count, double* loss) {
  __shared__ double part[kBlock / 64];
  double c = 0;
  for (uint32_t i = threadIdx.x; i < n * kOut; i += blockDim.x) c += M[i];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < kBlock / 64; ++i) t += part[i];
    *count = t > 0 ? t : 1.0;
    *loss = 0.0;
  }
}

__global__ void k_mlp_loss_mean(const double* count, double* loss) {
  if (threadIdx.x == 0) *loss /= *count;
}

__global__ void k_mlp_adam(float* __restrict__ params, const float* __restrict__ grad,
                           float* __restrict__ m, float* __restrict__ v, uint32_t np, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  params[i] -= lr * mh / (sqrtf(vh) + eps);
}

inline bool aligned4(const void* p) { return ((uintptr_t)p & 3) == 0; }

constexpr size_t grad_ws_bytes(uint32_t n) { return (size_t)n * (4 * kHid + kOut) * sizeof(float) + 512; }

// Workspace of mk_mlp_grad_static: one copy per GPU, held until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device array: the device address
// comes from hipGetSymbolAddress, once per device, and only that address is passed on.
constexpr size_t kStaticGradBytes = grad_ws_bytes(MK_MLP_GRAD_STATIC_MAX);
static __device__ __align__(256) unsigned char scratch[kStaticGradBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on its first use).
mk_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MK_ERR_HIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MK_ERR_HIP;
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return MK_OK;
}

// The gradient's kernels with the workspace at d_ws (at least grad_ws_bytes(n) bytes).
mk_status grad_launch(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                      uint32_t n, float* d_grad, void* d_ws, double* d_loss, hipStream_t stream) {
  float* ws = reinterpret_cast<float*>(((uintptr_t)d_ws + 255) & ~uintptr_t(255));
  float* H1 = ws;
  float* H2 = H1 + (size_t)n * kHid;
  float* D1 = H2 + (size_t)n * kHid;
  float* D2 = D1 + (size_t)n * kHid;
  float* DY = D2 + (size_t)n * kHid;
  double* cnt = reinterpret_cast<double*>(DY + (size_t)n * kOut + 1);  // 8-byte aligned below
  cnt = reinterpret_cast<double*>(((uintptr_t)cnt + 7) & ~uintptr_t(7));
  hipLaunchKernelGGL(k_mlp_mask_count, dim3(1), dim3(kBlock), 0, stream, d_mask, n, cnt, d_loss);
  hipLaunchKernelGGL(k_mlp_backward_samples, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                     d_params, d_x, d_t, d_mask, n, cnt, H1, H2, D1, D2, DY, d_loss);
  hipLaunchKernelGGL(k_mlp_weight_grads, dim3((kParams + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                     d_x, H1, H2, D1, D2, DY, n, d_grad);
  hipLaunchKernelGGL(k_mlp_loss_mean, dim3(1), dim3(64), 0, stream, cnt, d_loss);
  return hipGetLastError() == hipSuccess ? MK_OK : MK_ERR_HIP;
}

}  // namespace

namespace mk {
void mlp_forward_launch(const float* params, const float* x, uint32_t n, float* y, hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, params, x, n, y);
}
}  // namespace mk

extern "C" {

size_t mk_mlp_workspace_bytes(uint32_t n) { return grad_ws_bytes(n); }

mk_status mk_mlp_forward(const float* d_params, const float* d_x, uint32_t n, float* d_y,
                         hipStream_t stream) {
  if (!d_params || (n && (!d_x || !d_y)) || !aligned4(d_params)) return MK_ERR_INVALID_ARG;
  if (n == 0) return MK_OK;
  mlp_forward_launch(d_params, d_x, n, d_y, stream);
  return hipGetLastError() == hipSuccess ? MK_OK : MK_ERR_HIP;
}

mk_status mk_mlp_grad(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                      uint32_t n, float* d_grad, void* d_ws, size_t ws_bytes, double* d_loss,
                      hipStream_t stream) {
  if (!d_params || !d_grad || !d_loss || n == 0 || !d_x || !d_t || !d_mask || !d_ws)
    return MK_ERR_INVALID_ARG;
  if (ws_bytes < grad_ws_bytes(n)) return MK_ERR_CAPACITY;
  return grad_launch(d_params, d_x, d_t, d_mask, n, d_grad, d_ws, d_loss, stream);
}

mk_status mk_mlp_grad_static(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                             uint32_t n, float* d_grad, double* d_loss, hipStream_t stream) {
  if (!d_params || !d_grad || !d_loss || n == 0 || !d_x || !d_t || !d_mask) return MK_ERR_INVALID_ARG;
  if (n > MK_MLP_GRAD_STATIC_MAX) return MK_ERR_CAPACITY;
  void* ws = nullptr;
  if (mk_status st = scratch_address(&ws); st != MK_OK) return st;
  // every word the kernels read back (activations, error terms, the mask count) is written
  // first in the same call, so the array needs no clearing between calls
  return grad_launch(d_params, d_x, d_t, d_mask, n, d_grad, ws, d_loss, stream);
}


mk_status mk_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t n_params,
                      float lr, float beta1, float beta2, float eps, uint32_t step, hipStream_t stream) {
  if (!d_params || !d_grad || !d_m || !d_v || n_params == 0 || step == 0) return MK_ERR_INVALID_ARG;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((n_params + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, d_params,
                     d_grad, d_m, d_v, n_params, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? MK_OK : MK_ERR_HIP;
}

}  // extern "C"
