// mlp.hip -- forward, loss, backward and Adam kernels of the selector MLP.
//
// Network: x[16] -> relu(x W1 + b1)[64] -> relu(h1 W2 + b2)[64] -> h2 W3 + b3 [16].
// Every sum runs over its index in increasing order with explicit fused
// multiply-adds, and every batch reduction is a fixed loop or a fixed-shape tree,
// so the kernels are deterministic (no float atomics) and the host forward in
// selector.hip reproduces the device forward bit for bit.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"
#include "mlp.hpp"

namespace eiger {

namespace {

// y[b][j] = act(sum_i x[b][i] * W[i][j] + bias[j])
__global__ void k_mlp_layer(const float *__restrict__ x, int in, const float *__restrict__ W,
                            const float *__restrict__ bias, int out, float *__restrict__ y, int batch,
                            int relu) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(batch) * out) return;
  const int b = static_cast<int>(t / out), j = static_cast<int>(t % out);
  float acc = 0.f;
  for (int i = 0; i < in; ++i) acc = fmaf(x[int64_t(b) * in + i], W[i * out + j], acc);
  acc += bias[j];
  y[t] = (relu && acc < 0.f) ? 0.f : acc;
}

// Masked squared error: one workgroup, fixed-shape reduction. Writes
// out[0] = sum mask*(y-t)^2 / sum mask (0 when the mask is empty), out[1] = sum mask.
__global__ void __launch_bounds__(1024) k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t,
                                                   const float *__restrict__ m, int64_t n,
                                                   float *__restrict__ out) {
  __shared__ float se[1024], sm[1024];
  float a = 0.f, c = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float d = y[i] - t[i];
    a = fmaf(m[i] * d, d, a);
    c += m[i];
  }
  se[threadIdx.x] = a;
  sm[threadIdx.x] = c;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      se[threadIdx.x] += se[threadIdx.x + w];
      sm[threadIdx.x] += sm[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0] > 0.f ? se[0] / sm[0] : 0.f;
    out[1] = sm[0];
  }
}

// dY = 2 * mask * (y - t) / sum(mask)
__global__ void k_mlp_dy(const float *__restrict__ y, const float *__restrict__ t,
                         const float *__restrict__ m, int64_t n, const float *__restrict__ lossv,
                         float *__restrict__ dy) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float msum = lossv[1];
  dy[i] = msum > 0.f ? 2.f * m[i] * (y[i] - t[i]) / msum : 0.f;
}

// dW[i][j] = sum_b a[b][i] * dz[b][j]; db[j] = sum_b dz[b][j] (threads with i == in).
__global__ void k_mlp_grad_w(const float *__restrict__ a, int in, const float *__restrict__ dz, int out,
                             int batch, float *__restrict__ dW, float *__restrict__ db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (in + 1) * out) return;
  const int i = t / out, j = t % out;
  float acc = 0.f;
  if (i < in) {
    for (int b = 0; b < batch; ++b) acc = fmaf(a[int64_t(b) * in + i], dz[int64_t(b) * out + j], acc);
    dW[i * out + j] = acc;
  } else {
    for (int b = 0; b < batch; ++b) acc += dz[int64_t(b) * out + j];
    db[j] = acc;
  }
}

// da[b][i] = (sum_j dz[b][j] * W[i][j]) * [act[b][i] > 0]  (ReLU derivative)
__global__ void k_mlp_grad_in(const float *__restrict__ dz, int out, const float *__restrict__ W, int in,
                              const float *__restrict__ act, int batch, float *__restrict__ da) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(batch) * in) return;
  const int b = static_cast<int>(t / in), i = static_cast<int>(t % in);
  float acc = 0.f;
  for (int j = 0; j < out; ++j) acc = fmaf(dz[int64_t(b) * out + j], W[i * out + j], acc);
  da[t] = act[t] > 0.f ? acc : 0.f;
}

// Adam with bias correction (Kingma & Ba 2015).
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Inference without scratch memory: one 64-thread workgroup per row at a time,
// hidden activations in LDS; each output is the same ordered fused sum as in
// k_mlp_layer, so the result equals the layer-by-layer forward bit for bit.
__global__ void __launch_bounds__(64) k_mlp_forward_rows(const float *__restrict__ P, const float *__restrict__ x,
                                                         int batch, float *__restrict__ y) {
  __shared__ float xs[kIn], h1[kHid], h2[kHid];
  const MlpOffsets o;
  const int j = threadIdx.x;
  for (int b = blockIdx.x; b < batch; b += gridDim.x) {
    if (j < kIn) xs[j] = x[int64_t(b) * kIn + j];
    __syncthreads();
    float acc = 0.f;
    for (int i = 0; i < kIn; ++i) acc = fmaf(xs[i], P[o.W1 + i * kHid + j], acc);
    acc += P[o.b1 + j];
    h1[j] = acc < 0.f ? 0.f : acc;
    __syncthreads();
    acc = 0.f;
    for (int i = 0; i < kHid; ++i) acc = fmaf(h1[i], P[o.W2 + i * kHid + j], acc);
    acc += P[o.b2 + j];
    h2[j] = acc < 0.f ? 0.f : acc;
    __syncthreads();
    if (j < kOut) {
      acc = 0.f;
      for (int i = 0; i < kHid; ++i) acc = fmaf(h2[i], P[o.W3 + i * kOut + j], acc);
      y[int64_t(b) * kOut + j] = acc + P[o.b3 + j];
    }
    __syncthreads();
  }
}

unsigned blocks(int64_t n, int per = 256) { return static_cast<unsigned>((n + per - 1) / per); }

struct TrainWs {
  float *h1, *h2, *y, *dy, *dh2, *dh1, *lossv;
};

TrainWs train_layout(Workspace &ws, int batch) {
  TrainWs w;
  const size_t B = static_cast<size_t>(batch);
  w.h1 = ws.take<float>(B * kHid);
  w.h2 = ws.take<float>(B * kHid);
  w.y = ws.take<float>(B * kOut);
  w.dy = ws.take<float>(B * kOut);
  w.dh2 = ws.take<float>(B * kHid);
  w.dh1 = ws.take<float>(B * kHid);
  w.lossv = ws.take<float>(2);
  return w;
}

int forward(const float *P, const float *x, int batch, float *h1, float *h2, float *y, hipStream_t s) {
  const MlpOffsets o;
  EIGER_LAUNCH("mlp_forward", k_mlp_layer, dim3(blocks(int64_t(batch) * kHid)), dim3(256), 0, s, x, kIn,
               P + o.W1, P + o.b1, kHid, h1, batch, 1);
  EIGER_LAUNCH("mlp_forward", k_mlp_layer, dim3(blocks(int64_t(batch) * kHid)), dim3(256), 0, s, h1, kHid,
               P + o.W2, P + o.b2, kHid, h2, batch, 1);
  EIGER_LAUNCH("mlp_forward", k_mlp_layer, dim3(blocks(int64_t(batch) * kOut)), dim3(256), 0, s, h2, kHid,
               P + o.W3, P + o.b3, kOut, y, batch, 0);
  return EIGER_OK;
}

}  // namespace

}  // namespace eiger

using namespace eiger;

extern "C" int64_t eiger_mlp_param_count(void) { return kParams; }

extern "C" size_t eiger_mlp_train_workspace_size(int32_t batch) {
  if (batch <= 0) return 0;
  Workspace ws(nullptr, 0);
  train_layout(ws, batch);
  return ws.used;
}

extern "C" int eiger_mlp_forward(const float *params, const float *x, int32_t batch, float *y, void *stream) {
  if (!params || !y || batch < 0 || (batch > 0 && !x))
    return fail(EIGER_ERR_INVALID_ARG, "eiger_mlp_forward: bad arguments");
  if (batch == 0) return EIGER_OK;
  if (batch > (1 << 24)) return fail(EIGER_ERR_TOO_LARGE, "eiger_mlp_forward: batch above 2^24");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(batch, int64_t(device_cu_count()) * 16));
  EIGER_LAUNCH("mlp_forward_rows", k_mlp_forward_rows, dim3(grid), dim3(64), 0, s, params, x, batch, y);
  return EIGER_OK;
}

extern "C" int eiger_mlp_train_step(float *params, float *adam_m, float *adam_v, float *grads, const float *x,
                                    const float *target, const float *mask, int32_t batch, float lr,
                                    int32_t step, float *loss, void *ws_ptr, size_t ws_bytes, void *stream) {
  if (!params || !adam_m || !adam_v || !grads || !x || !target || !mask || !loss)
    return fail(EIGER_ERR_INVALID_ARG, "eiger_mlp_train_step: NULL pointer");
  if (batch <= 0 || batch > (1 << 24)) return fail(EIGER_ERR_INVALID_ARG, "eiger_mlp_train_step: batch out of range");
  if (step < 1) return fail(EIGER_ERR_INVALID_ARG, "eiger_mlp_train_step: step must be >= 1");
  if (!(lr > 0.f)) return fail(EIGER_ERR_INVALID_ARG, "eiger_mlp_train_step: lr must be > 0");
  Workspace ws(ws_ptr, ws_bytes);
  TrainWs w = train_layout(ws, batch);
  if (!ws_ptr || ws.used > ws_bytes)
    return fail(EIGER_ERR_WORKSPACE, "eiger_mlp_train_step: workspace too small (need " +
                                         std::to_string(ws.used) + " bytes)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const MlpOffsets o;
  const int64_t ny = int64_t(batch) * kOut;
  int rc;
  if ((rc = forward(params, x, batch, w.h1, w.h2, w.y, s))) return rc;
  EIGER_LAUNCH("mlp_loss", k_mlp_loss, dim3(1), dim3(1024), 0, s, w.y, target, mask, ny, w.lossv);
  EIGER_LAUNCH("mlp_backward", k_mlp_dy, dim3(blocks(ny)), dim3(256), 0, s, w.y, target, mask, ny, w.lossv,
               w.dy);
  EIGER_LAUNCH("mlp_backward", k_mlp_grad_w, dim3(blocks((kHid + 1) * kOut)), dim3(256), 0, s, w.h2, kHid,
               w.dy, kOut, batch, grads + o.W3, grads + o.b3);
  EIGER_LAUNCH("mlp_backward", k_mlp_grad_in, dim3(blocks(int64_t(batch) * kHid)), dim3(256), 0, s, w.dy,
               kOut, params + o.W3, kHid, w.h2, batch, w.dh2);
  EIGER_LAUNCH("mlp_backward", k_mlp_grad_w, dim3(blocks((kHid + 1) * kHid)), dim3(256), 0, s, w.h1, kHid,
               w.dh2, kHid, batch, grads + o.W2, grads + o.b2);
  EIGER_LAUNCH("mlp_backward", k_mlp_grad_in, dim3(blocks(int64_t(batch) * kHid)), dim3(256), 0, s, w.dh2,
               kHid, params + o.W2, kHid, w.h1, batch, w.dh1);
  EIGER_LAUNCH("mlp_backward", k_mlp_grad_w, dim3(blocks((kIn + 1) * kHid)), dim3(256), 0, s, x, kIn, w.dh1,
               kHid, batch, grads + o.W1, grads + o.b1);
  const float c1 = 1.f - std::pow(0.9f, static_cast<float>(step));
  const float c2 = 1.f - std::pow(0.999f, static_cast<float>(step));
  EIGER_LAUNCH("mlp_adam", k_adam, dim3(blocks(kParams)), dim3(256), 0, s, params, adam_m, adam_v, grads,
               static_cast<int>(kParams), lr, c1, c2);
  EIGER_HIP(hipMemcpyAsync(loss, w.lossv, sizeof(float), hipMemcpyDeviceToDevice, s));
  return EIGER_OK;
}
