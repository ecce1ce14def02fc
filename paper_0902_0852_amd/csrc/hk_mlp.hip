// The precision-proposal network: a float32 MLP 3 -> 64 -> 64 -> 64 -> 2
// with ReLU on the hidden layers, trained by mean squared error with Adam.
// Forward, backward, loss and optimiser step are HIP kernels; the host only
// launches them.
//
// Parameters are one packed vector: W1 (64x3), b1, W2 (64x64), b2, W3
// (64x64), b3, W4 (2x64), b4, matrices row-major (outputs x inputs).  The
// activation cache of one sample holds its input and the three post-ReLU
// hidden vectors (3 + 3*64 floats); the delta scratch holds the three hidden
// deltas (3*64 floats).
//
// Layout on the GPU: one 64-lane wavefront per block, lane u owns hidden unit
// u of every layer.  A block walks a contiguous tile of samples; per sample
// the previous layer's activations sit in LDS and are read as broadcasts,
// while each lane keeps the weights it needs in registers (row u of W2/W3 for
// the forward pass, column u for the backward pass), so the inner loops are
// plain FMAs with no LDS bank conflicts.
#include <hip/hip_runtime.h>

#include "hk_internal.hpp"

namespace hk {
namespace {

constexpr int NI = 3, NH = 64, NO = 2;
constexpr int O_W1 = 0, O_B1 = O_W1 + NH * NI, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH,
              O_W3 = O_B2 + NH, O_B3 = O_W3 + NH * NH, O_W4 = O_B3 + NH, O_B4 = O_W4 + NO * NH,
              NPARAM = O_B4 + NO;
constexpr int CACHE = NI + 3 * NH;
constexpr int TILE = 32;   // samples per block

__device__ __forceinline__ float relu(float z) { return z > 0.f ? z : 0.f; }

__global__ void __launch_bounds__(64) k_mlp_forward(const float* __restrict__ W,
                                                    const float* __restrict__ X, int batch,
                                                    float* __restrict__ Y, float* __restrict__ cache) {
  const int u = threadIdx.x;
  float w1[NI], w2[NH], w3[NH];
#pragma unroll
  for (int i = 0; i < NI; i++) w1[i] = W[O_W1 + u * NI + i];
#pragma unroll
  for (int i = 0; i < NH; i++) { w2[i] = W[O_W2 + u * NH + i]; w3[i] = W[O_W3 + u * NH + i]; }
  const float b1 = W[O_B1 + u], b2 = W[O_B2 + u], b3 = W[O_B3 + u];
  const float w40 = W[O_W4 + u], w41 = W[O_W4 + NH + u];
  const float b40 = W[O_B4], b41 = W[O_B4 + 1];
  __shared__ float hs[NH];
  __shared__ float red[2][NH];
  const int s0 = blockIdx.x * TILE, s1 = min(batch, s0 + TILE);
  for (int s = s0; s < s1; s++) {
    const float* x = X + (int64_t)s * NI;
    float z = b1;
#pragma unroll
    for (int i = 0; i < NI; i++) z = __builtin_fmaf(w1[i], x[i], z);
    const float a1 = relu(z);
    hs[u] = a1;
    __syncthreads();
    z = b2;
#pragma unroll
    for (int i = 0; i < NH; i++) z = __builtin_fmaf(w2[i], hs[i], z);
    const float a2 = relu(z);
    __syncthreads();
    hs[u] = a2;
    __syncthreads();
    z = b3;
#pragma unroll
    for (int i = 0; i < NH; i++) z = __builtin_fmaf(w3[i], hs[i], z);
    const float a3 = relu(z);
    red[0][u] = w40 * a3;
    red[1][u] = w41 * a3;
    __syncthreads();
    if (u < NO) {
      // fixed summation order: units 0..63
      float y = 0.f;
      for (int i = 0; i < NH; i++) y += red[u][i];
      Y[(int64_t)s * NO + u] = y + (u == 0 ? b40 : b41);
    }
    if (cache) {
      float* cp = cache + (int64_t)s * CACHE;
      if (u < NI) cp[u] = x[u];
      cp[NI + u] = a1;
      cp[NI + NH + u] = a2;
      cp[NI + 2 * NH + u] = a3;
    }
    __syncthreads();
  }
}

// per-sample deltas of the hidden layers:
//   d3 = (W4^T dY) * [h3 > 0],  d2 = (W3^T d3) * [h2 > 0],  d1 = (W2^T d2) * [h1 > 0]
__global__ void __launch_bounds__(64) k_mlp_deltas(const float* __restrict__ W,
                                                   const float* __restrict__ cache,
                                                   const float* __restrict__ dY, int batch,
                                                   float* __restrict__ delta) {
  const int u = threadIdx.x;
  float c2[NH], c3[NH];   // column u of W2 and of W3
#pragma unroll
  for (int o = 0; o < NH; o++) { c2[o] = W[O_W2 + o * NH + u]; c3[o] = W[O_W3 + o * NH + u]; }
  const float w40 = W[O_W4 + u], w41 = W[O_W4 + NH + u];
  __shared__ float ds[NH];
  const int s0 = blockIdx.x * TILE, s1 = min(batch, s0 + TILE);
  for (int s = s0; s < s1; s++) {
    const float* cp = cache + (int64_t)s * CACHE;
    float* dp = delta + (int64_t)s * 3 * NH;
    const float g0 = dY[(int64_t)s * NO], g1 = dY[(int64_t)s * NO + 1];
    const float d3 = cp[NI + 2 * NH + u] > 0.f ? __builtin_fmaf(w41, g1, w40 * g0) : 0.f;
    ds[u] = d3;
    __syncthreads();
    float g = 0.f;
#pragma unroll
    for (int o = 0; o < NH; o++) g = __builtin_fmaf(c3[o], ds[o], g);
    const float d2 = cp[NI + NH + u] > 0.f ? g : 0.f;
    __syncthreads();
    ds[u] = d2;
    __syncthreads();
    g = 0.f;
#pragma unroll
    for (int o = 0; o < NH; o++) g = __builtin_fmaf(c2[o], ds[o], g);
    const float d1 = cp[NI + u] > 0.f ? g : 0.f;
    dp[u] = d1;
    dp[NH + u] = d2;
    dp[2 * NH + u] = d3;
    __syncthreads();
  }
}

// weight gradients: one thread per parameter, a fixed-order sum over the
// batch (deterministic; a wavefront shares its output unit, so the delta
// load is a broadcast and the activation load is coalesced)
__global__ void __launch_bounds__(256) k_mlp_wgrad(const float* __restrict__ cache,
                                                   const float* __restrict__ delta,
                                                   const float* __restrict__ dY, int batch,
                                                   float* __restrict__ dW) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  int o, i, dsel, aoff, nin;   // dsel: 0..2 hidden delta, 3 output gradient
  if (p < O_B1)      { nin = NI; o = (p - O_W1) / nin; i = (p - O_W1) % nin; dsel = 0; aoff = 0; }
  else if (p < O_W2) { o = p - O_B1; i = -1; dsel = 0; aoff = 0; }
  else if (p < O_B2) { nin = NH; o = (p - O_W2) / nin; i = (p - O_W2) % nin; dsel = 1; aoff = NI; }
  else if (p < O_W3) { o = p - O_B2; i = -1; dsel = 1; aoff = 0; }
  else if (p < O_B3) { nin = NH; o = (p - O_W3) / nin; i = (p - O_W3) % nin; dsel = 2; aoff = NI + NH; }
  else if (p < O_W4) { o = p - O_B3; i = -1; dsel = 2; aoff = 0; }
  else if (p < O_B4) { nin = NH; o = (p - O_W4) / nin; i = (p - O_W4) % nin; dsel = 3; aoff = NI + 2 * NH; }
  else               { o = p - O_B4; i = -1; dsel = 3; aoff = 0; }
  float acc = 0.f;
  for (int s = 0; s < batch; s++) {
    const float d = dsel == 3 ? dY[(int64_t)s * NO + o] : delta[(int64_t)s * 3 * NH + dsel * NH + o];
    const float a = i < 0 ? 1.f : cache[(int64_t)s * CACHE + aoff + i];
    acc = __builtin_fmaf(d, a, acc);
  }
  dW[p] = acc;
}

// Adam (Kingma & Ba 2015, Algorithm 1) with the bias corrections c1 = 1 -
// b1^t, c2 = 1 - b2^t passed in
__global__ void k_mlp_adam(float* __restrict__ W, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  W[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// mean squared error over batch x 2 outputs and its gradient dY
__global__ void __launch_bounds__(256) k_mlp_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                                 int batch, float* __restrict__ dY,
                                                 float* __restrict__ loss) {
  __shared__ float part[256];
  const int n = batch * NO;
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d / (float)n;
    acc = __builtin_fmaf(d, d, acc);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)n;
}

hk_status mfail(const char* msg) { g_err = msg; return HK_EINVAL; }
hk_status launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return HK_OK;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HK_EDEVICE;
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" {

int hk_mlp_nparams(void) { return NPARAM; }
int hk_mlp_cache_floats(void) { return CACHE; }

hk_status hk_mlp_forward(const float* W, const float* X, int batch, float* Y, float* act_cache,
                         hipStream_t s) {
  if (!W || !X || !Y || batch < 1) return mfail("mlp forward: null pointer or empty batch");
  hipLaunchKernelGGL(k_mlp_forward, dim3((batch + TILE - 1) / TILE), dim3(64), 0, s, W, X, batch, Y,
                     act_cache);
  return launched("mlp forward");
}

hk_status hk_mlp_backward(const float* W, const float* act_cache, const float* dY, int batch, float* dW,
                          float* delta, hipStream_t s) {
  if (!W || !act_cache || !dY || !dW || !delta || batch < 1)
    return mfail("mlp backward: null pointer or empty batch");
  hipLaunchKernelGGL(k_mlp_deltas, dim3((batch + TILE - 1) / TILE), dim3(64), 0, s, W, act_cache, dY,
                     batch, delta);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((NPARAM + 255) / 256), dim3(256), 0, s, act_cache, delta, dY,
                     batch, dW);
  return launched("mlp backward");
}

hk_status hk_mlp_mse(const float* Y, const float* T, int batch, float* dY, float* loss, hipStream_t s) {
  if (!Y || !T || !dY || !loss || batch < 1) return mfail("mlp mse: null pointer or empty batch");
  hipLaunchKernelGGL(k_mlp_mse, dim3(1), dim3(256), 0, s, Y, T, batch, dY, loss);
  return launched("mlp mse");
}

hk_status hk_mlp_adam_step(float* W, float* m, float* v, const float* dW, int nparams, float lr,
                           float b1, float b2, float eps, int step, hipStream_t s) {
  if (!W || !m || !v || !dW || nparams < 1 || step < 1) return mfail("adam: bad arguments");
  const float c1 = (float)(1.0 - pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - pow((double)b2, (double)step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((nparams + 255) / 256), dim3(256), 0, s, W, m, v, dW, nparams, lr,
                     b1, b2, eps, c1, c2);
  return launched("adam");
}

}  // extern "C"
