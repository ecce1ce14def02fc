// Issue rate of the multiply instructions the update kernels use or could
// use, measured on the running GPU: the VALU multiplies, and the int8 matrix
// product of the matrix-core update (multiply-adds per second).  Every lane of a grid that fills
// every SIMD runs CH independent chains of one instruction kind (no chain
// waits on another, so the rate is the issue rate, not the latency); the
// chains' results are stored so that nothing is optimised away.  Each wave
// also records its shader-clock and constant-rate counter deltas,
// from which the clock during the run follows.
#include <hip/hip_runtime.h>

#include <chrono>
#include <string>

#include "hk_internal.hpp"

namespace hk {
namespace {

constexpr int RATE_CH = 16;       // independent chains per lane
constexpr int RATE_ITERS = 4096;  // steps of every chain
constexpr int RATE_WAVES_PER_SIMD = 8;

template <int KIND>
__global__ void __launch_bounds__(256) k_rate(int64_t* out, int64_t* clk, uint32_t seed) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t c0 = clock64(), w0 = wall_clock64();
  const uint32_t m = seed * 2654435761u + (uint32_t)tid;
  int64_t r = 0;
  // (the integer kinds are written as the instruction itself: as C the
  // compiler hoists the loop-invariant product out of the chains)
  if constexpr (KIND == HK_RATE_MAD_I64_I32) {
    // the update kernel's instruction: int64 += int32 * int32
    int64_t acc[RATE_CH];
    int32_t a[RATE_CH];
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) { acc[j] = j; a[j] = (int32_t)(m + 977u * j) & 0x1fffffff; }
    const int32_t b = (int32_t)(m >> 3) | 1;
    for (int i = 0; i < RATE_ITERS; i++) {
#pragma unroll
      for (int j = 0; j < RATE_CH; j++) {
        uint64_t cy;
        asm volatile("v_mad_i64_i32 %0, %1, %2, %3, %0" : "+v"(acc[j]), "=s"(cy) : "v"(a[j]), "v"(b));
      }
    }
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) r ^= acc[j];
  } else if constexpr (KIND == HK_RATE_MAD_U64_U32) {
    uint64_t acc[RATE_CH];
    uint32_t a[RATE_CH];
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) { acc[j] = j; a[j] = m + 977u * j; }
    const uint32_t b = (m >> 3) | 1u;
    for (int i = 0; i < RATE_ITERS; i++) {
#pragma unroll
      for (int j = 0; j < RATE_CH; j++) {
        uint64_t cy;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[j]), "=s"(cy) : "v"(a[j]), "v"(b));
      }
    }
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) r ^= (int64_t)acc[j];
  } else if constexpr (KIND == HK_RATE_MAD_U32_U24) {
    uint32_t acc[RATE_CH];
    uint32_t a[RATE_CH];
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) { acc[j] = j; a[j] = (m + 977u * j) & 0xffffffu; }
    const uint32_t b = ((m >> 3) | 1u) & 0xffffffu;
    for (int i = 0; i < RATE_ITERS; i++) {
#pragma unroll
      for (int j = 0; j < RATE_CH; j++)
        asm volatile("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(acc[j]) : "v"(a[j]), "v"(b));
    }
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) r ^= acc[j];
  } else if constexpr (KIND == HK_RATE_MFMA_I8) {
    // the matrix-core update's instruction: 32 x 32 x 32 int8 products into
    // int32, four independent accumulators per wave
    typedef int v16 __attribute__((ext_vector_type(16)));
    typedef int v4 __attribute__((ext_vector_type(4)));
    v16 c0 = {0}, c1 = {0}, c2 = {0}, c3 = {0};
    const v4 a = {(int)m, (int)(m * 3u), (int)(m * 5u), (int)(m * 7u)};
    const v4 b = {(int)(m ^ 1u), (int)(m ^ 2u), (int)(m ^ 3u), (int)(m ^ 4u)};
    for (int i = 0; i < RATE_ITERS / 16; i++) {
      c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, b, c3, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; v++) r ^= (int64_t)(c0[v] ^ c1[v] ^ c2[v] ^ c3[v]);
  } else {
    // HK_RATE_FMA_F64: the double-precision FMA, for comparison
    double acc[RATE_CH];
    double a[RATE_CH];
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) { acc[j] = j; a[j] = 1.0 + 1e-9 * (double)((m + j) & 1023); }
    const double b = 0.999999;
    for (int i = 0; i < RATE_ITERS; i++) {
#pragma unroll
      for (int j = 0; j < RATE_CH; j++) acc[j] = fma(a[j], b, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < RATE_CH; j++) r ^= (int64_t)acc[j];
  }
  out[tid] = r;
  if ((threadIdx.x & 63) == 0) {
    const int w = tid >> 6;
    clk[2 * w] = (int64_t)(clock64() - c0);
    clk[2 * w + 1] = (int64_t)(wall_clock64() - w0);
  }
}

struct RateShape { int blocks; int64_t threads, waves; };

RateShape rate_shape(int cus) {
  RateShape r;
  r.blocks = cus * 4 * RATE_WAVES_PER_SIMD / 4;   // 256-lane workgroups
  r.threads = (int64_t)r.blocks * 256;
  r.waves = r.threads / 64;
  return r;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" {

size_t hk_mul_rate_buffer_bytes(void) {
  const int cus = device_cus();
  if (cus <= 0) return 0;
  const RateShape r = rate_shape(cus);
  return sizeof(int64_t) * (size_t)(r.threads + 2 * r.waves);
}

hk_status hk_mul_rate(int kind, void* dev_buf, size_t buf_bytes, hipStream_t s, double* per_s, double* clock_hz) {
  if (!per_s || kind < HK_RATE_MAD_I64_I32 || kind > HK_RATE_MFMA_I8) {
    g_err = "bad arguments";
    return HK_EINVAL;
  }
  const int cus = device_cus();
  const size_t need = hk_mul_rate_buffer_bytes();
  if (cus <= 0 || need == 0) { g_err = "no device"; return HK_EDEVICE; }
  if (!dev_buf || buf_bytes < need) { g_err = "buffer too small: need " + std::to_string(need); return HK_EINVAL; }
  const RateShape r = rate_shape(cus);
  int64_t* out = (int64_t*)dev_buf;
  int64_t* clk = out + r.threads;
  auto launch = [&]() {
    switch (kind) {
      case HK_RATE_MAD_I64_I32:
        hipLaunchKernelGGL(k_rate<HK_RATE_MAD_I64_I32>, dim3(r.blocks), dim3(256), 0, s, out, clk, 7u); break;
      case HK_RATE_MAD_U64_U32:
        hipLaunchKernelGGL(k_rate<HK_RATE_MAD_U64_U32>, dim3(r.blocks), dim3(256), 0, s, out, clk, 7u); break;
      case HK_RATE_MAD_U32_U24:
        hipLaunchKernelGGL(k_rate<HK_RATE_MAD_U32_U24>, dim3(r.blocks), dim3(256), 0, s, out, clk, 7u); break;
      case HK_RATE_MFMA_I8:
        hipLaunchKernelGGL(k_rate<HK_RATE_MFMA_I8>, dim3(r.blocks), dim3(256), 0, s, out, clk, 7u); break;
      default:
        hipLaunchKernelGGL(k_rate<HK_RATE_FMA_F64>, dim3(r.blocks), dim3(256), 0, s, out, clk, 7u); break;
    }
    return hipGetLastError();
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();                       // warm-up (clock ramp, code load)
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  std::vector<int64_t> c((size_t)2 * r.waves);
  if (e == hipSuccess) e = hipMemcpyAsync(c.data(), clk, sizeof(int64_t) * c.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) { g_err = hipGetErrorString(e); return HK_EDEVICE; }
  // per lane: RATE_CH chains of RATE_ITERS steps, or (matrix products) four
  // chains of RATE_ITERS / 16 products of 32 x 32 x 32 multiply-adds a wave
  const double per_lane = kind == HK_RATE_MFMA_I8 ? 4.0 * (RATE_ITERS / 16) * 32768.0 / 64.0
                                                  : (double)RATE_CH * (double)RATE_ITERS;
  *per_s = (double)r.threads * per_lane / (1e-3 * (double)ms);
  if (clock_hz) {
    int dev = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
      wall_khz = 0;
    double cyc = 0, wall = 0;
    for (int64_t w = 0; w < r.waves; w++) { cyc += (double)c[2 * w]; wall += (double)c[2 * w + 1]; }
    *clock_hz = wall > 0 ? 1e3 * (double)wall_khz * cyc / wall : 0;
  }
  return HK_OK;
}

}  // extern "C"
