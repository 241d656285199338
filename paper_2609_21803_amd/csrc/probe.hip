// probe.hip -- microbenchmarks of the device's peak rates, for the denominators of the
// roofline figures: FP32 and FP64 vector FMA (non-packed: packed FP32 is disabled at compile
// time throughout this library), BF16 matrix-core products (v_mfma_f32_16x16x32_bf16), and
// a device-to-device copy through HBM.  Each arithmetic kernel runs independent dependency
// chains in registers for a fixed number of iterations and writes one value per thread so
// the work cannot be removed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "internal.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short pb_bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float pb_f32x4;

constexpr int PROBE_CHAINS = 16;   // independent FMA chains per lane
constexpr int PROBE_ACC = 8;       // independent matrix-core accumulators per wave

__global__ __launch_bounds__(256) void k_probe_fma32(float* out, int iters) {
  float a[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = 1e-3f * (threadIdx.x + c);
  const float b = 0.999999f, d = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = fmaf(a[c], b, d);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += a[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_fma64(double* out, int iters) {
  double a[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = 1e-3 * (threadIdx.x + c);
  const double b = 0.999999, d = 1e-7;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = fma(a[c], b, d);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += a[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// PROBE_ACC independent accumulators per wave; operands stay in registers
__global__ __launch_bounds__(256) void k_probe_mfma_bf16(float* out, int iters) {
  pb_bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (short)(0x3f80 + ((threadIdx.x + i) & 7));   // BF16 values near 1
    b[i] = (short)(0x3f80 - ((threadIdx.x + 2 * i) & 7));
  }
  pb_f32x4 acc[PROBE_ACC];
#pragma unroll
  for (int c = 0; c < PROBE_ACC; ++c) acc[c] = pb_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < PROBE_ACC; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_ACC; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// grid-stride copy in 16-byte vectors
__global__ __launch_bounds__(256) void k_probe_copy(const pb_f32x4* __restrict__ src, pb_f32x4* __restrict__ dst,
                                                   long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// one warm-up launch, then one launch between events; a negative time reports a failure
template <typename F>
float time_ms(hipStream_t s, hipEvent_t e0, hipEvent_t e1, F launch) {
  launch();
  if (hipGetLastError() != hipSuccess) return -1.f;
  if (hipEventRecord(e0, s) != hipSuccess) return -1.f;
  launch();
  if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return -1.f;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) return -1.f;
  return ms;
}

}  // namespace

extern "C" comet_status comet_probe_peaks(void* stream, double* out) {
  if (!out) return comet::fail_global(COMET_EINVAL, "null output pointer");
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();   // an error left by earlier, unrelated calls is not this probe's
  int dev = 0;
  hipDeviceProp_t prop;
  const hipError_t e_dev = hipGetDevice(&dev);
  const hipError_t e_prop = (e_dev == hipSuccess) ? hipGetDeviceProperties(&prop, dev) : e_dev;
  if (e_dev != hipSuccess || e_prop != hipSuccess || prop.multiProcessorCount < 1)
    return comet::fail_global(COMET_EHIP, std::string("device query failed: ") + hipGetErrorString(e_prop));
  const int n_cu = prop.multiProcessorCount;
  const int blocks = n_cu * 16, threads = 256, iters = 4096;
  const long long n_threads = (long long)blocks * threads;
  const long long copy_bytes = 1ll << 30;
  void *res = nullptr, *src = nullptr, *dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  comet_status st = COMET_OK;
  const char* what = "";
  if (hipMalloc(&res, sizeof(double) * n_threads) != hipSuccess || hipMalloc(&src, copy_bytes) != hipSuccess ||
      hipMalloc(&dst, copy_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = COMET_ENOMEM;
    what = "scratch allocation failed";
  } else if (hipMemsetAsync(src, 0, copy_bytes, s) != hipSuccess) {
    st = COMET_EHIP;
    what = "clearing the copy source failed";
  } else {
    const double fma_flop = 2.0 * PROBE_CHAINS * (double)iters * (double)n_threads;
    float ms = time_ms(s, e0, e1, [&] {
      hipLaunchKernelGGL(k_probe_fma32, dim3(blocks), dim3(threads), 0, s, (float*)res, iters);
    });
    out[0] = fma_flop / (ms * 1e-3) / 1e12;
    ms = time_ms(s, e0, e1, [&] {
      hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(threads), 0, s, (double*)res, iters);
    });
    out[1] = fma_flop / (ms * 1e-3) / 1e12;
    const int mfma_iters = 2048;
    ms = time_ms(s, e0, e1, [&] {
      hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(blocks), dim3(threads), 0, s, (float*)res, mfma_iters);
    });
    // one 16x16x32 product per wave and accumulator: 2 * 16 * 16 * 32 flop
    out[2] = 2.0 * 16 * 16 * 32 * PROBE_ACC * (double)mfma_iters * (double)(n_threads / 64) / (ms * 1e-3) / 1e12;
    const long long nv = copy_bytes / 16;
    ms = time_ms(s, e0, e1, [&] {
      hipLaunchKernelGGL(k_probe_copy, dim3(n_cu * 32), dim3(threads), 0, s, (const pb_f32x4*)src, (pb_f32x4*)dst, nv);
    });
    out[3] = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;   // read + write, GB/s
    static const char* names[4] = {"FP32 probe failed", "FP64 probe failed", "matrix-core probe failed",
                                   "copy probe failed"};
    for (int i = 3; i >= 0; --i)
      if (!(out[i] > 0.0)) {
        st = COMET_EHIP;
        what = names[i];
      }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (res) (void)hipFree(res);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  return st == COMET_OK ? st : comet::fail_global(st, what);
}
