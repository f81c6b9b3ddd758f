// Machine probes (rtcc_peak_probe): the sustained rate of the three MFMA instructions the contractions
// use, and the HBM bandwidth of a plain device copy, measured on the device the caller has current. They
// give the measured ceilings the kernels' roofline fractions can be read against, beside the datasheet
// figures.
//
// MFMA: every wave keeps eight (BF16, FP64) or sixteen (FP32) independent accumulator chains busy for `size`
// rounds, enough to cover each instruction's latency (measured: fewer chains give less; no memory traffic
// inside the loop; operands are lane-dependent values the compiler cannot fold) over a grid of 4096
// workgroups of 256 threads (64 waves per CU); flops = 2 M N K per instruction. Copy: 16-byte loads and
// stores (four loads in flight per thread) over two buffers of `size` bytes each; GB/s counts the bytes
// read plus the bytes written.
#include <algorithm>
#include <cstdint>

#include "../../include/rtcc.h"
#include "common.h"

using namespace rtcc;

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kBlocks = 4096, kThreads = 256;

// v_mfma_f32_32x32x16_bf16: 32 x 32 x 16, eight chains
__global__ __launch_bounds__(kThreads) void mfma_bf16_loop(int iters, float* out) {
  const int l = threadIdx.x;
  bf8 a, b;
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1e-3f * (float)((l + j) & 7));
    b[j] = (__bf16)(1e-3f * (float)((l * 3 + j) & 7));
  }
  f16v c[8];
  for (int q = 0; q < 8; ++q)
    for (int e = 0; e < 16; ++e) c[q][e] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[q], 0, 0, 0);
  }
  float s = 0.f;
  for (int q = 0; q < 8; ++q)
    for (int e = 0; e < 16; ++e) s += c[q][e];
  out[blockIdx.x * kThreads + l] = s;
}

// v_mfma_f32_16x16x4f32: 16 x 16 x 4, sixteen chains
__global__ __launch_bounds__(kThreads) void mfma_f32_loop(int iters, float* out) {
  const int l = threadIdx.x;
  const float a = 1e-3f * (float)(l & 7), b = 1e-3f * (float)((l * 3) & 7);
  f4v c[16];
  for (int q = 0; q < 16; ++q)
    for (int e = 0; e < 4; ++e) c[q][e] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[q], 0, 0, 0);
  }
  float s = 0.f;
  for (int q = 0; q < 16; ++q)
    for (int e = 0; e < 4; ++e) s += c[q][e];
  out[blockIdx.x * kThreads + l] = s;
}

// v_mfma_f64_16x16x4f64: 16 x 16 x 4, eight chains
__global__ __launch_bounds__(kThreads) void mfma_f64_loop(int iters, float* out) {
  const int l = threadIdx.x;
  const double a = 1e-3 * (double)(l & 7), b = 1e-3 * (double)((l * 3) & 7);
  d4v c[8];
  for (int q = 0; q < 8; ++q)
    for (int e = 0; e < 4; ++e) c[q][e] = 0.0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
  }
  double s = 0.0;
  for (int q = 0; q < 8; ++q)
    for (int e = 0; e < 4; ++e) s += c[q][e];
  out[blockIdx.x * kThreads + l] = (float)s;
}

// four 16-byte loads in flight per thread before its stores; n a multiple of 4 * 256
__global__ __launch_bounds__(256) void copy16(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 1024) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + 256 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[i + 256 * u] = v[u];
  }
}

// Average duration (ms) of `reps` launches issued by `launch` on `st`, after one untimed launch.
template <typename F>
double time_ms(hipStream_t st, int reps, F launch) {
  hipEvent_t e0, e1;
  RTCC_HIP(hipEventCreate(&e0));
  RTCC_HIP(hipEventCreate(&e1));
  launch();
  RTCC_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) launch();
  RTCC_HIP(hipEventRecord(e1, st));
  RTCC_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  RTCC_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

}  // namespace

extern "C" int rtcc_peak_probe(int kind, int64_t size, double* value) {
  if (kind < 0 || kind > 3 || size < 1 || !value) {
    set_noctx_error("rtcc_peak_probe: invalid arguments");
    return RTCC_EINVAL;
  }
  float* out = nullptr;
  void* a = nullptr;
  void* b = nullptr;
  hipStream_t st = nullptr;
  int rc = RTCC_OK;
  try {
    RTCC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    if (kind < 3) {
      RTCC_CHECK(size <= (1 << 24), kEInval, "rtcc_peak_probe: at most 2^24 rounds");
      const int iters = (int)size;
      RTCC_HIP(hipMalloc(&out, (size_t)kBlocks * kThreads * sizeof(float)));
      const double waves = (double)kBlocks * kThreads / 64;
      double ms = 0.0, flops = 0.0;
      if (kind == 2) {
        ms = time_ms(st, 3, [&] { hipLaunchKernelGGL(mfma_bf16_loop, dim3(kBlocks), dim3(kThreads), 0, st, iters, out); });
        flops = waves * iters * 8 * (2.0 * 32 * 32 * 16);
      } else if (kind == 1) {
        ms = time_ms(st, 3, [&] { hipLaunchKernelGGL(mfma_f32_loop, dim3(kBlocks), dim3(kThreads), 0, st, iters, out); });
        flops = waves * iters * 16 * (2.0 * 16 * 16 * 4);
      } else {
        ms = time_ms(st, 3, [&] { hipLaunchKernelGGL(mfma_f64_loop, dim3(kBlocks), dim3(kThreads), 0, st, iters, out); });
        flops = waves * iters * 8 * (2.0 * 16 * 16 * 4);
      }
      RTCC_HIP(hipGetLastError());
      *value = flops / (ms * 1e-3) / 1e12;
    } else {
      RTCC_CHECK(size % 16384 == 0 && size <= ((int64_t)1 << 36), kEInval,
                 "rtcc_peak_probe: copy size must be a multiple of 16 KiB, at most 64 GiB");
      RTCC_HIP(hipMalloc(&a, (size_t)size));
      RTCC_HIP(hipMalloc(&b, (size_t)size));
      RTCC_HIP(hipMemsetAsync(a, 0, (size_t)size, st));
      const int64_t n = size / 16;
      const double ms = time_ms(st, 5, [&] {
        hipLaunchKernelGGL(copy16, dim3((unsigned)std::min<int64_t>(n / 1024, 32768)), dim3(256), 0, st,
                           (const float4*)a, (float4*)b, n);
      });
      RTCC_HIP(hipGetLastError());
      *value = 2.0 * (double)size / (ms * 1e-3) / 1e9;
    }
    RTCC_HIP(hipStreamSynchronize(st));
  } catch (const Error& e) {
    set_noctx_error(e.what());
    rc = e.code;
  } catch (const std::exception& e) {
    set_noctx_error(e.what());
    rc = RTCC_EHIP;
  }
  if (st) (void)hipStreamSynchronize(st);
  if (out) (void)hipFree(out);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (st) (void)hipStreamDestroy(st);
  return rc;
}
