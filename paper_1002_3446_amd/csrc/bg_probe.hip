// Calibration of the roofline denominators: the VALU multiply-add rate this GPU sustains
// (bg_fma_rate), measured with chains of fused multiply-adds that have no other work and no
// memory traffic: every lane runs 16 independent accumulator chains (enough to cover the
// FMA latency at one wave per SIMD) for `iters` rounds, at eight waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bg_launch.hpp"

namespace bgk {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fma_chains(T a, T b, int iters, T* out) {
  T acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = a + T(j) * T(1e-3) + T(threadIdx.x) * T(1e-7);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = __builtin_fma(acc[j], b, a);
  }
  T s = acc[0];
#pragma unroll
  for (int j = 1; j < 16; ++j) s += acc[j];
  if (s == T(12345.678)) out[0] = s;  // keeps the chains live; never true for these inputs
}

template <>
__global__ __launch_bounds__(256) void k_fma_chains<float>(float a, float b, int iters, float* out) {
  float acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = a + float(j) * 1e-3f + float(threadIdx.x) * 1e-7f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = __builtin_fmaf(acc[j], b, a);
  }
  float s = acc[0];
#pragma unroll
  for (int j = 1; j < 16; ++j) s += acc[j];
  if (s == 12345.678f) out[0] = s;
}

}  // namespace

hipError_t measure_fma_rate(int prec, int iters, int ncu, double* flops_per_s, hipStream_t s) {
  const int blocks = ncu * 8;  // 256-lane workgroups: eight waves per SIMD
  void* out = nullptr;
  hipError_t e = hipMallocAsync(&out, 64, s);
  if (e != hipSuccess) return e;
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    hipEventDestroy(t0);
    return e;
  }
  float ms = 0.0f;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
    hipEventRecord(t0, s);
    if (prec == 32)
      hipLaunchKernelGGL(k_fma_chains<float>, dim3(blocks), dim3(256), 0, s, 1.0f, 0.999999f, iters, (float*)out);
    else
      hipLaunchKernelGGL(k_fma_chains<double>, dim3(blocks), dim3(256), 0, s, 1.0, 0.999999, iters, (double*)out);
    e = hipGetLastError();
    hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  }
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  hipFreeAsync(out, s);
  if (e != hipSuccess) return e;
  const double flops = 2.0 * 16.0 * (double)iters * (double)blocks * 256.0;
  *flops_per_s = ms > 0.0f ? flops / (ms * 1e-3) : 0.0;
  return hipSuccess;
}

}  // namespace bgk
