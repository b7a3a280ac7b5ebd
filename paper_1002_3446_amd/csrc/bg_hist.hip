// Exact histograms of event weights over observables (bg_hist_accumulate, bg_hist_read):
// the distributions of Sec. 4 (Fig. 3) on the device.  Arithmetic in bg_hist.hpp.
#include <hip/hip_runtime.h>

#include "bg_hist.hpp"
#include "bg_launch.hpp"

namespace bgk {

namespace {

// Bin of x on an axis: 0 below lo (underflow), nbins + 1 at or above hi and for NaN
// (overflow), else 1 + floor((x - lo) / (hi - lo) nbins), rounded as written.
__device__ __forceinline__ int hist_bin(double x, const HistAxis& a) {
#pragma clang fp contract(off)
  if (x < a.lo) return 0;
  if (!(x < a.hi)) return a.nbins + 1;
  const double t = (x - a.lo) / (a.hi - a.lo) * (double)a.nbins;
  const int b = (int)t;
  return (b < a.nbins ? b : a.nbins - 1) + 1;
}

// Grid-stride over the events; every workgroup adds its events' bits to a private copy of
// the limbs in LDS (64-bit LDS atomics), then adds its non-zero limbs to the caller's.
__global__ __launch_bounds__(256) void k_hist_accumulate(int64_t N, const double* __restrict__ weight,
                                                         const double* __restrict__ obs, HistAxes A,
                                                         unsigned long long* limbs) {
  extern __shared__ unsigned long long lds_limbs[];
  const int nl = A.total_bins * 2 * kHistLimbs;
  for (int k = threadIdx.x; k < nl; k += blockDim.x) lds_limbs[k] = 0ull;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double w = weight[i];
    if (w == 0.0) continue;
    const double w2 = w * w;
    for (int a = 0; a < A.naxes; ++a) {
      const HistAxis& ax = A.axis[a];
      const int b = hist_bin(obs[2 * i + ax.column], ax);
      unsigned long long* L = lds_limbs + (size_t)(ax.first_bin + b) * 2 * kHistLimbs;
      hist_split(w, [&](int j, int64_t c) { atomicAdd(L + j, (unsigned long long)c); });
      hist_split(w2, [&](int j, int64_t c) { atomicAdd(L + kHistLimbs + j, (unsigned long long)c); });
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nl; k += blockDim.x)
    if (lds_limbs[k] != 0ull) atomicAdd(limbs + k, lds_limbs[k]);
}

// One thread per (bin, quantity): carries in place, so that every call starts from limbs in
// [0, 2^32) (a call of at most 2^30 events then cannot overflow a limb).
__global__ __launch_bounds__(256) void k_hist_normalise(int nsums, int64_t* limbs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nsums) hist_normalise(limbs + (size_t)k * kHistLimbs);
}

__global__ __launch_bounds__(256) void k_hist_read(int nsums, const int64_t* __restrict__ limbs, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsums) return;
  int64_t L[kHistLimbs];
#pragma unroll
  for (int j = 0; j < kHistLimbs; ++j) L[j] = limbs[(size_t)k * kHistLimbs + j];
  hist_normalise(L);
  out[k] = hist_limbs_to_double(L);
}

}  // namespace

hipError_t launch_hist_accumulate(int64_t N, const double* weight, const double* obs, const HistAxes& A,
                                  int64_t* limbs, int cus, hipStream_t s) {
  const size_t lds = (size_t)A.total_bins * 2 * kHistLimbs * sizeof(unsigned long long);
  const int64_t want = (N + 4095) / 4096;
  const int grid = (int)(want < 2 * cus ? (want > 0 ? want : 1) : 2 * cus);
  hipLaunchKernelGGL(k_hist_accumulate, dim3(grid), dim3(256), lds, s, N, weight, obs, A,
                     reinterpret_cast<unsigned long long*>(limbs));
  const int nsums = A.total_bins * 2;
  hipLaunchKernelGGL(k_hist_normalise, dim3((nsums + 255) / 256), dim3(256), 0, s, nsums, limbs);
  return hipGetLastError();
}

hipError_t launch_hist_read(const HistAxes& A, const int64_t* limbs, double* out, hipStream_t s) {
  const int nsums = A.total_bins * 2;
  hipLaunchKernelGGL(k_hist_read, dim3((nsums + 255) / 256), dim3(256), 0, s, nsums, limbs, out);
  return hipGetLastError();
}

}  // namespace bgk
