// The fixed-order two-level reduction of per-workgroup partials (shared by every class).
#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

// Compensated sum of the partials [first, first + count) into (a, b) of thread 0 of the
// workgroup: lane t takes parts t, t + 256, ... in order, then a fixed butterfly and a
// fixed pass over the four waves.
__device__ __forceinline__ void group_sum(const double* __restrict__ partials, int64_t first, int64_t count, CSum& a,
                                          CSum& b) {
  a = CSum{0.0, 0.0};
  b = CSum{0.0, 0.0};
  for (int64_t p = first + threadIdx.x; p < first + count; p += blockDim.x) {
    a = cs_add(a, CSum{partials[4 * p], partials[4 * p + 1]});
    b = cs_add(b, CSum{partials[4 * p + 2], partials[4 * p + 3]});
  }
  __shared__ double red[4][4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    CSum oa{__shfl_down(a.s, off), __shfl_down(a.c, off)};
    CSum ob{__shfl_down(b.s, off), __shfl_down(b.c, off)};
    a = cs_add(a, oa);
    b = cs_add(b, ob);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = a.s; red[wave][1] = a.c; red[wave][2] = b.s; red[wave][3] = b.c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = CSum{red[0][0], red[0][1]};
    b = CSum{red[0][2], red[0][3]};
    for (int v = 1; v < 4; ++v) {
      a = cs_add(a, CSum{red[v][0], red[v][1]});
      b = cs_add(b, CSum{red[v][2], red[v][3]});
    }
  }
}

// Level 1: workgroup g reduces the g-th contiguous run of `per` partials.
__global__ __launch_bounds__(256) void k_finalize_runs(const double* __restrict__ partials, int64_t nparts, int64_t per,
                                                        double* level2) {
  const int64_t first = (int64_t)blockIdx.x * per;
  CSum a, b;
  group_sum(partials, first, first + per < nparts ? per : nparts - first, a, b);
  if (threadIdx.x == 0) {
    double* d = level2 + 4 * (int64_t)blockIdx.x;
    d[0] = a.s; d[1] = a.c; d[2] = b.s; d[3] = b.c;
  }
}

// Level 2 (one workgroup): the run results, in run order, are added to acc.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ level2, int64_t nruns, double* acc) {
  CSum a, b;
  group_sum(level2, 0, nruns, a, b);
  if (threadIdx.x == 0) {
    CSum ta{acc[0], acc[1]}, tb{acc[2], acc[3]};
    ta = cs_add(ta, a);
    tb = cs_add(tb, b);
    acc[0] = ta.s; acc[1] = ta.c; acc[2] = tb.s; acc[3] = tb.c;
  }
}

hipError_t launch_finalize(const double* partials, int64_t nparts, double* level2, double* acc, hipStream_t s) {
  if (nparts <= 0) return hipSuccess;
  // runs of at least 256 partials, at most kFinalizeGroups runs
  int64_t per = (nparts + kFinalizeGroups - 1) / kFinalizeGroups;
  if (per < 256) per = 256;
  const int64_t nruns = (nparts + per - 1) / per;
  hipLaunchKernelGGL(k_finalize_runs, dim3((unsigned)nruns), dim3(256), 0, s, partials, nparts, per, level2);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, level2, nruns, acc);
  return hipGetLastError();
}

}  // namespace bgk
