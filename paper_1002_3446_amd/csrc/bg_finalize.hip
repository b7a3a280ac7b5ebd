// The fixed-order reduction of per-workgroup partials (shared by every class).
#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

// Fixed-order compensated reduction of per-workgroup partials into acc[4] (one workgroup
// of 256 lanes): lane t takes parts t, t+256, ...; then the workgroup tree.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int64_t nparts, double* acc) {
  CSum a{0.0, 0.0}, b{0.0, 0.0};
  for (int64_t p = threadIdx.x; p < nparts; p += blockDim.x) {
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
    CSum ta{acc[0], acc[1]}, tb{acc[2], acc[3]};
    for (int v = 0; v < 4; ++v) {
      ta = cs_add(ta, CSum{red[v][0], red[v][1]});
      tb = cs_add(tb, CSum{red[v][2], red[v][3]});
    }
    acc[0] = ta.s; acc[1] = ta.c; acc[2] = tb.s; acc[3] = tb.c;
  }
}


hipError_t launch_finalize(const double* partials, int64_t nparts, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nparts, acc);
  return hipGetLastError();
}
}  // namespace bgk
