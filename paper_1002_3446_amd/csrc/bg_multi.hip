// Multi-class generation in one persistent launch (mixed multiplicities n = 4..12).
//
// The host builds a tile list (class, first event, count), ordered by decreasing n so the
// most expensive tiles start first, with each class's tiles contiguous.  Every workgroup
// takes tiles from a global counter until the list is exhausted (every wave reaches that
// exit), evaluates each event with the same per-multiplicity code as the single-class
// kernel, and writes one compensated (sum w, sum w^2) partial per tile.  A second kernel
// reduces each class's tile partials in tile order into that class's accumulator, so
// per-event outputs and totals do not depend on which workgroup ran which tile.
//
// Built for FP32 recursion (the mixed-multiplicity workload); FP64 classes of a
// multi-class call are launched one class at a time by the host layer.
#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

using Real = float;

namespace {

template <typename T>
__device__ __forceinline__ double generate_any(int n, const GenClass& C, int64_t e, PermLds perm) {
  switch (n) {
    case 4: return generate_one<4, T>(C, e, perm);
    case 5: return generate_one<5, T>(C, e, perm);
    case 6: return generate_one<6, T>(C, e, perm);
    case 7: return generate_one<7, T>(C, e, perm);
    case 8: return generate_one<8, T>(C, e, perm);
    case 9: return generate_one<9, T>(C, e, perm);
    case 10: return generate_one<10, T>(C, e, perm);
    case 11: return generate_one<11, T>(C, e, perm);
    default: return generate_one<12, T>(C, e, perm);
  }
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_generate_multi(
    const MultiClass* __restrict__ classes, const Tile* __restrict__ tiles, int ntiles, int* counter,
    double* partials) {
  __shared__ int s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
    __syncthreads();
    // uniform across the workgroup: class parameters are read with scalar loads
    const int t = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();
    if (t >= ntiles) break;
    const Tile tl = tiles[t];
    const MultiClass& mc = classes[tl.cls];
    CSum w{0.0, 0.0}, w2{0.0, 0.0};
    for (int64_t i = tl.first + threadIdx.x; i < tl.first + tl.count; i += blockDim.x) {
      const double x = generate_any<T>(mc.n, mc.C, i, dyn_perm());
      w = cs_add(w, CSum{x, 0.0});
      w2 = cs_add(w2, CSum{x * x, 0.0});
    }
    block_reduce_store(w, w2, partials + 4 * (int64_t)t);
    __syncthreads();
  }
}

// one workgroup per class: that class's tile partials, in tile order, into its accumulator
__global__ __launch_bounds__(256) void k_finalize_multi(const MultiClass* __restrict__ classes,
                                                        const double* __restrict__ partials) {
  const MultiClass& mc = classes[blockIdx.x];
  if (!mc.acc || mc.tile_end <= mc.tile_begin) return;
  CSum a{0.0, 0.0}, b{0.0, 0.0};
  for (int p = mc.tile_begin + (int)threadIdx.x; p < mc.tile_end; p += blockDim.x) {
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
    double* acc = mc.acc;
    CSum ta{acc[0], acc[1]}, tb{acc[2], acc[3]};
    for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
      ta = cs_add(ta, CSum{red[v][0], red[v][1]});
      tb = cs_add(tb, CSum{red[v][2], red[v][3]});
    }
    acc[0] = ta.s; acc[1] = ta.c; acc[2] = tb.s; acc[3] = tb.c;
  }
}

}  // namespace

hipError_t launch_generate_multi_p32(const MultiClass* classes, int nclasses, const Tile* tiles, int ntiles,
                                  int* counter, double* partials, int grid, int block, hipStream_t s) {
  // dynamic LDS: the momentum permutation column of the largest multiplicity
  hipLaunchKernelGGL((k_generate_multi<Real>), dim3(grid), dim3(block), perm_lds_bytes(12, block), s, classes, tiles,
                     ntiles, counter,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_multi, dim3(nclasses), dim3(256), 0, s, classes, partials);
  return hipGetLastError();
}

}  // namespace bgk
