// Multi-class generation (mixed multiplicities n = 4..12, FP32 recursion) in one persistent
// launch.
//
// The table classes (n <= 8) first run their kinematics in one multi-class kernel at several
// waves per SIMD (the same per-event body as the single-class k_kin), which stages every
// event of those classes.  Then one persistent kernel of one-wave workgroups takes tiles
// from a shared queue ordered by decreasing n, so that the expensive large-n tiles start
// first and the cheap staged tiles fill in behind them: a tile of a class with n >= 9 is
// generated start to finish with two lanes per event (the single-class two-lane body), a
// tile of a staged class is finished with one lane per event and the LDS span table (the
// single-class k_rec body).  Every wave reaches the queue's end, where the loop exits.  One
// compensated partial per tile; a last kernel reduces each class's partials in tile order.
// Per-event values are therefore bitwise those of the single-class launches.
#include "bg_kernels.hpp"
#include "bg_launch.hpp"
#include "bg_split.hpp"

namespace bgk {

namespace {

// the class of kinematics workgroup b (staged classes hold consecutive workgroup ranges)
__device__ __forceinline__ int kin_class(const MultiClass* __restrict__ classes, int nstaged, int64_t b) {
  int c = 0;
  for (int k = 1; k < nstaged; ++k) c = b >= classes[k].kin_begin ? k : c;
  return c;
}

// Launch: kKinBlock threads, perm_lds_bytes(8, kKinBlock) bytes of dynamic LDS, one
// workgroup per kKinBlock events of each staged class; classes[0 .. nstaged-1] are the
// staged ones, in workgroup order.
__global__ __launch_bounds__(kKinBlock) void k_kin_multi(const MultiClass* __restrict__ classes, int nstaged,
                                                         double* __restrict__ stage) {
  const int c = __builtin_amdgcn_readfirstlane(kin_class(classes, nstaged, blockIdx.x));
  const MultiClass& mc = classes[c];
  const int64_t j = ((int64_t)blockIdx.x - mc.kin_begin) * kKinBlock + threadIdx.x;
  if (j >= mc.C.count) return;
  double* buf = stage + mc.stage_off;
  switch (mc.n) {
    case 4: kin_one<4>(mc.C, j, j, buf, dyn_perm()); break;
    case 5: kin_one<5>(mc.C, j, j, buf, dyn_perm()); break;
    case 6: kin_one<6>(mc.C, j, j, buf, dyn_perm()); break;
    case 7: kin_one<7>(mc.C, j, j, buf, dyn_perm()); break;
    default: kin_one<8>(mc.C, j, j, buf, dyn_perm()); break;
  }
}

// The next tile of the queue for the whole (one-wave) workgroup.
__device__ __forceinline__ int next_tile(int* counter, int* s_tile) {
  if (threadIdx.x == 0) *s_tile = atomicAdd(counter, 1);
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(*s_tile);
  __syncthreads();
  return t;
}

// The per-multiplicity bodies are separate functions (not inlined into the kernel): each is
// register-allocated on its own, which keeps the kernel's compile time near the sum of the
// single-class kernels' instead of growing with the square of the whole body.  A call saves
// and restores the registers the calling convention assigns to the callee, so each function
// runs a whole run of tiles of its multiplicity (the queue is ordered by n, so a wave calls
// each at most once) and returns the first tile of another multiplicity, or one past the end.
template <int N>
__device__ __attribute__((noinline)) int staged_run(const MultiClass* __restrict__ classes,
                                                    const Tile* __restrict__ tiles, int ntiles, int* counter,
                                                    int* s_tile, int t, const double* __restrict__ stage, void* lds,
                                                    double* partials) {
  while (t < ntiles) {
    const Tile tl = tiles[t];
    const MultiClass& mc = classes[tl.cls];
    if (mc.n != N) return t;
    const double* buf = stage + mc.stage_off;  // slot = the class's local event index
    CSum w{0.0, 0.0}, w2{0.0, 0.0};
    for (int64_t i = tl.first + threadIdx.x; i < tl.first + tl.count; i += kMultiBlock) {
      const double x = rec_one<N>(mc.C, i, i, buf, reinterpret_cast<LdsTable<N>*>(lds));
      w = cs_add(w, CSum{x, 0.0});
      w2 = cs_add(w2, CSum{x * x, 0.0});
    }
    block_reduce_store(w, w2, partials + 4 * (int64_t)t);
    __syncthreads();
    t = next_tile(counter, s_tile);
  }
  return t;
}

template <int N>
__device__ __attribute__((noinline)) int paired_run(const MultiClass* __restrict__ classes,
                                                    const Tile* __restrict__ tiles, int ntiles, int* counter,
                                                    int* s_tile, int t, double* partials) {
  const int g = (int)(threadIdx.x & 1u);
  while (t < ntiles) {
    const Tile tl = tiles[t];
    const MultiClass& mc = classes[tl.cls];
    if (mc.n != N) return t;
    CSum w{0.0, 0.0}, w2{0.0, 0.0};
    for (int64_t i = tl.first + (threadIdx.x >> 1); i < tl.first + tl.count; i += kMultiBlock / 2) {
      const double x = generate_one<N, float, 2>(mc.C, i, PermLds{nullptr, 0}, g);
      w = cs_add(w, CSum{x, 0.0});
      w2 = cs_add(w2, CSum{x * x, 0.0});
    }
    block_reduce_store(w, w2, partials + 4 * (int64_t)t);
    __syncthreads();
    t = next_tile(counter, s_tile);
  }
  return t;
}

__global__ __launch_bounds__(kMultiBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_generate_multi(
    const MultiClass* __restrict__ classes, const Tile* __restrict__ tiles, int ntiles, int* counter,
    const double* __restrict__ stage, double* partials) {
  __shared__ LdsTable<8> lds;  // the span table of the staged classes (n <= 8 fits n = 8's)
  __shared__ int s_tile;
  int t = next_tile(counter, &s_tile);
  while (t < ntiles) {
    switch (classes[tiles[t].cls].n) {
      case 4: t = staged_run<4>(classes, tiles, ntiles, counter, &s_tile, t, stage, &lds, partials); break;
      case 5: t = staged_run<5>(classes, tiles, ntiles, counter, &s_tile, t, stage, &lds, partials); break;
      case 6: t = staged_run<6>(classes, tiles, ntiles, counter, &s_tile, t, stage, &lds, partials); break;
      case 7: t = staged_run<7>(classes, tiles, ntiles, counter, &s_tile, t, stage, &lds, partials); break;
      case 8: t = staged_run<8>(classes, tiles, ntiles, counter, &s_tile, t, stage, &lds, partials); break;
      case 9: t = paired_run<9>(classes, tiles, ntiles, counter, &s_tile, t, partials); break;
      case 10: t = paired_run<10>(classes, tiles, ntiles, counter, &s_tile, t, partials); break;
      case 11: t = paired_run<11>(classes, tiles, ntiles, counter, &s_tile, t, partials); break;
      default: t = paired_run<12>(classes, tiles, ntiles, counter, &s_tile, t, partials); break;
    }
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

hipError_t launch_generate_multi_p32(const MultiClass* classes, int nclasses, int nstaged, int64_t kin_blocks,
                                     const Tile* tiles, int ntiles, int* counter, double* stage, double* partials,
                                     int grid, hipStream_t s) {
  if (nstaged > 0 && kin_blocks > 0) {
    hipLaunchKernelGGL(k_kin_multi, dim3((unsigned)kin_blocks), dim3(kKinBlock), perm_lds_bytes(8, kKinBlock), s,
                       classes, nstaged, stage);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_generate_multi, dim3(grid), dim3(kMultiBlock), 0, s, classes, tiles, ntiles, counter, stage,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_multi, dim3(nclasses), dim3(256), 0, s, classes, partials);
  return hipGetLastError();
}

}  // namespace bgk
