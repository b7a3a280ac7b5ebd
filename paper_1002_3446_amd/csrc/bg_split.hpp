// The single-class generation of a table-recursion class (FP32, n <= 8) as two kernels:
// k_kin evaluates the kinematics (draws, parton fractions, RAMBO, boost, cuts) at several
// waves per SIMD, which hides the latency of its long FP64 chains, and hands each event's
// centre-of-mass momenta, s_hat, x1, x2, helicity word, cut flag and leg positions to
// k_rec through a stream-ordered staging buffer; k_rec evaluates |A|^2 at the recursion's
// register budget (one wave per SIMD), the weight and the workgroup partials.  Every value
// comes from the same device functions as in the fused kernel, and the partials have the
// fused kernel's workgroups (64 events each), so totals are formed in the same order.
#pragma once

#include <algorithm>

#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

// Staging layout: events in tiles of 64 (one wave), each tile holding its words one after
// another, word w of event j at buf[((j / 64) * kWords + w) * 64 + j % 64], so that a wave
// reads one contiguous block.  Words: 4N momenta (position t, component mu at 4 t + mu),
// s_hat, x1, x2, the helicity word with the cut flag at bit 32, and the leg positions
// (4 bits each).
template <int N>
struct SplitLayout {
  static constexpr int kMom = 0, kShat = 4 * N, kX1 = 4 * N + 1, kX2 = 4 * N + 2, kMeta = 4 * N + 3,
                       kLegs = 4 * N + 4, kWords = 4 * N + 5;
  __device__ static int64_t at(int64_t j, int w) { return ((j >> 6) * kWords + w) * 64 + (j & 63); }
};

// Launch: blockDim.x in {64, 128, 256}, perm_lds_bytes(N, blockDim.x) bytes of dynamic LDS,
// ceil(cnt / blockDim.x) workgroups; events first .. first + cnt - 1.
template <int N>
__global__ __launch_bounds__(256) void k_kin(GenClass C, int64_t first, int64_t cnt, int64_t cap,
                                             double* __restrict__ buf) {
  using L = SplitLayout<N>;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const int64_t i = first + j;
  const PermLds perm = dyn_perm();
  EventKin<N> ev;
  double ht, rmin;
  build_event<N>(C, i, ev, perm, true);
  const bool pass = cuts<N>(C, ev, perm, ht, rmin);
  if (C.out.pass) C.out.pass[i] = pass ? 1 : 0;
  if (C.out.obs) {
    C.out.obs[2 * i] = ht;
    C.out.obs[2 * i + 1] = rmin;
  }
#pragma unroll
  for (int t = 0; t < N; ++t)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) buf[L::at(j, L::kMom + 4 * t + mu)] = ev.pc[t][mu];
  buf[L::at(j, L::kShat)] = ev.shat;
  buf[L::at(j, L::kX1)] = ev.x1;
  buf[L::at(j, L::kX2)] = ev.x2;
  uint64_t legs = 0;
#pragma unroll
  for (int t = 0; t < N; ++t) legs |= (uint64_t)(ev.leg[t] & 15u) << (4 * t);
  buf[L::at(j, L::kMeta)] = __longlong_as_double((long long)((uint64_t)ev.hel | ((uint64_t)pass << 32)));
  buf[L::at(j, L::kLegs)] = __longlong_as_double((long long)legs);
}

// Launch: blockDim.x = kLdsLanes, ceil(cnt / kLdsLanes) workgroups, first a multiple of
// kLdsLanes; workgroup b writes the partial of the fused kernel's workgroup first / 64 + b.
template <int N, typename T>
__global__ __launch_bounds__(kLdsLanes) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rec(
    GenClass C, int64_t first, int64_t cnt, int64_t cap, const double* __restrict__ buf, double* partials) {
  using L = SplitLayout<N>;
  static_assert(UseLdsK<N, T>::value, "the split form is for the table-recursion classes");
  __shared__ LdsTable<N> tab;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  if (j < cnt) {
    const int64_t i = first + j;
    double pc[N][4];
    uint32_t leg[N];
#pragma unroll
    for (int t = 0; t < N; ++t)
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) pc[t][mu] = buf[L::at(j, L::kMom + 4 * t + mu)];
    const double shat = buf[L::at(j, L::kShat)];
    const double x1 = buf[L::at(j, L::kX1)];
    const double x2 = buf[L::at(j, L::kX2)];
    const uint64_t meta = (uint64_t)__double_as_longlong(buf[L::at(j, L::kMeta)]);
    const uint64_t legs = (uint64_t)__double_as_longlong(buf[L::at(j, L::kLegs)]);
#pragma unroll
    for (int t = 0; t < N; ++t) leg[t] = (uint32_t)(legs >> (4 * t)) & 15u;
    const uint32_t hel = (uint32_t)meta;
    const bool pass = ((meta >> 32) & 1u) != 0;
    const double a2 = ordered_amp2<N, T, true>(pc, leg, hel, &tab);
    double sp = 1.0;
#pragma unroll
    for (int k = 0; k < (N > 5 ? N - 5 : 5 - N); ++k) sp *= shat;
    if (N < 5) sp = 1.0 / sp;
    w = pass ? C.wconst * sp * a2 : 0.0;
    if (C.out.weight) C.out.weight[i] = w;
    if (C.out.amp2) C.out.amp2[i] = a2;
    if (C.out.logw) {
      double lw = log(a2) + (N - 5) * log(shat) + C.log_const;
      if (C.use_pdf) lw += C.pdf.a * (log(x1) + log(x2)) + C.pdf.b * (log1p(-x1) + log1p(-x2));
      C.out.logw[i] = a2 > 0.0 ? lw : -INFINITY;
    }
  }
  if (partials) block_reduce_store(CSum{w, 0.0}, CSum{w * w, 0.0}, partials + 4 * (first / kLdsLanes + (int64_t)blockIdx.x));
}

// Both kernels over the class in chunks of at most kSplitChunk events, through one
// stream-ordered staging buffer; returns hipErrorOutOfMemory (nothing launched) when the
// buffer cannot be allocated, so that the caller can run the fused kernel instead.
constexpr int64_t kSplitChunk = int64_t(1) << 21;
// below this many events the per-call allocation of the staging buffer costs more than the
// split saves, and the fused kernel runs
constexpr int64_t kSplitMinEvents = int64_t(1) << 20;
constexpr int kKinBlock = 128;

template <int N, typename T>
hipError_t launch_generate_split(const GenClass& C, double* partials, hipStream_t s) {
  using L = SplitLayout<N>;
  if (C.count <= 0) return hipSuccess;
  const int64_t cap = std::min<int64_t>(kSplitChunk, (C.count + kLdsLanes - 1) / kLdsLanes * kLdsLanes);
  double* buf = nullptr;
  if (hipMallocAsync((void**)&buf, (size_t)cap * L::kWords * sizeof(double), s) != hipSuccess) {
    (void)hipGetLastError();
    return hipErrorOutOfMemory;
  }
  hipError_t e = hipSuccess;
  for (int64_t first = 0; first < C.count && e == hipSuccess; first += cap) {
    const int64_t cnt = std::min<int64_t>(cap, C.count - first);
    hipLaunchKernelGGL((k_kin<N>), dim3((unsigned)((cnt + kKinBlock - 1) / kKinBlock)), dim3(kKinBlock),
                       perm_lds_bytes(N, kKinBlock), s, C, first, cnt, cap, buf);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL((k_rec<N, T>), dim3((unsigned)((cnt + kLdsLanes - 1) / kLdsLanes)), dim3(kLdsLanes), 0, s, C,
                       first, cnt, cap, buf, partials);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(buf, s);
  return e;
}

}  // namespace bgk
