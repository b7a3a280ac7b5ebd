// Generation of a table-recursion class (FP32, n <= 8) as two kernels: k_kin evaluates the
// kinematics (draws, parton fractions, RAMBO, boost, cuts) at several waves per SIMD, which
// hides the latency of its long FP64 chains, and hands each event's centre-of-mass momenta,
// s_hat, x1, x2, helicity word, cut flag and leg positions to k_rec through a staging
// buffer; k_rec evaluates |A|^2 at the recursion's register budget (one wave per SIMD), the
// weight and one compensated partial per 64 events.  The per-event bodies (kin_one, rec_one)
// are also the table classes' part of the persistent multi-class kernel, so an event gives
// bitwise the same values in either launch.
#pragma once

#include <algorithm>

#include "bg_kernels.hpp"
#include "bg_launch.hpp"

namespace bgk {

// Staging layout: events in tiles of 64 (one wave), each tile holding its words one after
// another, word w of event j at buf[((j / 64) * kWords + w) * 64 + j % 64], so that a wave
// reads one contiguous block.  Words: the centre-of-mass momenta of recursion positions
// 1..N-1 (position t, component mu at 4 (t - 1) + mu; position 0 is always the beam leg 0,
// which follows from s_hat), s_hat, x1, x2, the weight factor of the dynamic scale
// (scale_ratio, 1 with a fixed scale), the helicity word with the cut flag at bit 32, and the
// leg positions (4 bits each).
template <int N>
struct SplitLayout {
  static constexpr int kMom = 0, kShat = 4 * (N - 1), kX1 = kShat + 1, kX2 = kShat + 2, kR = kShat + 3,
                       kMeta = kShat + 4, kLegs = kShat + 5, kWords = kShat + 6;
  static_assert(kWords == split_words(N), "staging words");
  __device__ static int64_t at(int64_t j, int w) { return ((j >> 6) * kWords + w) * 64 + (j & 63); }
};

// Kinematics of event i (staging slot j): writes the cut flag and observables and stages
// the event.  perm: the lane's LDS column (perm_lds_bytes).
template <int N>
__device__ __forceinline__ void kin_one(const GenClass& C, int64_t i, int64_t j, double* __restrict__ buf,
                                        PermLds perm) {
  using L = SplitLayout<N>;
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
  for (int t = 1; t < N; ++t)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) buf[L::at(j, L::kMom + 4 * (t - 1) + mu)] = ev.pc[t][mu];
  buf[L::at(j, L::kShat)] = ev.shat;
  buf[L::at(j, L::kX1)] = ev.x1;
  buf[L::at(j, L::kX2)] = ev.x2;
  buf[L::at(j, L::kR)] = scale_ratio<N>(C, ht, ev.x1, ev.x2);
  uint64_t legs = 0;
#pragma unroll
  for (int t = 0; t < N; ++t) legs |= (uint64_t)(ev.leg[t] & 15u) << (4 * t);
  buf[L::at(j, L::kMeta)] = __longlong_as_double((long long)((uint64_t)ev.hel | ((uint64_t)pass << 32)));
  buf[L::at(j, L::kLegs)] = __longlong_as_double((long long)legs);
}

// One event's staged words in registers.
template <int N>
struct Staged {
  double pc[N - 1][4];  // positions 1..N-1
  double shat, x1, x2, r;
  uint64_t meta, legs;
};

template <int N>
__device__ __forceinline__ void load_staged(const double* __restrict__ buf, int64_t j, Staged<N>& s) {
  using L = SplitLayout<N>;
#pragma unroll
  for (int t = 1; t < N; ++t)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) s.pc[t - 1][mu] = buf[L::at(j, L::kMom + 4 * (t - 1) + mu)];
  s.shat = buf[L::at(j, L::kShat)];
  s.x1 = buf[L::at(j, L::kX1)];
  s.x2 = buf[L::at(j, L::kX2)];
  s.r = buf[L::at(j, L::kR)];
  s.meta = (uint64_t)__double_as_longlong(buf[L::at(j, L::kMeta)]);
  s.legs = (uint64_t)__double_as_longlong(buf[L::at(j, L::kLegs)]);
}

// |A|^2, weight and outputs of event i from its staged words (one lane per event, the span
// table in tab); returns w.
template <int N, int POL = 0>
__device__ __forceinline__ double rec_staged(const GenClass& C, int64_t i, const Staged<N>& s, LdsTable<N>* tab) {
  double pc[N][4];
  // position 0: the beam leg 0, as build_event forms it
  const double hb = 0.5 * (C.use_pdf ? sqrt(s.shat) : C.sqrt_s);
  pc[0][0] = hb;
  pc[0][1] = 0.0;
  pc[0][2] = 0.0;
  pc[0][3] = hb;
#pragma unroll
  for (int t = 1; t < N; ++t)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) pc[t][mu] = s.pc[t - 1][mu];
  uint32_t leg[N];
#pragma unroll
  for (int t = 0; t < N; ++t) leg[t] = (uint32_t)(s.legs >> (4 * t)) & 15u;
  const uint32_t hel = (uint32_t)s.meta;
  const bool pass = ((s.meta >> 32) & 1u) != 0;
  double a2;
  if constexpr (POL == 1) {
    double cs[N][2];
    polarisation_angles<N>(C, i, cs);
    a2 = ordered_amp2_real<N, float, true>(pc, leg, cs, tab);
  } else {
    a2 = ordered_amp2<N, float, true>(pc, leg, hel, tab);
  }
  return finish_event<N>(C, i, pass, a2, s.shat, s.x1, s.x2, s.r);
}

// The same from staging slot j.
template <int N, int POL = 0>
__device__ __forceinline__ double rec_one(const GenClass& C, int64_t i, int64_t j, const double* __restrict__ buf,
                                          LdsTable<N>* tab) {
  Staged<N> s;
  load_staged<N>(buf, j, s);
  return rec_staged<N, POL>(C, i, s, tab);
}

// The same with the event on the G lanes of a group (the grouped recursion; span momenta
// from this lane's column ktab of the workgroup's LDS table where span_k_table); lane g = 0
// writes the outputs and returns w, the others return 0.
template <int N, typename T, int G>
__device__ __forceinline__ double rec_one_g(const GenClass& C, int64_t i, int64_t j, const double* __restrict__ buf,
                                            int g, T* ktab, int lanes) {
  using L = SplitLayout<N>;
  const double shat = buf[L::at(j, L::kShat)];
  double pc[N][4];
  const double hb = 0.5 * (C.use_pdf ? sqrt(shat) : C.sqrt_s);
  pc[0][0] = hb;
  pc[0][1] = 0.0;
  pc[0][2] = 0.0;
  pc[0][3] = hb;
#pragma unroll
  for (int t = 1; t < N; ++t)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) pc[t][mu] = buf[L::at(j, L::kMom + 4 * (t - 1) + mu)];
  const uint64_t meta = (uint64_t)__double_as_longlong(buf[L::at(j, L::kMeta)]);
  const uint64_t legs = (uint64_t)__double_as_longlong(buf[L::at(j, L::kLegs)]);
  uint32_t leg[N];
#pragma unroll
  for (int t = 0; t < N; ++t) leg[t] = (uint32_t)(legs >> (4 * t)) & 15u;
  const double a2 = ordered_amp2_g<N, T, G, span_k_table<T>()>(pc, leg, (uint32_t)meta, g, ktab, lanes);
  if (g != 0) return 0.0;
  const bool pass = ((meta >> 32) & 1u) != 0;
  return finish_event<N>(C, i, pass, a2, shat, buf[L::at(j, L::kX1)], buf[L::at(j, L::kX2)], buf[L::at(j, L::kR)]);
}

// Launch: blockDim.x = kKinBlock, perm_lds_bytes(N, kKinBlock) bytes of dynamic LDS,
// ceil(cnt / kKinBlock) workgroups; events first .. first + cnt - 1 into slots 0 .. cnt - 1.
template <int N>
__global__ __launch_bounds__(kKinBlock) void k_kin(GenClass C, int64_t first, int64_t cnt, double* __restrict__ buf) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  kin_one<N>(C, first + j, j, buf, dyn_perm());
}

// Launch: blockDim.x = kLdsLanes, ceil(cnt / kLdsLanes) workgroups, first a multiple of
// kLdsLanes; workgroup b writes the partial of events first + 64 b .. (partial first / 64 + b).
// With ahead > 0 the workgroup, after issuing its own loads, pulls the staged words of tile
// blockIdx.x + ahead into the L2 cache (one 4-byte load per 128-byte line, written to a
// 256-byte LDS scrap area and never read).  Workgroups go to the XCDs in turn and one runs
// per SIMD, so with ahead a multiple of 8 and below the number resident at once, that tile
// starts on the same XCD a fraction of a workgroup's duration later and its first loads hit
// L2 instead of HBM.  Only from N = 8: the shorter workgroups of smaller N measured slower
// with it (n = 4: 0.253 against 0.238 ms per 2^22 events).
template <int N>
constexpr bool rec_prefetch() { return N >= 8; }

template <int N, int POL>
__global__ __launch_bounds__(kLdsLanes) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rec(
    GenClass C, int64_t first, int64_t cnt, const double* __restrict__ buf, double* partials, int64_t ahead) {
  __shared__ LdsTable<N> tab;
  __shared__ unsigned int scrap[rec_prefetch<N>() ? kLdsLanes : 1];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Staged<N> st;
  if (j < cnt) load_staged<N>(buf, j, st);
  const int64_t t = (int64_t)blockIdx.x + ahead;
  if (rec_prefetch<N>() && ahead > 0 && t * kLdsLanes < cnt) {
    // the tile's words are contiguous (SplitLayout): kWords x 64 doubles
    constexpr int kBytes = SplitLayout<N>::kWords * kLdsLanes * 8;
    const char* base = reinterpret_cast<const char*>(buf + t * kLdsLanes * SplitLayout<N>::kWords);
#pragma unroll
    for (int off = 0; off < kBytes; off += kLdsLanes * 128) {
      const int o = off + (int)threadIdx.x * 128;
      if (o < kBytes)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(base + o),
                                         (__attribute__((address_space(3))) void*)scrap, 4, 0, 0);
    }
  }
  double w = 0.0;
  if (j < cnt) w = rec_staged<N, POL>(C, first + j, st, &tab);
  if (partials) block_reduce_store(CSum{w, 0.0}, CSum{w * w, 0.0}, partials + 4 * (first / kLdsLanes + (int64_t)blockIdx.x));
}

// Launch: blockDim.x a multiple of 64 (at most 256), ceil(cnt G / blockDim.x) workgroups,
// grouped_lds_bytes<N, T, G>(blockDim.x) bytes of dynamic LDS, first a multiple of
// blockDim.x / G; workgroup b writes the partial of its blockDim.x / G events at
// first G / blockDim.x + b, as the one-kernel form numbers them.
template <int N, typename T, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rec_g(
    GenClass C, int64_t first, int64_t cnt, const double* __restrict__ buf, double* partials) {
  extern __shared__ unsigned char gdyn[];
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int g = (int)(threadIdx.x % G);
  double w = 0.0;
  if (j < cnt) w = rec_one_g<N, T, G>(C, first + j, j, buf, g, reinterpret_cast<T*>(gdyn) + threadIdx.x, (int)blockDim.x);
  if (partials)
    block_reduce_store(CSum{w, 0.0}, CSum{w * w, 0.0},
                       partials + 4 * (first * G / (int64_t)blockDim.x + (int64_t)blockIdx.x));
}

// The kinematics kernel and the grouped recursion kernel over the class in chunks of
// W.stage_cap events (a multiple of 256); workgroups of `block` lanes.
template <int N, typename T, int G>
hipError_t launch_generate_split_g(const GenClass& C, const GenWork& W, int block, hipStream_t s) {
  if (C.count <= 0) return hipSuccess;
  if (!W.stage || W.stage_cap < 256 || W.stage_cap % 256 != 0 || block % 64 != 0 || block > 256)
    return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  for (int64_t first = 0; first < C.count && e == hipSuccess; first += W.stage_cap) {
    const int64_t cnt = std::min<int64_t>(W.stage_cap, C.count - first);
    hipLaunchKernelGGL((k_kin<N>), dim3((unsigned)((cnt + kKinBlock - 1) / kKinBlock)), dim3(kKinBlock),
                       perm_lds_bytes(N, kKinBlock), s, C, first, cnt, W.stage);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL((k_rec_g<N, T, G>), dim3((unsigned)((cnt * G + block - 1) / block)), dim3(block),
                       (grouped_lds_bytes<N, T, G>(block)), s, C, first, cnt, W.stage, W.partials);
    e = hipGetLastError();
  }
  return e;
}

// Both kernels over the class in chunks of W.stage_cap events (a multiple of 64) through the
// caller's staging buffer; one partial per 64 events, in event order, whatever the chunking.
template <int N, int POL = 0>
hipError_t launch_generate_split(const GenClass& C, const GenWork& W, hipStream_t s) {
  if (C.count <= 0) return hipSuccess;
  if (!W.stage || W.stage_cap < kLdsLanes || W.stage_cap % kLdsLanes != 0) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  for (int64_t first = 0; first < C.count && e == hipSuccess; first += W.stage_cap) {
    const int64_t cnt = std::min<int64_t>(W.stage_cap, C.count - first);
    hipLaunchKernelGGL((k_kin<N>), dim3((unsigned)((cnt + kKinBlock - 1) / kKinBlock)), dim3(kKinBlock),
                       perm_lds_bytes(N, kKinBlock), s, C, first, cnt, W.stage);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL((k_rec<N, POL>), dim3((unsigned)((cnt + kLdsLanes - 1) / kLdsLanes)), dim3(kLdsLanes), 0, s, C,
                       first, cnt, W.stage, W.partials, W.ahead);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace bgk
