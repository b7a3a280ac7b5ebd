// Instantiates one kernel kind (BG_KIND: 0 generate, 1 amp2, 2 gradient) of one
// multiplicity (BG_N, 4..12) and recursion precision (BG_PREC, 32 or 64), and exports its
// launcher through a host function resolved by the C-ABI layer.
#include "bg_adjoint.hpp"
#include "bg_kernels.hpp"
#include "bg_launch.hpp"
#if BG_KIND == 0 && BG_PREC == 32 && BG_N <= 8
#include "bg_split.hpp"
#define BG_SPLIT 1
#else
#define BG_SPLIT 0
#endif

#if !defined(BG_N) || !defined(BG_PREC) || !defined(BG_KIND)
#error "BG_N, BG_PREC and BG_KIND must be defined"
#endif

#define BG_CAT4(a, b, c, d) a##b##_p##c##_k##d
#define BG_NAME(a, b, c, d) BG_CAT4(a, b, c, d)

namespace bgk {

#if BG_PREC == 32
using Real = float;
#else
using Real = double;
#endif

// the two-lane forms, for the multiplicities of has_lane_pairs
#if (BG_PREC == 32 && BG_N >= 9) || (BG_PREC == 64 && BG_N >= 6)
#define BG_PAIRS 1
#else
#define BG_PAIRS 0
#endif
static_assert(has_lane_pairs(BG_N, BG_PREC) == (BG_PAIRS == 1), "lane-pair build condition");

// Launchers take the workgroup size chosen by the host (which also sizes the partials:
// one per workgroup, ceil(count * lanes / block) workgroups).
#if BG_KIND == 0
hipError_t BG_NAME(launch_generate_n, BG_N, BG_PREC, BG_KIND)(const GenClass& C, double* partials, int block,
                                                              hipStream_t s) {
  const bool table = lds_span_table(BG_N, BG_PREC);
  if (table) block = kLdsLanes;
#if BG_SPLIT
  // kinematics and recursion as two kernels for large calls; the fused kernel for small
  // ones and if there is no staging memory
  if (C.count >= kSplitMinEvents) {
    const hipError_t e = launch_generate_split<BG_N, Real>(C, partials, s);
    if (e != hipErrorOutOfMemory) return e;
  }
#endif
  const int64_t nb = (C.count + block - 1) / block;
  hipLaunchKernelGGL((k_generate<BG_N, Real>), dim3((unsigned)nb), dim3(block), table ? 0 : perm_lds_bytes(BG_N, block),
                     s, C, partials);
  return hipGetLastError();
}
#if BG_PAIRS
hipError_t BG_NAME(launch_generate2_n, BG_N, BG_PREC, BG_KIND)(const GenClass& C, double* partials, int block,
                                                               hipStream_t s) {
  const int64_t nb = (2 * C.count + block - 1) / block;
  hipLaunchKernelGGL((k_generate_g<BG_N, Real, 2>), dim3((unsigned)nb), dim3(block), 0, s, C, partials);
  return hipGetLastError();
}
#endif
#elif BG_KIND == 1
hipError_t BG_NAME(launch_amp2_n, BG_N, BG_PREC, BG_KIND)(int64_t count, const double* mom, const uint32_t* hel,
                                                          const uint8_t* order, double* out, int block,
                                                          hipStream_t s) {
  if (lds_span_table(BG_N, BG_PREC)) block = kLdsLanes;
  const int64_t nb = (count + block - 1) / block;
  hipLaunchKernelGGL((k_amp2<BG_N, Real>), dim3((unsigned)nb), dim3(block), 0, s, count, mom, hel, order, out);
  return hipGetLastError();
}
#if BG_PAIRS
hipError_t BG_NAME(launch_amp2_2_n, BG_N, BG_PREC, BG_KIND)(int64_t count, const double* mom, const uint32_t* hel,
                                                            const uint8_t* order, double* out, int block,
                                                            hipStream_t s) {
  const int64_t nb = (2 * count + block - 1) / block;
  hipLaunchKernelGGL((k_amp2_g<BG_N, Real, 2>), dim3((unsigned)nb), dim3(block), 0, s, count, mom, hel, order, out);
  return hipGetLastError();
}
#endif
#elif BG_KIND == 2
// Two kernels: the recursion and its reverse sweep (one or two lanes per event), then the
// helicity-source, momentum, RAMBO and x adjoints (one lane per event).
#if BG_PREC == 32 && BG_N >= 6 && BG_N <= 8
#define BG_GRAD_PAIRS 1
#else
#define BG_GRAD_PAIRS 0
#endif
static_assert(grad_lane_pairs(BG_N, BG_PREC) == (BG_GRAD_PAIRS == 1), "gradient lane-pair condition");
hipError_t BG_NAME(launch_grad_n, BG_N, BG_PREC, BG_KIND)(const GradArgs& G, int block, hipStream_t s) {
#if BG_GRAD_PAIRS
  (void)block;
  const int64_t nb = (2 * G.count + 255) / 256;  // 256 lanes: the LDS staging fills a CU
  hipLaunchKernelGGL((k_grad_g<BG_N, Real>), dim3((unsigned)nb), dim3(256), 0, s, G);
#else
  const int64_t nb = (G.count + block - 1) / block;
  hipLaunchKernelGGL((k_grad<BG_N, Real>), dim3((unsigned)nb), dim3(block), 0, s, G);
#endif
  hipLaunchKernelGGL((k_grad_back<BG_N>), dim3((unsigned)((G.count + 255) / 256)), dim3(256), 0, s, G);
  return hipGetLastError();
}
#endif

}  // namespace bgk
