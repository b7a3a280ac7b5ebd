// Instantiates one kernel of the library and exports its launcher through a host function
// resolved by the C-ABI layer:
//   BG_KIND 0 generate, 1 amp2, 2 gradient;  BG_N 4..12;  BG_PREC 32 or 64;
//   BG_FORM 1 one event per lane (for generation of the table classes: the split form),
//           2 two lanes per event (kinds 0 and 1 only),
//           3 one event per lane with real polarisations (kind 0 only),
//           4 the W-tensor form, 16 lanes per event (kinds 0 and 1),
//           5 four lanes per event (kinds 0 and 1 only).
// One kernel per translation unit keeps every unit small enough to compile in parallel.
#include "bg_adjoint.hpp"
#include "bg_kernels.hpp"
#include "bg_launch.hpp"
#include "bg_split.hpp"
#include "bg_wtensor.hpp"

#if !defined(BG_N) || !defined(BG_PREC) || !defined(BG_KIND) || !defined(BG_FORM)
#error "BG_N, BG_PREC, BG_KIND and BG_FORM must be defined"
#endif

#define BG_CAT4(a, b, c, d) a##b##_p##c##_k##d
#define BG_NAME(a, b, c, d) BG_CAT4(a, b, c, d)

namespace bgk {

#if BG_PREC == 32
using Real = float;
#else
using Real = double;
#endif

static_assert(BG_KIND == 2 || (BG_FORM == 1 && has_one_lane(BG_N, BG_PREC)) ||
                  (BG_FORM == 2 && has_lane_pairs(BG_N, BG_PREC)) || (BG_FORM == 3 && has_real_pol(BG_N, BG_PREC)) ||
                  (BG_FORM == 4 && has_wtensor(BG_N, BG_PREC)) || (BG_FORM == 5 && has_lane_quads(BG_N, BG_PREC)),
              "this lane form is not built for (n, prec)");

// Lanes per event of the grouped forms
#define BG_GROUP (BG_FORM == 5 ? 4 : 2)

// Launchers take the workgroup size chosen by the host (which also sizes the partials:
// one per workgroup, ceil(count * lanes / block) workgroups; the table classes always use
// one partial per kLdsLanes events).
#if BG_KIND == 0 && BG_FORM == 1
hipError_t BG_NAME(launch_generate_n, BG_N, BG_PREC, BG_KIND)(const GenClass& C, const GenWork& W, int block,
                                                              hipStream_t s) {
#if BG_PREC == 32 && BG_N <= 8
  (void)block;
  static_assert(split_form(BG_N, BG_PREC), "split-form classes");
  return launch_generate_split<BG_N>(C, W, s);
#else
  const int64_t nb = (C.count + block - 1) / block;
  hipLaunchKernelGGL((k_generate<BG_N, Real>), dim3((unsigned)nb), dim3(block), perm_lds_bytes(BG_N, block), s, C,
                     W.partials);
  return hipGetLastError();
#endif
}
#elif BG_KIND == 0 && BG_FORM == 3
hipError_t BG_NAME(launch_generate_real_n, BG_N, BG_PREC, BG_KIND)(const GenClass& C, const GenWork& W, int block,
                                                                   hipStream_t s) {
#if BG_PREC == 32 && BG_N <= 8
  (void)block;
  return launch_generate_split<BG_N, 1>(C, W, s);
#else
  const int64_t nb = (C.count + block - 1) / block;
  hipLaunchKernelGGL((k_generate<BG_N, Real, 1>), dim3((unsigned)nb), dim3(block), perm_lds_bytes(BG_N, block), s,
                     C, W.partials);
  return hipGetLastError();
#endif
}
#elif BG_KIND == 0 && BG_FORM == 4
hipError_t BG_NAME(launch_generate_w_n, BG_N, BG_PREC, BG_KIND)(const GenClass& C, const GenWork& W, int block,
                                                                hipStream_t s) {
  (void)block;
  return launch_generate_w<BG_N, Real>(C, W, s);
}
#elif BG_KIND == 1 && BG_FORM == 4
hipError_t BG_NAME(launch_amp2_w_n, BG_N, BG_PREC, BG_KIND)(int64_t count, const double* mom, const uint32_t* hel,
                                                            const uint8_t* order, double* out, int block,
                                                            hipStream_t s) {
  (void)block;
  hipLaunchKernelGGL((k_amp2_w<BG_N, Real>), dim3((unsigned)((count + 3) / 4)), dim3(64), (w_lds_bytes<BG_N, Real>()),
                     s, count, mom, hel, order, out);
  return hipGetLastError();
}
#elif BG_KIND == 0 && (BG_FORM == 2 || BG_FORM == 5)
#if BG_FORM == 2
#define BG_GEN_GROUP launch_generate2_n
#else
#define BG_GEN_GROUP launch_generate4_n
#endif
hipError_t BG_NAME(BG_GEN_GROUP, BG_N, BG_PREC, BG_KIND)(const GenClass& C, const GenWork& W, int block,
                                                         hipStream_t s) {
  return launch_generate_split_g<BG_N, Real, BG_GROUP>(C, W, block, s);
}
#elif BG_KIND == 1 && BG_FORM == 1
hipError_t BG_NAME(launch_amp2_n, BG_N, BG_PREC, BG_KIND)(int64_t count, const double* mom, const uint32_t* hel,
                                                          const uint8_t* order, double* out, int block,
                                                          hipStream_t s) {
  if (lds_span_table(BG_N, BG_PREC)) block = kLdsLanes;
  const int64_t nb = (count + block - 1) / block;
  hipLaunchKernelGGL((k_amp2<BG_N, Real>), dim3((unsigned)nb), dim3(block), 0, s, count, mom, hel, order, out);
  return hipGetLastError();
}
#elif BG_KIND == 1 && (BG_FORM == 2 || BG_FORM == 5)
#if BG_FORM == 2
#define BG_AMP2_GROUP launch_amp2_2_n
#else
#define BG_AMP2_GROUP launch_amp2_4_n
#endif
hipError_t BG_NAME(BG_AMP2_GROUP, BG_N, BG_PREC, BG_KIND)(int64_t count, const double* mom, const uint32_t* hel,
                                                          const uint8_t* order, double* out, int block,
                                                          hipStream_t s) {
  const int64_t nb = (BG_GROUP * count + block - 1) / block;
  hipLaunchKernelGGL((k_amp2_g<BG_N, Real, BG_GROUP>), dim3((unsigned)nb), dim3(block),
                     (grouped_lds_bytes<BG_N, Real, BG_GROUP>(block)), s, count, mom, hel, order, out);
  return hipGetLastError();
}
#elif BG_KIND == 2
// Two kernels: the recursion and its reverse sweep (one, two or four lanes per event), then
// the helicity-source, momentum, RAMBO and x adjoints (one lane per event).
hipError_t BG_NAME(launch_grad_n, BG_N, BG_PREC, BG_KIND)(const GradArgs& G, int block, hipStream_t s) {
  constexpr int GL = grad_lanes(BG_N, BG_PREC);
  if constexpr (GL == 1) {
    const int64_t nb = (G.count + block - 1) / block;
    hipLaunchKernelGGL((k_grad<BG_N, Real>), dim3((unsigned)nb), dim3(block), 0, s, G);
  } else {
    (void)block;
    const int64_t nb = (GL * G.count + 255) / 256;
    hipLaunchKernelGGL((k_grad_g<BG_N, Real, GL>), dim3((unsigned)nb), dim3(256), 0, s, G);
  }
  hipLaunchKernelGGL((k_grad_back<BG_N>), dim3((unsigned)((G.count + 255) / 256)), dim3(256), 0, s, G);
  return hipGetLastError();
}
#else
#error "unknown kernel kind or form"
#endif

}  // namespace bgk
