// Host-visible launch table: one entry per (multiplicity, precision), filled by the
// per-multiplicity translation units (bg_inst.hip compiled with BG_N = 4..12).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bg_params.hpp"

namespace bgk {

// FP32 classes with n <= 8 keep their span momenta and propagators in an LDS table
// (SpanKLds) and run with 64-lane workgroups: at n = 8 four workgroups use 143 KB of a
// compute unit's 160 KB.  Larger n and FP64 sum the FP64 leg momenta at every use.
constexpr int kLdsLanes = 64;

// Dynamic LDS of the generation kernels without the span table: the per-lane column of the
// leg-to-position momentum permutation, 4 (n - 2) doubles per lane.
constexpr unsigned perm_lds_bytes(int n, int block) { return 8u * 4u * (unsigned)(n - 2) * (unsigned)block; }
constexpr bool lds_span_table(int n, int prec) { return prec == 32 && n <= 8; }

// The table classes generate events in two kernels (kinematics at several waves per SIMD,
// then the recursion at one), joined by a staging buffer of split_words(n) doubles per event.
constexpr bool split_form(int n, int prec) { return lds_span_table(n, prec); }
constexpr int split_words(int n) { return 4 * (n - 1) + 6; }

// Lane forms the library holds per (n, prec): one event per lane where the recursion fits a
// lane's 512 registers (FP32 n <= 9, FP64 n <= 6); two lanes per event from FP32 n = 9 and
// FP64 n = 6 on (the one-lane form spills kilobytes per lane beyond that); four lanes for
// FP64 n >= 10, where two still spill (FP64 n = 12: 2.9 KB per lane with two, 448 B with
// four).  Which form runs is a launch
// setting (bg_set_lanes), defaulting to default_lanes.
constexpr bool has_one_lane(int n, int prec) { return prec == 32 ? n <= 9 : n <= 6; }
constexpr bool has_lane_pairs(int n, int prec) { return prec == 32 ? n >= 9 : n >= 6; }
constexpr bool has_lane_quads(int n, int prec) { return prec == 64 && n >= 10; }
constexpr int default_lanes(int n, int prec) { return prec == 32 ? (n >= 10 ? 2 : 1) : (n >= 10 ? 4 : (n >= 7 ? 2 : 1)); }

// Classes built with real polarisations (real currents: half the registers of complex ones,
// so one lane per event fits every FP32 class).
constexpr bool has_real_pol(int n, int prec) { return prec == 32 ? n <= 12 : n <= 8; }

// Classes built with the W-tensor form of the recursion (Eqs. 3.3-3.4), an alternative for
// large n chosen per class (bg_set_form); FP64 at n = 6 and 10 for parity with the oracle.
constexpr bool has_wtensor(int n, int prec) { return prec == 32 ? (n == 8 || n >= 10) : (n == 6 || n == 10); }

// Lanes per event of the gradient's recursion kernel: one (k_grad) for FP32 n <= 5 and
// FP64 n = 4; else the grouped reverse sweep (k_grad_g), with two lanes (two Lorentz
// components each) while the currents and their adjoints fit a lane's registers (FP32
// n = 6..8, FP64 n = 5, 6: fewer cross-lane sums, and the kinematics on half as many lanes),
// and four lanes beyond (no scratch through FP32 n = 11 and FP64 n = 8).
constexpr int grad_lanes(int n, int prec) {
  return prec == 32 ? (n <= 5 ? 1 : (n <= 8 ? 2 : 4)) : (n <= 4 ? 1 : (n <= 6 ? 2 : 4));
}

struct GradArgs {
  int64_t count;
  double sqrt_s;
  int32_t use_pdf;
  double pdf_a;
  int32_t pdf_b;
  const double* u;
  const double* x12;
  const uint32_t* hel;
  const uint8_t* order;
  const double* gout;
  double* grad_u;
  double* grad_x;
  double* logw;
  double log_const;  // log of the event-independent factors of w_int
  double* pbuf;      // workspace [12 (n - 1) + 1][count]: recursion adjoints between the two kernels
};

// Device memory a generation launch works in: per-workgroup partials (NULL: no totals) and,
// for the split form, a staging buffer of stage_cap events.
struct GenWork {
  double* partials;
  double* stage;
  int64_t stage_cap;
  int64_t ahead;  // one-lane recursion kernel: tiles between a workgroup and the tile whose
                  // staged words it pulls into the L2 cache for a later workgroup (0: none)
};

using GenerateFn = hipError_t (*)(const GenClass& C, const GenWork& W, int block, hipStream_t s);
using Amp2Fn = hipError_t (*)(int64_t count, const double* mom, const uint32_t* hel, const uint8_t* order,
                              double* out, int block, hipStream_t s);
using GradFn = hipError_t (*)(const GradArgs& G, int block, hipStream_t s);

struct Launchers {
  GenerateFn generate;   // one lane per event (the split form for the table classes)
  Amp2Fn amp2;
  GradFn grad;
  GenerateFn generate2;  // two lanes per event (where has_lane_pairs)
  Amp2Fn amp2_2;
  GenerateFn generate_real;  // real polarisations, one lane per event (where has_real_pol)
  GenerateFn generate_w;     // W-tensor form, 16 lanes per event (where has_wtensor)
  Amp2Fn amp2_w;
  GenerateFn generate4;      // four lanes per event (where has_lane_quads)
  Amp2Fn amp2_4;
};

// Fixed-order compensated reduction of nparts partials into acc, through level2
// (kFinalizeGroups x 4 doubles of scratch): at most kFinalizeGroups workgroups reduce
// contiguous runs of partials, then one workgroup adds their results to acc.
constexpr int kFinalizeGroups = 512;
hipError_t launch_finalize(const double* partials, int64_t nparts, double* level2, double* acc, hipStream_t s);

// One class of a multi-class launch and one tile of its work list (device-resident).
// Table classes (n <= 8) are staged: their kinematics run in the multi-class kinematics
// kernel (workgroups kin_begin .. of it), their stage is at stage + stage_off; the others
// are generated two lanes per event inside the persistent kernel.
struct MultiClass {
  GenClass C;
  int32_t n;
  int32_t tile_begin, tile_end;  // this class's tiles in the list
  int32_t staged;
  int64_t kin_begin;             // first kinematics workgroup (staged classes)
  int64_t stage_off;             // offset of the class's stage, in doubles
  double* acc;
};

struct Tile {
  int64_t first;  // first local event index
  int32_t count;
  int32_t cls;
};

constexpr int kKinBlock = 128;   // workgroup of the kinematics kernels
constexpr int kMultiBlock = 64;  // workgroup (one wave) of the persistent kernel

// Sustained multiply-add rate of the VALU (bg_probe.hip): flops per second of `iters` rounds
// of 16 independent fused multiply-add chains per lane, at eight waves per SIMD on ncu
// compute units; synchronises the stream.
hipError_t measure_fma_rate(int prec, int iters, int ncu, double* flops_per_s, hipStream_t s);

// (weak: a library built without bg_multi.hip runs mixed calls one class after another)
__attribute__((weak)) hipError_t launch_generate_multi_p32(const MultiClass* classes, int nclasses, int nstaged,
                                                           int64_t kin_blocks, const Tile* tiles, int ntiles,
                                                           int* counter, double* stage, double* partials, int grid,
                                                           hipStream_t s);

// Histogram axes of one bg_hist_accumulate / bg_hist_read call (bg_hist.hip): axis a
// reads obs column `column`, bins [lo, hi) into nbins, and owns bins first_bin ..
// first_bin + nbins + 1 (underflow, nbins, overflow) of the call's limb array.
constexpr int kHistMaxAxes = 8;
constexpr int kHistMaxBinsTotal = 400;  // bins over all axes of one call (LDS of the accumulation)
struct HistAxis {
  int32_t column, nbins, first_bin;
  double lo, hi;
};
struct HistAxes {
  int32_t naxes, total_bins;
  HistAxis axis[kHistMaxAxes];
};
hipError_t launch_hist_accumulate(int64_t N, const double* weight, const double* obs, const HistAxes& A,
                                  int64_t* limbs, int cus, hipStream_t s);
hipError_t launch_hist_read(const HistAxes& A, const int64_t* limbs, double* out, hipStream_t s);

}  // namespace bgk
