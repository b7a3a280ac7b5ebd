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

// Multiplicities whose kernels are also built with an event spread over two lanes (the
// one-lane recursion needs more than 512 registers there); which form runs is a launch
// setting (bg_set_lanes), defaulting to default_lanes.
constexpr bool has_lane_pairs(int n, int prec) { return prec == 32 ? n >= 9 : n >= 6; }
constexpr int default_lanes(int n, int prec) { return prec == 32 ? (n >= 10 ? 2 : 1) : (n >= 7 ? 2 : 1); }

// The gradient kernel with an event on two lanes (forward values staged in LDS, which
// bounds it to FP32 n <= 8); elsewhere one lane per event.
constexpr bool grad_lane_pairs(int n, int prec) { return prec == 32 && n >= 6 && n <= 8; }

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

using GenerateFn = hipError_t (*)(const GenClass& C, double* partials, int block, hipStream_t s);
using Amp2Fn = hipError_t (*)(int64_t count, const double* mom, const uint32_t* hel, const uint8_t* order,
                              double* out, int block, hipStream_t s);
using GradFn = hipError_t (*)(const GradArgs& G, int block, hipStream_t s);

struct Launchers {
  GenerateFn generate;
  Amp2Fn amp2;
  GradFn grad;
  GenerateFn generate2;  // two lanes per event (where has_lane_pairs)
  Amp2Fn amp2_2;
};

// Fixed-order compensated reduction of nparts partials into acc, through level2
// (kFinalizeGroups x 4 doubles of scratch): at most kFinalizeGroups workgroups reduce
// contiguous runs of partials, then one workgroup adds their results to acc.
constexpr int kFinalizeGroups = 512;
hipError_t launch_finalize(const double* partials, int64_t nparts, double* level2, double* acc, hipStream_t s);

// One class of a multi-class launch and one tile of its work list (device-resident).
struct MultiClass {
  GenClass C;
  int32_t n;
  int32_t tile_begin, tile_end;  // this class's tiles in the list
  double* acc;
};

struct Tile {
  int64_t first;  // first local event index
  int32_t count;
  int32_t cls;
};

hipError_t launch_generate_multi_p32(const MultiClass* classes, int nclasses, const Tile* tiles, int ntiles,
                                     int* counter, double* partials, int grid, int block, hipStream_t s);

}  // namespace bgk
