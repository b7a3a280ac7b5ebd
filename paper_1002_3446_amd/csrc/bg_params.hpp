// Kernel-side parameter blocks, filled by the host layer from bg_config / bg_inputs /
// bg_outputs (see include/bg.h for the meaning and layout of every array).
#pragma once

#include <stdint.h>

#include "bg_device.hpp"

namespace bgk {

struct OutPtrs {
  double* weight;
  double* amp2;
  double* obs;
  uint8_t* pass;
  double* momenta;
  uint32_t* hel;
  uint8_t* order;
  double* x12;
  double* uniforms;
  double* logw;
};

// One event class of a generation launch.
struct GenClass {
  int64_t count;
  uint64_t first_event;
  uint32_t key0, key1;
  int32_t use_pdf, random_order;
  int32_t polarisation;       // 0 helicity states, 1 random real unit vectors
  int32_t dynamic_scale;      // 1: mu = H_T, alpha_s(mu) and f(x, mu) from the grids
  double lmu0;                // ln of the reference scale (alpha_s, f(x) hold there)
  double log_alpha0;          // ln alpha_s(mu0)
  double sqrt_s;              // collider sqrt(S), or the fixed sqrt(s_hat) without PDF
  double pt_min, eta_max, dr_min;
  double wconst;              // event-independent weight factor (pb GeV^(2(5-n)))
  double log_const;           // log of the event-independent factors of w_int
  PdfParams pdf;
  ScaleGrid grid;
  const double* in_u;
  const double* in_x;
  const uint32_t* in_hel;
  const uint8_t* in_order;
  OutPtrs out;
};

}  // namespace bgk
