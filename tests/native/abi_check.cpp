// Host-side checks of the C ABI layer, built with AddressSanitizer and UndefinedBehavior-
// Sanitizer on the host code (tests/test_abi_sanitized.py) together with bg_capi.hip,
// bg_finalize.hip, bg_hist.hip and bg_probe.hip but none of the kernel units, and run on a machine
// without a GPU: every entry point's argument checks, its table lookups and, where the
// arguments are valid, its first HIP call (which then fails: BG_EHIP) run under the
// sanitizers.  Prints one "name status" line per call; the test compares them.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "bg.h"

static void show(const char* name, int st) { printf("%s %d\n", name, st); }

static bg_config cfg(int n, int prec) {
  bg_config c;
  memset(&c, 0, sizeof(c));
  c.n = n;
  c.prec = prec;
  c.sqrt_s = 14000.0;
  c.use_pdf = 1;
  c.pdf_a = -1.3;
  c.pdf_b = 5;
  c.alpha_s = 0.118;
  c.pt_min = 20.0;
  c.eta_max = 2.5;
  c.dr_min = 0.4;
  c.random_order = 1;
  c.seed = 7;
  return c;
}

int main() {
  printf("version %d\n", bg_version());
  printf("hash %s\n", bg_source_hash() ? "set" : "null");
  for (int s = 1; s >= -5; --s) printf("strerror %d %s\n", s, bg_strerror(s) ? "text" : "null");

  // bg_generate
  bg_config c = cfg(8, 32);
  int64_t cnt = 1000;
  bg_outputs out;
  memset(&out, 0, sizeof(out));
  show("generate_null_cfgs", bg_generate(NULL, 1, &cnt, NULL, &out, NULL));
  show("generate_ncfg0", bg_generate(&c, 0, &cnt, NULL, &out, NULL));
  show("generate_ncfg17", bg_generate(&c, 17, &cnt, NULL, &out, NULL));
  int64_t neg = -1;
  show("generate_negative_count", bg_generate(&c, 1, &neg, NULL, &out, NULL));
  bg_config c3 = cfg(3, 32);
  show("generate_n3", bg_generate(&c3, 1, &cnt, NULL, &out, NULL));
  bg_config c13 = cfg(13, 32);
  show("generate_n13", bg_generate(&c13, 1, &cnt, NULL, &out, NULL));
  bg_config cp = cfg(8, 16);
  show("generate_prec16", bg_generate(&cp, 1, &cnt, NULL, &out, NULL));
  bg_config cpol = cfg(8, 32);
  cpol.polarisation = 2;
  show("generate_polarisation2", bg_generate(&cpol, 1, &cnt, NULL, &out, NULL));
  bg_config cres = cfg(8, 32);
  cres.reserved = 1;
  show("generate_reserved", bg_generate(&cres, 1, &cnt, NULL, &out, NULL));
  bg_config cs = cfg(8, 32);
  cs.sqrt_s = -1.0;
  show("generate_sqrt_s", bg_generate(&cs, 1, &cnt, NULL, &out, NULL));
  int64_t zero = 0;
  show("generate_empty", bg_generate(&c, 1, &zero, NULL, &out, NULL));
  show("generate_valid", bg_generate(&c, 1, &cnt, NULL, &out, NULL));
  bg_config two[2] = {cfg(4, 32), cfg(12, 64)};
  int64_t cnt2[2] = {100, 100};
  bg_outputs out2[2];
  memset(out2, 0, sizeof(out2));
  show("generate_two_valid", bg_generate(two, 2, cnt2, NULL, out2, NULL));

  // bg_generate_noalloc
  show("noalloc_null", bg_generate_noalloc(NULL, 10, NULL, &out, NULL));
  show("noalloc_oversize", bg_generate_noalloc(&c, (int64_t)1 << 25, NULL, &out, NULL));
  bg_config cdyn = cfg(8, 32);
  cdyn.dynamic_scale = 1;
  show("noalloc_dynamic", bg_generate_noalloc(&cdyn, 10, NULL, &out, NULL));
  show("noalloc_valid", bg_generate_noalloc(&c, 10, NULL, &out, NULL));

  // bg_amp2 and bg_amp2_grad
  double d[8];
  uint32_t h[1];
  uint8_t o[16];
  show("amp2_n13", bg_amp2(13, 32, 4, d, h, o, d, NULL));
  show("amp2_negative", bg_amp2(8, 32, -1, d, h, o, d, NULL));
  show("amp2_empty", bg_amp2(8, 32, 0, NULL, NULL, NULL, NULL, NULL));
  show("amp2_null", bg_amp2(8, 64, 4, NULL, NULL, NULL, NULL, NULL));
  show("amp2_valid", bg_amp2(8, 64, 4, d, h, o, d, NULL));
  show("grad_null_cfg", bg_amp2_grad(NULL, 4, d, d, h, o, NULL, d, d, NULL, NULL));
  show("grad_empty", bg_amp2_grad(&c, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL));
  show("grad_polarisation", bg_amp2_grad(&cpol, 4, d, d, h, o, NULL, d, d, NULL, NULL));
  show("grad_valid", bg_amp2_grad(&c, 4, d, d, h, o, NULL, d, d, NULL, NULL));

  // histograms
  bg_hist_axis ax[2] = {{0, 40, 0.0, 2000.0}, {1, 30, 0.0, 6.0}};
  int64_t limbs[8];
  show("hist_null_axes", bg_hist_accumulate(10, d, d, 2, NULL, limbs, NULL));
  bg_hist_axis bad = {2, 10, 0.0, 1.0};
  show("hist_bad_column", bg_hist_accumulate(10, d, d, 1, &bad, limbs, NULL));
  bg_hist_axis big = {0, 500, 0.0, 1.0};
  show("hist_too_many_bins", bg_hist_accumulate(10, d, d, 1, &big, limbs, NULL));
  bg_hist_axis inv = {0, 10, 1.0, 0.0};
  show("hist_lo_ge_hi", bg_hist_accumulate(10, d, d, 1, &inv, limbs, NULL));
  show("hist_valid", bg_hist_accumulate(10, d, d, 2, ax, limbs, NULL));
  show("hist_read_null", bg_hist_read(2, ax, NULL, d, NULL));

  // settings
  int b = 0, it = 0, l = 0, f = 0;
  show("set_launch_bad_block", bg_set_launch(8, 32, 96, 1));
  show("set_launch_n2", bg_set_launch(2, 32, 128, 1));
  show("set_launch_ok", bg_set_launch(8, 32, 128, 4));
  show("get_launch", bg_get_launch(8, 32, &b, &it));
  printf("launch %d %d\n", b, it);
  show("set_launch_default", bg_set_launch(8, 32, 0, 0));
  show("set_lanes_3", bg_set_lanes(8, 32, 3));
  show("set_lanes_n8_2", bg_set_lanes(8, 32, 2));
  show("get_lanes", bg_get_lanes(12, 64, &l));
  printf("lanes %d\n", l);
  show("set_form_bad", bg_set_form(10, 32, 2));
  show("set_form_n9", bg_set_form(9, 32, 1));
  show("get_form", bg_get_form(12, 32, &f));
  printf("form %d\n", f);
  show("set_mixed_bad", bg_set_mixed_launch(3));
  show("set_mixed_ok", bg_set_mixed_launch(0));
  printf("mixed %d\n", bg_get_mixed_launch());
  int64_t first_bad = 0;
  show("check_n3", bg_check_events(3, 5, h, o, &first_bad, NULL));
  show("check_null", bg_check_events(8, 5, NULL, NULL, NULL, NULL));
  double tf = 0.0;
  show("fma_prec16", bg_fma_rate(16, &tf, NULL));
  show("fma_null", bg_fma_rate(32, NULL, NULL));
  show("fma_valid", bg_fma_rate(32, &tf, NULL));
  return 0;
}
