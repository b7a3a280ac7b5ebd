/* bg.h - C ABI of libbg: leading-colour gg -> (n-2) g tree amplitudes by Berends-Giele
 * recursion, RAMBO phase space, jet cuts and event weights, one event per GPU lane,
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: W. T. Giele, G. C. Stavenga, J. Winter, "Thread-Scalable Evaluation of
 * Multi-Jet Observables" (FERMILAB-PUB-10-025-T):
 *   Sec. 3, Eq. 3.1-3.2   the recursion for colour-ordered off-shell currents,
 *   Sec. 3, Eq. 3.5-3.6   the amputated closure m of the ordered amplitude,
 *   Sec. 3, Eq. 3.7-3.8   leading colour and the random-ordering cross section,
 *   Sec. 3 (text)         RAMBO phase space, flag-only jet cuts, observables,
 *   Sec. 4                jet cuts pT > 20 GeV, |eta| < 2.5, dR > 0.4; compensated sums.
 *
 * Conventions shared by every entry point
 *   - Pointers to per-event arrays are HIP device pointers owned by the caller; every
 *     array is dense, row-major, with the layout stated at each argument.  The library
 *     keeps no pointer after the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and the call
 *     returns without synchronising.  A kernel fault surfaces at the caller's next
 *     synchronisation of that stream.
 *   - Host-side argument errors return a negative bg_status before anything is
 *     enqueued; a failed HIP launch or allocation returns BG_EHIP / BG_ENOMEM.  No C++
 *     exception crosses this interface.
 *   - Momenta are (E, px, py, pz) in GeV, metric (+,-,-,-).  Legs 0 and 1 are the
 *     incoming partons along +z and -z; legs 2..n-1 the outgoing gluons.
 *   - A helicity word has bit i set when leg i has all-outgoing helicity +.
 *   - A colour ordering is n bytes: order[0] is the closing leg (always 0 for
 *     generated events), order[1..n-1] the ordered recursion legs.  The compute entry
 *     points do not check per-event array contents (that order is a permutation, that
 *     momenta conserve); a malformed leg index is clamped into range, never followed
 *     out of bounds.  bg_check_events checks orderings and helicity words on request.
 *   - |A|^2 is reported in the Parke-Taylor normalisation (Tr(T^a T^b) = delta^ab):
 *     the printed brackets of Eq. 3.2 carry coefficient 1, so |m|^2 = 2^(n-2) |A|^2.
 */
#ifndef BG_H
#define BG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BG_OK = 0,
  BG_EINVAL = -1,   /* NULL required pointer, bad size or inconsistent configuration */
  BG_ENOTSUP = -2,  /* n outside 4..12, prec not 32 or 64 */
  BG_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
  BG_ENOMEM = -4    /* device workspace could not be allocated */
} bg_status;

/* One event class (Sec. 3, Eq. 3.8 with the synthetic density replacing LHAPDF). */
typedef struct {
  int32_t n;            /* external gluons, 4..12 */
  int32_t prec;         /* 32 or 64: precision of helicity vectors, currents and closure;
                           phase space, cuts, span invariants K^2 and weights are FP64 */
  double sqrt_s;        /* GeV: collider sqrt(S) when use_pdf = 1, else the fixed sqrt(s_hat) */
  int32_t use_pdf;      /* 1: x1, x2 drawn from f(x) = x^pdf_a (1-x)^pdf_b on [tau_min, 1) */
  int32_t pdf_b;        /* integer exponent b, 0..16 */
  double pdf_a;         /* exponent a; a + k + 1 must not vanish for k = 0..b */
  double tau_min;       /* lower end of x; <= 0 means ((n-2) pt_min / sqrt_s)^2 */
  double alpha_s;       /* fixed strong coupling, g^2 = 4 pi alpha_s */
  double pt_min;        /* GeV; cut pT > pt_min on every outgoing gluon */
  double eta_max;       /* cut |eta| < eta_max */
  double dr_min;        /* cut Delta R > dr_min on every outgoing pair */
  int32_t random_order; /* 1: colour ordering drawn per event (Eq. 3.8); 0: identity */
  int32_t polarisation; /* 0: helicity states drawn uniformly from the 2^n (the helicity word);
                           1: random real unit vectors orthogonal to each momentum (Sec. 3,
                           the paper's choice): eps = cos(psi) e1 + sin(psi) e2 in the
                           transverse basis of the physical momentum, psi = 2 pi u with u
                           from Philox (block 1 + (n-2) + ceil((n-2)/4) + k/4, word k%4 for
                           leg k); every current is real.  2^n |A|^2 averages to the helicity
                           sum either way, so the weight is the same formula.  bg_generate
                           only: FP32 n = 4..12 and FP64 n = 4..8 (else BG_ENOTSUP), one lane
                           per event, never in the persistent launch; the hel output then
                           holds the drawn but unused helicity word */
  uint64_t seed;        /* Philox-4x32-10 key */
  uint64_t first_event; /* event index of the first event (Philox counter offset) */
  int32_t dynamic_scale;/* 0: fixed alpha_s and density (the fields above);
                           1: the scale of each event is mu = H_T (Sec. 4, Fig. 3): the weight
                           takes alpha_s(mu)^(n-2) f(x1, mu) f(x2, mu), read from grids with
                           linear interpolation (Sec. 3): alpha_s(mu) at one loop with
                           n_f = 5, alpha_s(mu0) = alpha_s, on 512 nodes uniform in ln mu over
                           [5, 20000] GeV; ln f(x, mu) with the exponents a + pdf_da ln(mu/mu0),
                           b + pdf_db ln(mu/mu0) on 64 x 1024 nodes uniform in ln mu and in
                           ln(x/(1-x)) over x in [1e-6, 1 - 1e-9]; scales and x outside take
                           the edge values.  x1, x2 are still drawn from f(x) at mu0 (the
                           ratio enters the weight).  Not for bg_amp2_grad or
                           bg_generate_noalloc (BG_ENOTSUP) */
  int32_t reserved;     /* must be 0 */
  double mu0;           /* GeV, the reference scale of alpha_s and f(x); <= 0 means 91.188 */
  double pdf_da, pdf_db;/* d a / d ln mu and d b / d ln mu of the density's exponents */
} bg_config;

/* Optional caller-supplied draws for bg_generate; any NULL field is drawn from Philox.
 * Used to evaluate given phase-space points (tests, the log-weight gradient). */
typedef struct {
  const double *uniforms;  /* [N][4(n-2)]: rho1..rho4 of outgoing gluons 2..n-1, in (0,1) */
  const double *x12;       /* [N][2]: x1, x2 VALUES in [tau_min, 1) (ignored unless use_pdf) */
  const uint32_t *hel;     /* [N] helicity words */
  const uint8_t *order;    /* [N][n] colour orderings */
} bg_inputs;

/* Per-class outputs; every pointer may be NULL (skipped). */
typedef struct {
  double *weight;    /* [N] event weight in pb; exactly 0 when the event fails the cuts */
  double *amp2;      /* [N] |A(sigma; h)|^2, GeV^(2(4-n)), computed for every event */
  double *obs;       /* [N][2] H_T = sum pT (GeV), R_min = min Delta R */
  uint8_t *pass;     /* [N] 1 when the event passes all cuts */
  double *momenta;   /* [N][n][4] lab-frame physical momenta */
  uint32_t *hel;     /* [N] helicity words used */
  uint8_t *order;    /* [N][n] colour orderings used */
  double *x12;       /* [N][2] x1, x2 used (1, 1 when use_pdf = 0) */
  double *uniforms;  /* [N][4(n-2)] RAMBO uniforms used */
  double *acc;       /* [4] sum w, its compensation, sum w^2, its compensation; the call's
                        compensated totals are ADDED (caller zeroes before the first call) */
  double *logw;      /* [N] log w_int: the log integrand weight of bg_amp2_grad (no cut step
                        function, no sampling density); -inf when |A|^2 = 0 */
} bg_outputs;

/* Generate events of ncfg classes (Sec. 3).  One class: a kinematics kernel (one lane per
 * event) and a recursion kernel joined by a staging buffer ((4n + 2) * 8 B per event, chunks
 * of at most 2^22 events), for FP32 n <= 8 and every form with two or four lanes per event
 * or the W-tensor form; the one-lane classes without the LDS span table (FP32 n = 9 with one
 * lane, FP64 n <= 6) and real polarisations beyond FP32 n = 8 as one kernel.  A small setup
 * launch, once per density and device, tabulates the inverse CDF of the parton density when
 * x1, x2 are sampled.  Several classes (mixed multiplicities): as chosen by
 * bg_set_mixed_launch, either one after another, or the FP32 classes in one persistent
 * launch whose workgroups take tiles (largest n first) from a shared queue, or side by side
 * on concurrent streams.  Class k gets counts[k] events with indices
 * cfgs[k].first_event + 0..counts[k]-1; event i of a class is a pure function of
 * (seed, first_event + i, n) and of ins[k] when given, and its per-event outputs are
 * bitwise the same for every call size, split of the event range and launch mode (the
 * persistent launch evaluates n = 9 with two lanes per event, as bg_set_lanes(9, 32, 2)
 * does); the totals agree within the compensated-sum bound.
 * Device workspace (partials, staging) is allocated stream-ordered from a library-owned
 * memory pool per device, which keeps up to 4 GiB reserved between calls.
 * cfgs, counts, outs: host arrays of ncfg entries; ins: NULL or ncfg entries.
 * counts[k] = 0 is allowed.  Given draws are not validated; an event whose uniforms or
 * x1, x2 are not finite gets pass = 0 and w = 0, so it never enters the totals, and its
 * momenta, observables, |A|^2 and log w are not finite.  Errors: BG_EINVAL (ncfg < 1 or > 16, counts < 0,
 * bad parameters), BG_ENOTSUP (n, prec, or a lane form not built), BG_ENOMEM. */
int bg_generate(const bg_config *cfgs, int ncfg, const int64_t *counts,
                const bg_inputs *ins, const bg_outputs *outs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bg_generate for ONE class (cfg, count,
 * in, out as bg_generate's entries; in may be NULL) with no allocation and no copy of its
 * own.  Every buffer the call needs lives in a library array that each GPU holds from the
 * first such call until the process ends (about 27 MiB): the inverse-CDF table of the
 * density last used (rebuilt by a small kernel when the density changes), the partials of
 * the compensated sums and the split form's staging (chunks of 2^16 events at n = 8, fewer
 * at larger n).  The kernels,
 * the partial layout and their reduction are bg_generate's, so every per-event output and
 * the totals equal bg_generate's bitwise.  count <= 2^24 and at most 2^18 + 1 workgroups
 * (count x lanes per event / workgroup size), else BG_EINVAL.  All calls on
 * one GPU share that array and it keeps the last call's contents: calls that overlap on one
 * GPU (other streams, other threads) race; order them.  Errors as bg_generate. */
int bg_generate_noalloc(const bg_config *cfg, int64_t count, const bg_inputs *in, const bg_outputs *out,
                        void *stream);

/* |A(sigma; h)|^2 for given physical momenta (Sec. 3, Eqs. 3.1, 3.2, 3.6).
 * mom [N][n][4] FP64, hel [N], order [N][n]; amp2_out [N] FP64.  Span invariants K^2
 * are formed in FP64 for both precisions.  N = 0 is a no-op.  Non-finite momenta give a
 * non-finite |A|^2 for that event only. */
int bg_amp2(int n, int prec, int64_t N, const double *mom, const uint32_t *hel,
            const uint8_t *order, double *amp2_out, void *stream);

/* Gradient of the log integrand weight (Eq. 3.8 without the cut step function and
 * without the sampling density),
 *   log w_int = log f(x1) + log f(x2) - log(2 s_hat) + log V_{n-2}(s_hat)
 *               + log(colour, helicity and ordering factors) + log |A|^2,
 * with respect to the RAMBO uniforms and x1, x2, by a hand-written adjoint of
 * closure, recursion, helicity vectors and RAMBO (|A|^2 is evaluated on the partonic
 * centre-of-mass momenta, so the longitudinal boost drops out).  The forward pass is
 * recomputed inside the kernel; log w_int matches bg_outputs.logw of bg_generate.
 * cfg: host pointer (n, prec, sqrt_s, use_pdf, pdf_a, pdf_b, alpha_s are used);
 * uniforms [N][4(n-2)], x12 [N][2] (ignored unless use_pdf), hel [N], order [N][n];
 * gout [N] (dL/dlog w, may be NULL = all ones); grad_u [N][4(n-2)], grad_x [N][2]
 * (zeros when use_pdf = 0) receive gout * d log w_int; logw [N] optional.
 * Events with |A|^2 = 0 or not finite (non-finite inputs) get log w = -inf and zero
 * gradients.
 * Supported for n = 4..12 in both precisions.  The recursion's reverse sweep runs one lane
 * per event for FP32 n <= 5 and FP64 n = 4, two lanes for FP32 n = 6..8 and FP64 n = 5, 6,
 * else four (a lane holds 4 / lanes Lorentz components of every current and its adjoint).  BG_ENOTSUP for real
 * polarisations and the dynamic scale. */
int bg_amp2_grad(const bg_config *cfg, int64_t N, const double *uniforms, const double *x12,
                 const uint32_t *hel, const uint8_t *order, const double *gout,
                 double *grad_u, double *grad_x, double *logw, void *stream);

/* Exact histograms of event weights (Sec. 4: the distributions of Fig. 3, accumulated over
 * many calls as in Fig. 2).  One axis bins one observable column of bg_outputs.obs
 * (0: H_T, 1: R_min) uniformly on [lo, hi) into nbins; each axis also has an underflow
 * (x < lo) and an overflow bin (x >= hi or NaN), so it owns nbins + 2 bins, in the order
 * underflow, 1..nbins, overflow; axes follow one another.  Per bin, sum w and sum w^2 over
 * the events with w != 0 are accumulated EXACTLY, as fixed-point integers of
 * BG_HIST_LIMBS limbs (2^-160 resolution; weights must be finite, non-negative and below
 * 2^112): in any order, over any number of calls, the totals are bitwise reproducible, and
 * bg_hist_read returns each as the correctly rounded double of the exact sum (the paper's
 * Kahan sums, without their residual error). */
typedef struct {
  int32_t column;  /* 0: H_T, 1: R_min */
  int32_t nbins;   /* >= 1; at most 400 bins (nbins + 2 summed over axes) per call */
  double lo, hi;   /* finite, lo < hi; bin b (1..nbins) covers lo + (b-1)(hi-lo)/nbins .. */
} bg_hist_axis;

#define BG_HIST_LIMBS 12

/* Adds N events (weight [N] FP64, obs [N][2] FP64, device) into limbs: a device array of
 * [sum over axes of (nbins + 2)][2][BG_HIST_LIMBS] int64 (per bin: sum w, then sum w^2),
 * zeroed by the caller before the first call and kept between calls.  N <= 2^30 per call.
 * naxes 1..8, axes a host array.  Errors: BG_EINVAL. */
int bg_hist_accumulate(int64_t N, const double *weight, const double *obs, int naxes, const bg_hist_axis *axes,
                       int64_t *limbs, void *stream);

/* out: device [sum over axes of (nbins + 2)][2] FP64: per bin (sum w, sum w^2), each the
 * correctly rounded double of its exact sum.  limbs are read only. */
int bg_hist_read(int naxes, const bg_hist_axis *axes, const int64_t *limbs, double *out, void *stream);

/* Validation of the per-event inputs that bg_amp2 and bg_amp2_grad take unchecked (the
 * ordering and helicity conventions above): writes to first_bad (a device int64_t) the
 * smallest event index whose order row [N][n] is not a permutation of 0..n-1 or whose
 * helicity word [N] has a bit at or above n, or -1 when every event is well formed.  Three
 * small kernels on `stream`; read first_bad after synchronising it.  N = 0 writes -1 (hel,
 * order may then be NULL).  Errors: BG_ENOTSUP (n outside 4..12), BG_EINVAL (N < 0 or
 * N > (2^31 - 1) * 256, NULL first_bad, NULL hel/order with N > 0). */
int bg_check_events(int n, int64_t N, const uint32_t *hel, const uint8_t *order, int64_t *first_bad,
                    void *stream);

/* Launch shape for one (n, prec) class: threads per workgroup (64, 128, 192 or 256) and
 * events per lane in one tile of the persistent multi-class launch (1..64; a tile holds
 * block * tile_iters events).  The autotuner writes these; (0, 0) restores the built-in
 * default.  Affects speed only: per-event outputs are identical for every shape, totals
 * agree within the compensated-sum bound.  Errors: BG_ENOTSUP, BG_EINVAL. */
int bg_set_launch(int n, int prec, int block, int tile_iters);
int bg_get_launch(int n, int prec, int *block, int *tile_iters);

/* Lanes of a wave that share one event in the single-class kernels of (n, prec) (bg_generate
 * and bg_amp2; bg_amp2_grad chooses its own, see there): 1 where the library holds the
 * one-lane form (FP32 n <= 9, FP64 n <= 6), 2 where it holds the two-lane form (FP32 n >= 9,
 * FP64 n >= 6), 4 where it holds the four-lane form (FP64 n >= 10), else BG_ENOTSUP; other
 * values BG_EINVAL; 0 restores the default (4 for FP64 n >= 10, 2 for FP32 n >= 10 and
 * FP64 n = 7..9, else 1).  With G lanes each holds 4/G of the four
 * Lorentz components of every current: 1/G of the registers, at the price of cross-lane
 * sums in every Minkowski product.  Affects speed only: |A|^2 agrees to the recursion
 * precision's rounding between the forms. */
int bg_set_lanes(int n, int prec, int lanes);
int bg_get_lanes(int n, int prec, int *lanes);

/* Form of the recursion in the single-class kernels of (n, prec) (bg_generate with helicity
 * states, and bg_amp2): 0 (default) the direct sums of Eqs. 3.1-3.2; 1 the W-tensor form of
 * Eqs. 3.3-3.4 (with the propagator 1/K^2 that Eq. 3.3 leaves implicit): a 4x4 tensor W per
 * span removes the double sum of the four-gluon terms, O(n^3) instead of O(n^4) work, at the
 * price of the tensors' storage.  One event takes 16 lanes (lane (mu, nu) holds W_mu,nu of
 * every span, the currents are shared through LDS); generation then stages the kinematics
 * as the split form does.  Built for FP32 n = 8, 10, 11, 12 and FP64 n = 6, 10 (else
 * BG_ENOTSUP); the persistent mixed launch, real polarisations and bg_amp2_grad keep the
 * direct form.  |A|^2 agrees with the direct form to the recursion precision's rounding. */
int bg_set_form(int n, int prec, int form);
int bg_get_form(int n, int prec, int *form);

/* Strategy for bg_generate calls with several classes (process-wide setting):
 *   0  each class's single-class kernel, one after another on the caller's stream;
 *   1  (default) the FP32 classes in one persistent launch (FP64 classes as in 0): the
 *      kinematics of the classes with n <= 8 in one kernel, then one persistent kernel
 *      whose one-wave workgroups take tiles, largest n first, from a shared queue (n >= 9
 *      generated two lanes per event, n <= 8 finished from the staged kinematics), then one
 *      reduction per class; falls back to 0 when the staging would exceed 8 GiB;
 *   2  the classes' single-class kernels on up to four library-owned side streams (created
 *      once per device at default priority, kept until the process ends), forked from and
 *      joined back into the caller's stream with events, so that classes too small to
 *      fill the GPU run side by side.
 * The autotuner times the three and records the fastest.  Per-event outputs are bitwise
 * identical in every mode (the persistent launch uses the two-lane form for n = 9);
 * totals agree within the compensated-sum bound.  Errors: BG_EINVAL for another value. */
int bg_set_mixed_launch(int mode);
int bg_get_mixed_launch(void);

/* Calibration of the roofline: the fused multiply-add rate (TFLOP/s, a multiply-add counted
 * as two) that this GPU's vector ALUs sustain in precision prec (32 or 64), measured with
 * chains of independent multiply-adds and nothing else, all compute units at eight waves per
 * SIMD (about 10 ms; synchronises the stream).  The published MI355X vector peaks count
 * packed FP32 (157.3 TFLOP/s); this library emits scalar FP32, whose ceiling is half that.
 * Errors: BG_EINVAL (prec, NULL), BG_EHIP. */
int bg_fma_rate(int prec, double *tflops, void *stream);

/* Static message for a status code. */
const char *bg_strerror(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int bg_version(void);

/* Identity of the sources the library was built from: the first 16 hexadecimal digits of a
 * sha256 over the kernel sources, this header and the build script with its compiler flags
 * (static string). */
const char *bg_source_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* BG_H */
