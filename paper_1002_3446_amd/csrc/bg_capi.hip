// C-ABI of libbg (include/bg.h): argument checking, per-class constants, launch shapes,
// stream-ordered workspace for the compensated reduction, and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/bg.h"
#include "bg_launch.hpp"

// Launchers of every (kind, n, prec, form) translation unit; weak, so that forms and
// multiplicities the library was not built with report BG_ENOTSUP.
#define BG_DECL_ONE(N, P)                                                                                  \
  __attribute__((weak)) hipError_t launch_generate_n##N##_p##P##_k0(const GenClass&, const GenWork&, int,  \
                                                                    hipStream_t);                         \
  __attribute__((weak)) hipError_t launch_amp2_n##N##_p##P##_k1(int64_t, const double*, const uint32_t*,  \
                                                                const uint8_t*, double*, int, hipStream_t); \
  __attribute__((weak)) hipError_t launch_grad_n##N##_p##P##_k2(const GradArgs&, int, hipStream_t);       \
  __attribute__((weak)) hipError_t launch_generate2_n##N##_p##P##_k0(const GenClass&, const GenWork&, int, \
                                                                     hipStream_t);                        \
  __attribute__((weak)) hipError_t launch_amp2_2_n##N##_p##P##_k1(int64_t, const double*, const uint32_t*, \
                                                                  const uint8_t*, double*, int, hipStream_t); \
  __attribute__((weak)) hipError_t launch_generate4_n##N##_p##P##_k0(const GenClass&, const GenWork&, int, \
                                                                     hipStream_t);                        \
  __attribute__((weak)) hipError_t launch_amp2_4_n##N##_p##P##_k1(int64_t, const double*, const uint32_t*, \
                                                                  const uint8_t*, double*, int, hipStream_t); \
  __attribute__((weak)) hipError_t launch_generate_real_n##N##_p##P##_k0(const GenClass&, const GenWork&, int, \
                                                                         hipStream_t); \
  __attribute__((weak)) hipError_t launch_generate_w_n##N##_p##P##_k0(const GenClass&, const GenWork&, int,  \
                                                                      hipStream_t);                         \
  __attribute__((weak)) hipError_t launch_amp2_w_n##N##_p##P##_k1(int64_t, const double*, const uint32_t*,   \
                                                                  const uint8_t*, double*, int, hipStream_t);
#define BG_DECL(N) BG_DECL_ONE(N, 32) BG_DECL_ONE(N, 64)
namespace bgk {
BG_DECL(4) BG_DECL(5) BG_DECL(6) BG_DECL(7) BG_DECL(8) BG_DECL(9) BG_DECL(10) BG_DECL(11) BG_DECL(12)
}

#ifndef BG_SOURCE_HASH
#define BG_SOURCE_HASH "unknown"
#endif

namespace {

using namespace bgk;

#define BG_ROW(N)                                                                                       \
  {{launch_generate_n##N##_p32_k0, launch_amp2_n##N##_p32_k1, launch_grad_n##N##_p32_k2,                \
    launch_generate2_n##N##_p32_k0, launch_amp2_2_n##N##_p32_k1, launch_generate_real_n##N##_p32_k0,    \
    launch_generate_w_n##N##_p32_k0, launch_amp2_w_n##N##_p32_k1, launch_generate4_n##N##_p32_k0,        \
    launch_amp2_4_n##N##_p32_k1},                                                                        \
   {launch_generate_n##N##_p64_k0, launch_amp2_n##N##_p64_k1, launch_grad_n##N##_p64_k2,                \
    launch_generate2_n##N##_p64_k0, launch_amp2_2_n##N##_p64_k1, launch_generate_real_n##N##_p64_k0,    \
    launch_generate_w_n##N##_p64_k0, launch_amp2_w_n##N##_p64_k1, launch_generate4_n##N##_p64_k0,        \
    launch_amp2_4_n##N##_p64_k1}}

const Launchers* table(int n, int prec) {
  static const Launchers t[9][2] = {BG_ROW(4),  BG_ROW(5),  BG_ROW(6), BG_ROW(7), BG_ROW(8),
                                    BG_ROW(9), BG_ROW(10), BG_ROW(11), BG_ROW(12)};
  if (n < 4 || n > 12) return nullptr;
  if (prec != 32 && prec != 64) return nullptr;
  return &t[n - 4][prec == 32 ? 0 : 1];
}

// launch shapes per (n, prec): threads per workgroup, and events per lane in one tile of
// the multi-class launch (cheap small-n events get longer tiles)
struct Shape {
  int block, tile_iters;
};
std::mutex g_shape_mu;
Shape g_shape[13][2];
int g_lanes[13][2];  // lanes per event of single-class kernels (0 = default_lanes)
int g_form[13][2];   // recursion form of single-class kernels: 0 direct, 1 W-tensor

int form_of(int n, int prec) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  return g_form[n][prec == 32 ? 0 : 1];
}

int lanes_of(int n, int prec) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  const int l = g_lanes[n][prec == 32 ? 0 : 1];
  return l ? l : default_lanes(n, prec);
}

Shape default_shape(int n) {
  static const int iters[13] = {0, 0, 0, 0, 8, 6, 4, 3, 2, 1, 1, 1, 1};
  return Shape{256, iters[n]};
}

Shape shape_of(int n, int prec) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  Shape s = g_shape[n][prec == 32 ? 0 : 1];
  if (s.block == 0) s = default_shape(n);
  return s;
}

// strategy for several classes in one call (bg_set_mixed_launch)
enum MixedMode { kSequential = 0, kPersistent = 1, kConcurrent = 2 };
std::atomic<int> g_mixed_mode{kPersistent};

// Side streams for concurrent classes: created once per device (default priority,
// non-blocking), kept until the process ends.
constexpr int kSideStreams = 4;
int side_streams(hipStream_t** out) {
  static std::mutex mu;
  static hipStream_t pool[64][kSideStreams];
  static bool ready[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BG_EHIP;
  std::lock_guard<std::mutex> lk(mu);
  if (!ready[dev]) {
    for (int i = 0; i < kSideStreams; ++i)
      if (hipStreamCreateWithFlags(&pool[dev][i], hipStreamNonBlocking) != hipSuccess) return BG_EHIP;
    ready[dev] = true;
  }
  *out = pool[dev];
  return BG_OK;
}

// rough relative cost of one event (FP32; FP64 about three times), for balancing classes
// over the side streams
double event_cost(int n, int prec) {
  static const double ns[13] = {0, 0, 0, 0, 0.31, 0.38, 0.47, 0.60, 0.75, 1.4, 2.7, 5.0, 8.7};
  return ns[n] * (prec == 64 ? 3.0 : 1.0);
}

// compute units of the current device (cached per device)
int cu_count() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lk(mu);
  if (cache[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cache[dev] = c;
  }
  return cache[dev];
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kHbarc2Pb = 0.3893793721e9;  // (hbar c)^2 in pb GeV^2
constexpr double kNc = 3.0;
constexpr double kMuZ = 91.188;  // GeV, the default reference scale (Sec. 4)

double lfact(int k) { return std::lgamma((double)k + 1.0); }

// log of the event-independent factors of the integrand weight (Eq. 3.8 with Eq. 3.7):
// flux 1/2, massless (n-2)-body volume constant, 1/(n-2)!, 2^n (n-1)! helicity and ordering
// factors, g^(2(n-2)) N^(n-2) / (4 (N^2-1)) colour factor, (hbar c)^2.
double log_weight_const(int n, double alpha_s) {
  const int nf = n - 2;
  const double lv = (4 - 3 * nf) * std::log(2 * kPi) + (nf - 1) * std::log(kPi / 2) - lfact(nf - 1) - lfact(nf - 2);
  const double g2 = 4 * kPi * alpha_s;
  const double lme = n * std::log(2.0) + lfact(n - 1) + (n - 2) * std::log(g2) + (n - 2) * std::log(kNc) -
                     std::log(4.0 * (kNc * kNc - 1.0));
  return lv - lfact(n - 2) + lme + std::log(kHbarc2Pb) - std::log(2.0);
}

// binomial(b, k)
double binom(int b, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (b - k + i) / i;
  return r;
}

int fill_class(const bg_config& c, int64_t count, const bg_inputs* in, const bg_outputs* out, GenClass& G) {
  if (c.n < 4 || c.n > 12 || (c.prec != 32 && c.prec != 64)) return BG_ENOTSUP;
  if (count < 0 || (c.polarisation != 0 && c.polarisation != 1) || !(c.sqrt_s > 0) || (c.use_pdf != 0 && c.use_pdf != 1) ||
      (c.random_order != 0 && c.random_order != 1) || !(c.alpha_s > 0) || !(c.pt_min >= 0) ||
      !(c.eta_max > 0) || !(c.dr_min >= 0) || (c.dynamic_scale != 0 && c.dynamic_scale != 1) || c.reserved != 0 ||
      !std::isfinite(c.pdf_da) || !std::isfinite(c.pdf_db) || !(c.mu0 < 1e300))
    return BG_EINVAL;
  std::memset(&G, 0, sizeof(G));
  G.count = count;
  G.first_event = c.first_event;
  G.key0 = (uint32_t)c.seed;
  G.key1 = (uint32_t)(c.seed >> 32);
  G.use_pdf = c.use_pdf;
  G.random_order = c.random_order;
  G.polarisation = c.polarisation;
  G.dynamic_scale = c.dynamic_scale;
  G.lmu0 = std::log(c.mu0 > 0 ? c.mu0 : kMuZ);
  G.log_alpha0 = std::log(c.alpha_s);
  G.sqrt_s = c.sqrt_s;
  G.pt_min = c.pt_min;
  G.eta_max = c.eta_max;
  G.dr_min = c.dr_min;
  double ratio = 1.0;
  if (c.use_pdf) {
    if (c.pdf_b < 0 || c.pdf_b > 16) return BG_EINVAL;
    double tau = c.tau_min;
    if (!(tau > 0)) tau = std::pow((c.n - 2) * c.pt_min / c.sqrt_s, 2);
    if (!(tau > 0 && tau < 1)) return BG_EINVAL;
    PdfParams& P = G.pdf;
    P.a = c.pdf_a;
    P.b = c.pdf_b;
    P.tau = tau;
    double ptau = 0.0, p1 = 0.0;
    for (int k = 0; k <= c.pdf_b; ++k) {
      const double e = c.pdf_a + k + 1.0;
      if (e == 0.0) return BG_EINVAL;
      P.coef[k] = binom(c.pdf_b, k) * ((k & 1) ? -1.0 : 1.0) / e;
    }
    for (int k = c.pdf_b; k >= 0; --k) {
      ptau = ptau * tau + P.coef[k];
      p1 += P.coef[k];
    }
    P.x0base = std::pow(tau, c.pdf_a + 1.0);
    P.Ftau = P.x0base * ptau;
    P.F1 = p1;
    P.Z = p1 - P.Ftau;
    if (!(P.Z > 0)) return BG_EINVAL;
    // branch point of the sampler: x_split = 0.2 (or the midpoint of [tau, 1) if tau >= 0.2)
    P.xsplit = tau < 0.2 ? 0.2 : 0.5 * (tau + 1.0);
    double psplit = 0.0;
    for (int k = c.pdf_b; k >= 0; --k) psplit = psplit * P.xsplit + P.coef[k];
    P.usplit = (std::pow(P.xsplit, c.pdf_a + 1.0) * psplit - P.Ftau) / P.Z;
    ratio = P.Z * P.Z;
  }
  G.log_const = log_weight_const(c.n, c.alpha_s);
  G.wconst = ratio * std::exp(G.log_const);
  if (in) {
    G.in_u = in->uniforms;
    G.in_x = in->x12;
    G.in_hel = in->hel;
    G.in_order = in->order;
  }
  if (out) {
    G.out.weight = out->weight;
    G.out.amp2 = out->amp2;
    G.out.obs = out->obs;
    G.out.pass = out->pass;
    G.out.momenta = out->momenta;
    G.out.hel = out->hel;
    G.out.order = out->order;
    G.out.x12 = out->x12;
    G.out.uniforms = out->uniforms;
    G.out.logw = out->logw;
  }
  return BG_OK;
}

int from_hip(hipError_t e) { return e == hipSuccess ? BG_OK : BG_EHIP; }

// ----------------------------------------------------------------------------------------
// Device workspace.  Every per-call buffer (compensated-sum partials, staging between the
// kinematics and recursion kernels, the gradient's intermediate adjoints, the multi-class
// work list) is allocated stream-ordered on the caller's stream from a memory pool the
// library creates once per device; the pool keeps up to kPoolKeep bytes reserved between
// calls, so that repeated calls do not map fresh device memory each time.
// ----------------------------------------------------------------------------------------
constexpr uint64_t kPoolKeep = uint64_t(4) << 30;

hipMemPool_t device_pool() {
  static std::mutex mu;
  static hipMemPool_t pools[64];
  static int state[64] = {0};  // 0 untried, 1 ready, -1 unavailable (use the default pool)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (state[dev] == 0) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    state[dev] = -1;
    if (hipMemPoolCreate(&pools[dev], &props) == hipSuccess) {
      uint64_t keep = kPoolKeep;
      (void)hipMemPoolSetAttribute(pools[dev], hipMemPoolAttrReleaseThreshold, &keep);
      state[dev] = 1;
    } else {
      (void)hipGetLastError();
    }
  }
  return state[dev] == 1 ? pools[dev] : nullptr;
}

int ws_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) return BG_OK;
  hipMemPool_t pool = device_pool();
  const hipError_t e = pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return BG_ENOMEM;
  }
  return BG_OK;
}

// Stream-ordered device workspace, released on the stream when the owner goes out of scope.
struct Workspace {
  void* p = nullptr;
  hipStream_t s;
  ~Workspace() {
    if (p) (void)hipFreeAsync(p, s);
  }
  double* d() const { return static_cast<double*>(p); }
};

// ----------------------------------------------------------------------------------------
// Inverse-CDF tables of the parton density (layout at pdf_sample).  The table is evaluated
// by a small device kernel (k_pdf_table), the same one the allocation-free entry point uses,
// so that both give bitwise the same parton fractions; the host evaluates it once as well,
// only to reject densities whose table would not be finite.  One table per distinct
// (pdf_a, pdf_b, tau) and device, built at first use (which synchronises the caller's stream
// once) and kept, immutable, until the process ends (10.5 KB each).
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_pdf_table(PdfParams P, double* out) {
  const int seg = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (seg < kPdfSegs) pdf_table_segment(P, seg, out + 4 * seg);
}

hipError_t launch_pdf_table(const PdfParams& P, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pdf_table, dim3((kPdfSegs + 63) / 64), dim3(64), 0, s, P, out);
  return hipGetLastError();
}

bool pdf_table_finite_host(const PdfParams& P) {
  double seg[4];
  for (int k = 0; k < kPdfSegs; ++k) {
    pdf_table_segment(P, k, seg);
    for (double v : seg)
      if (!std::isfinite(v)) return false;
  }
  return true;
}

int pdf_table(const PdfParams& P, const double** out, hipStream_t s) {
  struct Entry {
    int dev;
    double a, tau;
    int b;
    double* d;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BG_EHIP;
  std::lock_guard<std::mutex> lk(mu);
  for (const Entry& e : cache)
    if (e.dev == dev && e.a == P.a && e.b == P.b && e.tau == P.tau) {
      *out = e.d;
      return BG_OK;
    }
  if (!pdf_table_finite_host(P)) return BG_EINVAL;
  double* d = nullptr;
  if (hipMalloc((void**)&d, (size_t)kPdfSegs * 4 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return BG_ENOMEM;
  }
  if (launch_pdf_table(P, d, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(d);
    return BG_EHIP;
  }
  cache.push_back(Entry{dev, P.a, P.tau, P.b, d});
  *out = d;
  return BG_OK;
}

// ----------------------------------------------------------------------------------------
// Grids of the dynamic scale (ScaleGrid, bg_device.hpp): alpha_s at one loop,
//   alpha_s(mu) = alpha_s(mu0) / (1 + alpha_s(mu0) b0 ln(mu^2 / mu0^2)),  b0 = (33 - 2 n_f) / (12 pi),
// n_f = 5, and ln f(x, mu) = (a + da L) ln x + (b + db L) ln(1 - x), L = ln(mu / mu0), at the
// grid nodes; built on the host once per (alpha_s, mu0, a, b, da, db) and device, kept until
// the process ends (1 MB each).  BG_EINVAL when the Landau pole lies inside the grid.
// ----------------------------------------------------------------------------------------
int scale_grid(const bg_config& c, const GenClass& G, ScaleGrid& out) {
  struct Entry {
    int dev;
    double alpha_s, lmu0, a, da, db;
    int b;
    double* d;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BG_EHIP;
  const double a = c.use_pdf ? c.pdf_a : 0.0, da = c.use_pdf ? c.pdf_da : 0.0, db = c.use_pdf ? c.pdf_db : 0.0;
  const int b = c.use_pdf ? c.pdf_b : 0;
  out.lmu_lo = std::log(kGridMuLo);
  out.dlmu_alpha = (std::log(kGridMuHi) - out.lmu_lo) / (kAlphaNodes - 1);
  out.dlmu_pdf = (std::log(kGridMuHi) - out.lmu_lo) / (kGridMuNodes - 1);
  out.y_lo = std::log(kGridXLo) - std::log1p(-kGridXLo);
  out.dy = (std::log(kGridXHi) - std::log1p(-kGridXHi) - out.y_lo) / (kGridYNodes - 1);
  std::lock_guard<std::mutex> lk(mu);
  double* d = nullptr;
  for (const Entry& e : cache)
    if (e.dev == dev && e.alpha_s == c.alpha_s && e.lmu0 == G.lmu0 && e.a == a && e.b == b && e.da == da && e.db == db)
      d = e.d;
  if (!d) {
    const double b0 = (33.0 - 2.0 * 5.0) / (12.0 * kPi);
    std::vector<double> h((size_t)kAlphaNodes + (size_t)kGridMuNodes * kGridYNodes);
    for (int k = 0; k < kAlphaNodes; ++k) {
      const double den = 1.0 + c.alpha_s * b0 * 2.0 * (out.lmu_lo + k * out.dlmu_alpha - G.lmu0);
      if (!(den > 0.0)) return BG_EINVAL;
      h[k] = c.alpha_s / den;
    }
    for (int im = 0; im < kGridMuNodes; ++im) {
      const double L = out.lmu_lo + im * out.dlmu_pdf - G.lmu0;
      for (int iy = 0; iy < kGridYNodes; ++iy) {
        const double y = out.y_lo + iy * out.dy;
        const double lx = -std::log1p(std::exp(-y)), l1x = -std::log1p(std::exp(y));
        h[kAlphaNodes + (size_t)im * kGridYNodes + iy] = (a + da * L) * lx + (b + db * L) * l1x;
      }
    }
    for (double v : h)
      if (!std::isfinite(v)) return BG_EINVAL;
    if (hipMalloc((void**)&d, h.size() * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return BG_ENOMEM;
    }
    if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return BG_EHIP;
    }
    cache.push_back(Entry{dev, c.alpha_s, G.lmu0, a, da, db, b, d});
  }
  out.alpha = d;
  out.lnf = d + kAlphaNodes;
  return BG_OK;
}

// ----------------------------------------------------------------------------------------
// Single-class launches.
// ----------------------------------------------------------------------------------------
// Staging of the split forms: chunks of at most kStageChunk events (1.14 GB at n = 8, 1.68 GB
// at n = 12).  Every chunk costs two kernel boundaries, at which the GPU drains (the last
// workgroups of one kernel finish unevenly before the next kernel starts), so fewer, larger
// chunks waste less, up to the memory pool's 4 GiB release threshold (n = 8 FP32, 2^24
// events: 6.78 ms in chunks of 2^21, 6.59 ms in chunks of 2^22, 6.63 ms in 2^23, 6.76 ms in
// one chunk of 4.6 GB).
constexpr int64_t kStageChunk = int64_t(1) << 22;

struct ClassPlan {
  int lanes, block;
  bool wform, staged;  // W-tensor form; kinematics staged for a separate recursion kernel
  int64_t nblocks;  // workgroups = compensated partials
  GenerateFn fn;
};

int plan_class(const bg_config& c, const GenClass& G, ClassPlan& P) {
  const Launchers* L = table(c.n, c.prec);
  P.wform = !c.polarisation && form_of(c.n, c.prec) == 1;
  P.lanes = (c.polarisation || P.wform) ? 1 : lanes_of(c.n, c.prec);
  P.fn = c.polarisation ? L->generate_real
                        : (P.wform ? L->generate_w
                                   : (P.lanes == 4 ? L->generate4 : (P.lanes == 2 ? L->generate2 : L->generate)));
  if (!P.fn) return BG_ENOTSUP;
  // staged: the W-tensor form, the table classes, and every grouped form (kinematics in
  // their own kernel, one lane per event, instead of on every lane of a group)
  P.staged = P.wform || (P.lanes == 1 && split_form(c.n, c.prec)) || P.lanes > 1;
  P.block = (P.wform || P.lanes == 1) && P.staged ? kLdsLanes : shape_of(c.n, c.prec).block;
  P.nblocks = (P.lanes * G.count + P.block - 1) / P.block;
  return BG_OK;
}

// Persistent multi-class launch over the FP32 classes ks (see bg_multi.hip).  Returns
// BG_ENOTSUP, with nothing enqueued, when the classes' staging would exceed
// kMultiStageMax (the caller then runs them one after another).
constexpr size_t kMultiStageMax = size_t(8) << 30;

int generate_multi(const bg_config* cfgs, const GenClass* G, const bg_outputs* outs, const std::vector<int>& ks,
                   hipStream_t s) {
  if (!launch_generate_multi_p32) return BG_ENOTSUP;
  std::vector<int> order;  // staged classes first (kinematics workgroup order), then the others
  for (int k : ks)
    if (split_form(cfgs[k].n, 32)) order.push_back(k);
  const int nstaged = (int)order.size();
  for (int k : ks)
    if (!split_form(cfgs[k].n, 32)) order.push_back(k);
  std::vector<MultiClass> mcs(order.size());
  int64_t kin_blocks = 0, stage_words = 0;
  for (size_t c = 0; c < order.size(); ++c) {
    const int k = order[c];
    MultiClass& m = mcs[c];
    std::memset(&m, 0, sizeof(m));
    m.C = G[k];
    m.n = cfgs[k].n;
    m.acc = outs[k].acc;
    m.staged = (int)c < nstaged;
    if (m.staged) {
      m.kin_begin = kin_blocks;
      m.stage_off = stage_words;
      kin_blocks += (G[k].count + kKinBlock - 1) / kKinBlock;
      stage_words += (G[k].count + kLdsLanes - 1) / kLdsLanes * kLdsLanes * split_words(m.n);
    }
  }
  if ((size_t)stage_words * sizeof(double) > kMultiStageMax) return BG_ENOTSUP;
  // tiles by decreasing n: the most expensive events start first
  std::vector<int> byn(order.size());
  for (size_t c = 0; c < byn.size(); ++c) byn[c] = (int)c;
  std::stable_sort(byn.begin(), byn.end(), [&](int a, int b) { return mcs[a].n > mcs[b].n; });
  std::vector<Tile> tiles;
  for (int c : byn) {
    MultiClass& m = mcs[c];
    const int per_iter = m.staged ? kMultiBlock : kMultiBlock / 2;
    const int64_t tile = (int64_t)per_iter * shape_of(m.n, 32).tile_iters;
    m.tile_begin = (int)tiles.size();
    for (int64_t f = 0; f < m.C.count; f += tile)
      tiles.push_back(Tile{f, (int32_t)std::min<int64_t>(tile, m.C.count - f), (int32_t)c});
    m.tile_end = (int)tiles.size();
  }
  if (tiles.empty()) return BG_OK;
  if (tiles.size() > (size_t)0x7fffffff) return BG_EINVAL;
  const size_t o_cls = 0;
  const size_t o_tiles = (o_cls + mcs.size() * sizeof(MultiClass) + 255) & ~size_t(255);
  const size_t o_ctr = (o_tiles + tiles.size() * sizeof(Tile) + 255) & ~size_t(255);
  const size_t o_part = o_ctr + 256;
  const size_t bytes = o_part + tiles.size() * 4 * sizeof(double);
  std::vector<unsigned char> blob(o_part, 0);  // classes, tiles and a zero counter
  std::memcpy(blob.data() + o_cls, mcs.data(), mcs.size() * sizeof(MultiClass));
  std::memcpy(blob.data() + o_tiles, tiles.data(), tiles.size() * sizeof(Tile));
  Workspace ws{nullptr, s}, stage{nullptr, s};
  int st = ws_alloc(&ws.p, bytes, s);
  if (st == BG_OK) st = ws_alloc(&stage.p, (size_t)stage_words * sizeof(double), s);
  if (st != BG_OK) return st;
  unsigned char* w = static_cast<unsigned char*>(ws.p);
  // pageable source: the copy is staged before hipMemcpyAsync returns, so blob may go
  st = from_hip(hipMemcpyAsync(w, blob.data(), o_part, hipMemcpyHostToDevice, s));
  if (st != BG_OK) return st;
  const int grid = cu_count() * 4;  // one one-wave workgroup per SIMD
  return from_hip(launch_generate_multi_p32((const MultiClass*)(w + o_cls), (int)mcs.size(), nstaged, kin_blocks,
                                            (const Tile*)(w + o_tiles), (int)tiles.size(), (int*)(w + o_ctr),
                                            stage.d(), (double*)(w + o_part), grid, s));
}

// Input check behind bg_check_events: the smallest index of an event whose ordering is not a
// permutation of 0..n-1 or whose helicity word has bits at or above n.
__global__ void k_check_init(int64_t* first_bad) {
  if (threadIdx.x == 0) first_bad[0] = INT64_MAX;
}

__global__ __launch_bounds__(256) void k_check_events(int n, int64_t count, const uint32_t* __restrict__ hel,
                                                      const uint8_t* __restrict__ order, int64_t* first_bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  bool ok = (hel[i] >> n) == 0u;
  uint32_t seen = 0u;
  for (int t = 0; t < n; ++t) {
    const uint32_t l = order[i * n + t];
    ok = ok && l < (uint32_t)n && ((seen >> l) & 1u) == 0u;
    seen |= 1u << (l & 31u);
  }
  if (!ok) atomicMin(reinterpret_cast<unsigned long long*>(first_bad), (unsigned long long)i);
}

__global__ void k_check_final(int64_t* first_bad) {
  if (threadIdx.x == 0 && first_bad[0] == INT64_MAX) first_bad[0] = -1;
}

// ----------------------------------------------------------------------------------------
// Allocation-free generation (bg_generate_noalloc).  Every device buffer such a call needs
// lives in one file-scope array, `scratch`, which each GPU holds once until the process
// ends (about 27 MiB): the inverse-CDF table of the density last used, the compensated-sum
// partials and their second level, and the staging of the split form (chunks of
// kNoAllocStage events).  Host code never uses the array's name as an address: its device
// address is looked up once per device (noalloc_scratch) and passed to the kernels.
// ----------------------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxEvents = int64_t(1) << 24;
constexpr int64_t kNoAllocStage = int64_t(1) << 16;
constexpr size_t round256(size_t doubles) { return (doubles + 31) / 32 * 32; }
constexpr size_t kNoAllocParts = (size_t)(kNoAllocMaxEvents / 64 + 1);  // workgroups of >= 64 events
constexpr size_t kOffPdf = 0;
constexpr size_t kOffParts = kOffPdf + round256((size_t)kPdfSegs * 4);
constexpr size_t kOffLevel2 = kOffParts + round256(kNoAllocParts * 4);
constexpr size_t kOffStage = kOffLevel2 + round256((size_t)kFinalizeGroups * 4);
constexpr size_t kScratchDoubles = kOffStage + round256((size_t)kNoAllocStage * split_words(8));

static __device__ __align__(256) double scratch[kScratchDoubles];

struct NoAllocDevice {
  double* ptr = nullptr;  // device address of this GPU's scratch
  bool pdf_valid = false;  // the density whose table scratch holds
  double a = 0.0, tau = 0.0;
  int b = 0;
};

// This device's scratch address (looked up with the device current, once per device) and
// its table record.
int noalloc_device(NoAllocDevice** out) {
  static std::mutex mu;
  static NoAllocDevice devs[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BG_EHIP;
  std::lock_guard<std::mutex> lk(mu);
  if (!devs[dev].ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return BG_EHIP;
    }
    devs[dev].ptr = static_cast<double*>(p);
  }
  *out = &devs[dev];
  return BG_OK;
}

}  // namespace

extern "C" {

int bg_generate_noalloc(const bg_config* cfg, int64_t count, const bg_inputs* in, const bg_outputs* out,
                        void* stream) {
  if (!cfg || !out) return BG_EINVAL;
  if (count > kNoAllocMaxEvents) return BG_EINVAL;
  if (cfg->dynamic_scale) return BG_ENOTSUP;
  GenClass G;
  ClassPlan P;
  int st = fill_class(*cfg, count, in, out, G);
  if (st == BG_OK) st = plan_class(*cfg, G, P);
  if (st != BG_OK) return st;
  if (count == 0) return BG_OK;
  if ((size_t)P.nblocks > kNoAllocParts) return BG_EINVAL;
  NoAllocDevice* D = nullptr;
  if ((st = noalloc_device(&D)) != BG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (G.use_pdf && !G.in_x) {
    // the table of this density, rebuilt in scratch when the density changed
    const PdfParams& Q = G.pdf;
    if (!(D->pdf_valid && D->a == Q.a && D->b == Q.b && D->tau == Q.tau)) {
      if (!pdf_table_finite_host(Q)) return BG_EINVAL;
      if ((st = from_hip(launch_pdf_table(Q, D->ptr + kOffPdf, s))) != BG_OK) return st;
      D->pdf_valid = true;
      D->a = Q.a;
      D->b = Q.b;
      D->tau = Q.tau;
    }
    G.pdf.tab = D->ptr + kOffPdf;
  }
  // the staging region holds kNoAllocStage events of n = 8; larger n take shorter chunks
  const int64_t cap = (int64_t)(kNoAllocStage * split_words(8) / split_words(cfg->n)) / 256 * 256;
  GenWork W{out->acc ? D->ptr + kOffParts : nullptr, P.staged ? D->ptr + kOffStage : nullptr,
            P.staged ? cap : 0};
  st = from_hip(P.fn(G, W, P.block, s));
  if (st == BG_OK && W.partials)
    st = from_hip(launch_finalize(W.partials, P.nblocks, D->ptr + kOffLevel2, out->acc, s));
  return st;
}


int bg_fma_rate(int prec, double* tflops, void* stream) {
  if ((prec != 32 && prec != 64) || !tflops) return BG_EINVAL;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BG_EHIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) return BG_EHIP;
  double r = 0.0;
  const int st = from_hip(measure_fma_rate(prec, 4096, ncu, &r, (hipStream_t)stream));
  if (st == BG_OK) *tflops = r * 1e-12;
  return st;
}

int bg_version(void) { return 10100; }

const char* bg_source_hash(void) { return BG_SOURCE_HASH; }

const char* bg_strerror(int status) {
  switch (status) {
    case BG_OK: return "ok";
    case BG_EINVAL: return "invalid argument";
    case BG_ENOTSUP: return "unsupported multiplicity, precision or lane form";
    case BG_EHIP: return "HIP runtime error";
    case BG_ENOMEM: return "device workspace allocation failed";
    default: return "unknown status";
  }
}

int bg_set_mixed_launch(int mode) {
  if (mode != kSequential && mode != kPersistent && mode != kConcurrent) return BG_EINVAL;
  g_mixed_mode.store(mode);
  return BG_OK;
}

int bg_get_mixed_launch(void) { return g_mixed_mode.load(); }

int bg_set_launch(int n, int prec, int block, int tile_iters) {
  if (!table(n, prec)) return BG_ENOTSUP;
  if (block == 0 && tile_iters == 0) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape[n][prec == 32 ? 0 : 1] = Shape{0, 0};
    return BG_OK;
  }
  if (block < 64 || block > 256 || block % 64 != 0 || tile_iters < 1 || tile_iters > 64) return BG_EINVAL;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_shape[n][prec == 32 ? 0 : 1] = Shape{block, tile_iters};
  return BG_OK;
}

int bg_set_lanes(int n, int prec, int lanes) {
  const Launchers* L = table(n, prec);
  if (!L) return BG_ENOTSUP;
  if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4) return BG_EINVAL;
  if (lanes == 1 && !(L->generate && L->amp2)) return BG_ENOTSUP;
  if (lanes == 2 && !(L->generate2 && L->amp2_2)) return BG_ENOTSUP;
  if (lanes == 4 && !(L->generate4 && L->amp2_4)) return BG_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_lanes[n][prec == 32 ? 0 : 1] = lanes;
  return BG_OK;
}

int bg_set_form(int n, int prec, int form) {
  const Launchers* L = table(n, prec);
  if (!L) return BG_ENOTSUP;
  if (form != 0 && form != 1) return BG_EINVAL;
  if (form == 1 && !(L->generate_w && L->amp2_w)) return BG_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_form[n][prec == 32 ? 0 : 1] = form;
  return BG_OK;
}

int bg_get_form(int n, int prec, int* form) {
  if (!table(n, prec)) return BG_ENOTSUP;
  if (!form) return BG_EINVAL;
  *form = form_of(n, prec);
  return BG_OK;
}

int bg_get_lanes(int n, int prec, int* lanes) {
  if (!table(n, prec)) return BG_ENOTSUP;
  if (!lanes) return BG_EINVAL;
  *lanes = lanes_of(n, prec);
  return BG_OK;
}

int bg_get_launch(int n, int prec, int* block, int* tile_iters) {
  if (!table(n, prec)) return BG_ENOTSUP;
  if (!block || !tile_iters) return BG_EINVAL;
  const Shape s = shape_of(n, prec);
  *block = s.block;
  *tile_iters = s.tile_iters;
  return BG_OK;
}

int bg_generate(const bg_config* cfgs, int ncfg, const int64_t* counts, const bg_inputs* ins,
                const bg_outputs* outs, void* stream) {
  if (!cfgs || !counts || !outs || ncfg < 1 || ncfg > 16) return BG_EINVAL;
  GenClass G[16];
  ClassPlan P[16];
  for (int k = 0; k < ncfg; ++k) {
    int st = fill_class(cfgs[k], counts[k], ins ? &ins[k] : nullptr, &outs[k], G[k]);
    if (st == BG_OK) st = plan_class(cfgs[k], G[k], P[k]);
    if (st != BG_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  // inverse-CDF tables of the classes that sample x1, x2; grids of dynamic-scale classes
  for (int k = 0; k < ncfg; ++k) {
    if (G[k].dynamic_scale && G[k].count > 0) {
      const int st = scale_grid(cfgs[k], G[k], G[k].grid);
      if (st != BG_OK) return st;
    }
    if (!(G[k].use_pdf && !G[k].in_x && G[k].count > 0)) continue;
    const int st = pdf_table(G[k].pdf, &G[k].pdf.tab, s);
    if (st != BG_OK) return st;
  }
  const int mode = ncfg > 1 ? g_mixed_mode.load() : kSequential;
  // persistent mode: the FP32 classes in one launch; FP64 classes run their single-class
  // kernels below
  bool multi32 = false;
  if (mode == kPersistent) {
    std::vector<int> ks;
    for (int k = 0; k < ncfg; ++k)
      if (cfgs[k].prec == 32 && cfgs[k].polarisation == 0 && G[k].count > 0) ks.push_back(k);
    if (ks.size() > 1) {
      const int st = generate_multi(cfgs, G, outs, ks, s);
      if (st != BG_OK && st != BG_ENOTSUP) return st;
      multi32 = st == BG_OK;
    }
  }
  std::vector<int> todo;
  for (int k = 0; k < ncfg; ++k)
    if (G[k].count > 0 && !(multi32 && cfgs[k].prec == 32 && cfgs[k].polarisation == 0)) todo.push_back(k);
  if (todo.empty()) return BG_OK;
  // compensated-sum partials and staging buffers, allocated on the caller's stream before
  // any fork and released on it after the join
  size_t off[16], soff[16];
  int64_t scap[16];
  size_t bytes = 0;
  for (int k : todo) {
    off[k] = bytes;
    if (outs[k].acc) bytes += ((size_t)P[k].nblocks + kFinalizeGroups) * 4 * sizeof(double);
    scap[k] = 0;
  }
  const bool concurrent = mode == kConcurrent && todo.size() > 1;
  // the split form's staging: one buffer per class when classes may run side by side,
  // else one buffer reused by every class in turn
  size_t shared_stage = 0;
  for (int k : todo) {
    if (!P[k].staged) continue;
    scap[k] = std::min<int64_t>(kStageChunk, (G[k].count + 255) / 256 * 256);  // a multiple of 256
    const size_t sb = (size_t)scap[k] * split_words(cfgs[k].n) * sizeof(double);
    if (concurrent) {
      soff[k] = bytes;
      bytes += sb;
    } else {
      shared_stage = std::max(shared_stage, sb);
    }
  }
  if (!concurrent)
    for (int k : todo) soff[k] = bytes;
  bytes += shared_stage;
  Workspace ws{nullptr, s};
  if (int st = ws_alloc(&ws.p, bytes, s); st != BG_OK) return st;
  // the one-lane recursion prefetches the tile half a resident round ahead (two workgroups per
  // CU): a full round ahead, more than half of the prefetched lines left L2 before their use
  // (the recursion kernel read 58% more from HBM, for the same time)
  auto run_class = [&](int k, hipStream_t t) {
    GenWork W{outs[k].acc ? ws.d() + off[k] / sizeof(double) : nullptr,
              scap[k] > 0 ? ws.d() + soff[k] / sizeof(double) : nullptr, scap[k], (int64_t)cu_count() * 2};
    int st = from_hip(P[k].fn(G[k], W, P[k].block, t));
    if (st == BG_OK && W.partials)
      st = from_hip(launch_finalize(W.partials, P[k].nblocks, W.partials + 4 * P[k].nblocks, outs[k].acc, t));
    return st;
  };
  if (!concurrent) {
    for (int k : todo) {
      const int st = run_class(k, s);
      if (st != BG_OK) return st;
    }
    return BG_OK;
  }
  // concurrent mode: classes spread over the side streams (largest estimated work first,
  // each to the least loaded stream), forked from and joined back into the caller's stream
  hipStream_t* side = nullptr;
  int st = side_streams(&side);
  if (st != BG_OK) return st;
  std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) {
    return G[a].count * event_cost(cfgs[a].n, cfgs[a].prec) > G[b].count * event_cost(cfgs[b].n, cfgs[b].prec);
  });
  hipEvent_t fork, join[kSideStreams];
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return BG_EHIP;
  int nev = 0;
  for (; nev < kSideStreams; ++nev)
    if (hipEventCreateWithFlags(&join[nev], hipEventDisableTiming) != hipSuccess) break;
  double load[kSideStreams] = {0.0};
  bool used[kSideStreams] = {false};
  st = nev == kSideStreams ? from_hip(hipEventRecord(fork, s)) : BG_EHIP;
  for (size_t c = 0; c < todo.size() && st == BG_OK; ++c) {
    const int k = todo[c];
    const int t = (int)(std::min_element(load, load + kSideStreams) - load);
    if (!used[t]) {
      st = from_hip(hipStreamWaitEvent(side[t], fork, 0));
      used[t] = true;
    }
    load[t] += G[k].count * event_cost(cfgs[k].n, cfgs[k].prec);
    if (st == BG_OK) st = run_class(k, side[t]);
  }
  // join every stream that received work, also after a failed launch
  for (int t = 0; t < kSideStreams && t < nev; ++t) {
    if (!used[t]) continue;
    const int j = from_hip(hipEventRecord(join[t], side[t]));
    const int w = j == BG_OK ? from_hip(hipStreamWaitEvent(s, join[t], 0)) : j;
    if (st == BG_OK) st = w;
  }
  (void)hipEventDestroy(fork);
  for (int t = 0; t < nev; ++t) (void)hipEventDestroy(join[t]);
  return st;
}

}  // extern "C"

namespace {

int hist_axes(int naxes, const bg_hist_axis* axes, HistAxes& A) {
  if (naxes < 1 || naxes > kHistMaxAxes || !axes) return BG_EINVAL;
  std::memset(&A, 0, sizeof(A));
  A.naxes = naxes;
  int total = 0;
  for (int a = 0; a < naxes; ++a) {
    const bg_hist_axis& x = axes[a];
    if ((x.column != 0 && x.column != 1) || x.nbins < 1 || !(std::isfinite(x.lo) && std::isfinite(x.hi)) ||
        !(x.lo < x.hi))
      return BG_EINVAL;
    A.axis[a] = HistAxis{x.column, x.nbins, total, x.lo, x.hi};
    total += x.nbins + 2;
    if (total > kHistMaxBinsTotal) return BG_EINVAL;
  }
  A.total_bins = total;
  return BG_OK;
}

}  // namespace

extern "C" {

int bg_hist_accumulate(int64_t N, const double* weight, const double* obs, int naxes, const bg_hist_axis* axes,
                       int64_t* limbs, void* stream) {
  HistAxes A;
  int st = hist_axes(naxes, axes, A);
  if (st != BG_OK) return st;
  if (N < 0 || N > (int64_t(1) << 30) || !limbs) return BG_EINVAL;
  if (N == 0) return BG_OK;
  if (!weight || !obs) return BG_EINVAL;
  return from_hip(launch_hist_accumulate(N, weight, obs, A, limbs, cu_count(), (hipStream_t)stream));
}

int bg_hist_read(int naxes, const bg_hist_axis* axes, const int64_t* limbs, double* out, void* stream) {
  HistAxes A;
  int st = hist_axes(naxes, axes, A);
  if (st != BG_OK) return st;
  if (!limbs || !out) return BG_EINVAL;
  return from_hip(launch_hist_read(A, limbs, out, (hipStream_t)stream));
}

int bg_amp2(int n, int prec, int64_t N, const double* mom, const uint32_t* hel, const uint8_t* order,
            double* amp2_out, void* stream) {
  const Launchers* L = table(n, prec);
  if (!L) return BG_ENOTSUP;
  if (N < 0) return BG_EINVAL;
  const int lanes = lanes_of(n, prec);
  const Amp2Fn f = form_of(n, prec) == 1 ? L->amp2_w : (lanes == 4 ? L->amp2_4 : (lanes == 2 ? L->amp2_2 : L->amp2));
  if (!f) return BG_ENOTSUP;
  if (N == 0) return BG_OK;
  if (!mom || !hel || !order || !amp2_out) return BG_EINVAL;
  const Shape sh = shape_of(n, prec);
  return from_hip(f(N, mom, hel, order, amp2_out, sh.block, (hipStream_t)stream));
}

int bg_check_events(int n, int64_t N, const uint32_t* hel, const uint8_t* order, int64_t* first_bad, void* stream) {
  if (n < 4 || n > 12) return BG_ENOTSUP;
  if (N < 0 || N > (int64_t)0x7fffffff * 256 || !first_bad || (N > 0 && (!hel || !order))) return BG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_check_init, dim3(1), dim3(64), 0, s, first_bad);
  if (N > 0)
    hipLaunchKernelGGL(k_check_events, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, n, N, hel, order, first_bad);
  hipLaunchKernelGGL(k_check_final, dim3(1), dim3(64), 0, s, first_bad);
  return from_hip(hipGetLastError());
}

int bg_amp2_grad(const bg_config* cfg, int64_t N, const double* uniforms, const double* x12, const uint32_t* hel,
                 const uint8_t* order, const double* gout, double* grad_u, double* grad_x, double* logw,
                 void* stream) {
  if (!cfg) return BG_EINVAL;
  const Launchers* L = table(cfg->n, cfg->prec);
  if (!L) return BG_ENOTSUP;
  if (N < 0) return BG_EINVAL;
  if (!L->grad) return BG_ENOTSUP;
  if (N == 0) return BG_OK;
  if (!uniforms || !hel || !order || !grad_u || !grad_x || (cfg->use_pdf && !x12)) return BG_EINVAL;
  if (!(cfg->sqrt_s > 0) || !(cfg->alpha_s > 0) || (cfg->use_pdf != 0 && cfg->use_pdf != 1)) return BG_EINVAL;
  if (cfg->polarisation != 0 || cfg->dynamic_scale != 0) return BG_ENOTSUP;
  GradArgs G{};
  G.count = N;
  G.sqrt_s = cfg->sqrt_s;
  G.use_pdf = cfg->use_pdf;
  G.pdf_a = cfg->pdf_a;
  G.pdf_b = cfg->pdf_b;
  G.u = uniforms;
  G.x12 = x12;
  G.hel = hel;
  G.order = order;
  G.gout = gout;
  G.grad_u = grad_u;
  G.grad_x = grad_x;
  G.logw = logw;
  G.log_const = log_weight_const(cfg->n, cfg->alpha_s);
  hipStream_t s = (hipStream_t)stream;
  Workspace ws{nullptr, s};
  // the recursion's adjoints between the two gradient kernels: 12 (n - 1) + 1 words per event
  if (int st = ws_alloc(&ws.p, (size_t)N * (12 * (cfg->n - 1) + 1) * sizeof(double), s); st != BG_OK) return st;
  G.pbuf = ws.d();
  const Shape sh = shape_of(cfg->n, cfg->prec);
  return from_hip(L->grad(G, sh.block, s));
}

}  // extern "C"
