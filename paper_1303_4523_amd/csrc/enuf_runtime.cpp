// enuf_runtime.cpp -- host side of the ENUF C ABI: argument validation, window
// and influence tables, FFT factorisation, device buffers and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/enuf.h"
#include "enuf_dpd.h"
#include "enuf_internal.h"

using namespace enuf;

namespace {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

#define HIP_OR_RETURN(call, code)                                             \
  do {                                                                        \
    hipError_t _e = (call);                                                   \
    if (_e != hipSuccess) {                                                   \
      set_error(std::string(#call) + ": " + hipGetErrorString(_e));           \
      return code;                                                            \
    }                                                                         \
  } while (0)

// Modified Bessel function I0 by its power series sum (x/2)^{2k} / (k!)^2
// (all terms positive; long double keeps ~18 digits for the arguments used).
long double bessel_i0(long double x) {
  const long double h = x * x / 4.0L;
  long double term = 1.0L, sum = 1.0L;
  for (int k = 1; k < 500; ++k) {
    term *= h / ((long double)k * (long double)k);
    sum += term;
    if (term < sum * 1e-21L) break;
  }
  return sum;
}

bool factor_235(int n, FftPlan *pl) {
  pl->n = n;
  pl->npass = 0;
  int m = n;
  const int order[5] = {8, 4, 2, 3, 5};  // fewest passes first: each pass is an LDS round trip
  for (int oi = 0; oi < 5; ++oi) {
    const int r = order[oi];
    while (m % r == 0) {
      if (pl->npass >= kMaxRadixPasses) return false;
      pl->radix[pl->npass++] = r;
      m /= r;
    }
  }
  return m == 1;
}

}  // namespace

namespace {

size_t arena_slot(size_t n) { return ((n == 0 ? 16 : n) + 255) & ~(size_t)255; }

size_t arena_bytes(const size_t *sizes, int n) {
  size_t t = 0;
  for (int k = 0; k < n; ++k) t += arena_slot(sizes[k]);
  return t;
}

// Event timing of one kernel class (ENUF_K_* ids) over at most `cap`
// launches: a pair of events per launch, summed by total().
struct EventTimer {
  KernelTimer t;
  std::vector<hipEvent_t> ev;
  KernelTimer *active() { return t.kernel >= 0 ? &t : nullptr; }
  void drop() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    t = KernelTimer();
  }
  // kernel < 0 stops timing.  False if the events cannot be created.
  bool start(int kernel, int cap) {
    drop();
    if (kernel < 0) return true;
    ev.resize(2 * (size_t)cap);
    for (size_t k = 0; k < ev.size(); ++k) {
      if (hipEventCreate(&ev[k]) != hipSuccess) {
        ev.resize(k);
        drop();
        return false;
      }
    }
    t.kernel = kernel;
    t.cap = cap;
    t.count = 0;
    t.ev = ev.data();
    return true;
  }
  // Milliseconds summed over the recorded launches (the stream that holds
  // them must have been synchronised).
  hipError_t total(double *ms, int *launches) const {
    double sum = 0.0;
    for (int k = 0; k < t.count; ++k) {
      float m = 0.0f;
      const hipError_t e = hipEventElapsedTime(&m, ev[2 * k], ev[2 * k + 1]);
      if (e != hipSuccess) return e;
      sum += m;
    }
    *ms = sum;
    *launches = t.count;
    return hipSuccess;
  }
  ~EventTimer() { drop(); }
};

bool valid_timer_args(int kernel, int max_launches) {
  return kernel < 0 || (kernel <= ENUF_K_DPD_POST && max_launches >= 1 && max_launches <= (1 << 20));
}

}  // namespace

struct enuf_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  double L = 0, alpha = 0, sigma = 0, r_cut = 0, lambda = 0;
  int p = 0, M = 0, Kc = 0;
  int precision = ENUF_FP64, window = ENUF_WINDOW_KB;
  size_t max_lds = 0;
  int part_slots = 1;      // gather partial slots allocated per (charge, x offset)
  int max_parts = 1;       // partial spectra the spectrum buffer holds (plane parts)
  ComputeConfig cfg{};
  ComputeBuffers buf{};
  std::vector<void *> allocations;
  size_t bytes = 0;
  EventTimer timer;  // enuf_plan_time_kernel
  int concurrent = 1;                    // real-space term beside the mesh passes
  hipStream_t side = nullptr;            // created at the first overlapped evaluation
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;

  // All buffers in one device allocation (one hipMalloc / hipFree per
  // object), each at a 256-byte aligned offset.  False on failure.
  bool alloc_arena(const size_t *sizes, int n, void **ptrs) {
    const size_t total = arena_bytes(sizes, n);
    void *base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) return false;
    allocations.push_back(base);
    bytes += total;
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
      ptrs[k] = (char *)base + off;
      off += arena_slot(sizes[k]);
    }
    return true;
  }
  ~enuf_plan() {
    if (side) (void)hipStreamSynchronize(side);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (side) (void)hipStreamDestroy(side);
    for (void *ptr : allocations) (void)hipFree(ptr);
  }
};

namespace {

WindowParams make_window(int kind, int p, double sigma) {
  WindowParams w{};
  w.kind = kind;
  w.p = p;
  w.b = M_PI * (2.0 - 1.0 / sigma);
  w.c1 = 1.0 / (1.0 - std::exp(-2.0 * w.b * p));
  w.inv_sinh_bp = 1.0 / std::sinh(w.b * p);
  const double bg = 2.0 * sigma * p / ((2.0 * sigma - 1.0) * M_PI);
  w.inv_bg = 1.0 / bg;
  return w;
}

// Fourier transform of the normalised window at xi = k / M:
//   Kaiser-Bessel  Phi(xi) = I0(p sqrt(b^2 - (2 pi xi)^2)) * pi p / sinh(b p)
//   Gaussian       Phi(xi) = sqrt(pi b_G) exp(-b_G pi^2 xi^2)
long double window_hat(const WindowParams &w, long double xi) {
  if (w.kind == ENUF_WINDOW_GAUSS) {
    const long double bg = 1.0L / (long double)w.inv_bg;
    return std::sqrt((long double)M_PI * bg) * std::exp(-bg * (long double)M_PI * (long double)M_PI * xi * xi);
  }
  const long double b = w.b, p = w.p;
  const long double om = 2.0L * (long double)M_PI * xi;
  const long double arg = p * std::sqrt(b * b - om * om);
  return bessel_i0(arg) * (long double)M_PI * p / std::sinh(b * p);
}

// Normalised window phi(u) (phi(0) = 1) and phi'(u) in long double, for the
// host-side series fit.  Kaiser-Bessel: p sinh(b s)/(s sinh(b p)),
// s = sqrt(p^2 - u^2) (an even function of s, hence entire in u); its
// derivative -p u (b s cosh(b s) - sinh(b s)) / (s^3 sinh(b p)), summed as a
// series for small b s.  Gaussian: exp(-u^2 / b_G).
void window_exact(const WindowParams &w, long double u, long double *val, long double *der) {
  if (w.kind == ENUF_WINDOW_GAUSS) {
    const long double ib = w.inv_bg;
    const long double g = std::exp(-u * u * ib);
    *val = g;
    *der = -2.0L * u * ib * g;
    return;
  }
  const long double p = w.p, b = w.b;
  const long double isb = 1.0L / std::sinh(b * p);
  long double s2 = p * p - u * u;
  if (s2 < 0) s2 = 0;
  const long double s = std::sqrt(s2), z = b * s;
  if (z > 0.5L) {
    *val = p * std::sinh(z) / s * isb;
    *der = -p * u * (z * std::cosh(z) - std::sinh(z)) / (s2 * s) * isb;
  } else {
    // sinh(z)/z = sum z^{2m}/(2m+1)!;  (z cosh z - sinh z)/z^3 = sum z^{2m}/((2m+3)(2m+1)!)
    long double a = 1.0L, h = 1.0L / 3.0L, ta = 1.0L, th = 1.0L / 3.0L;
    for (int k = 1; k < 20; ++k) {
      ta *= z * z / ((2.0L * k) * (2.0L * k + 1.0L));
      th *= z * z / ((2.0L * k) * (2.0L * k + 3.0L));
      a += ta;
      h += th;
    }
    *val = p * b * a * isb;
    *der = -p * u * b * b * b * h * isb;
  }
}

// Chebyshev series of the window on each of the 2p unit intervals: offset s,
// x = 2 frac - 1, u = frac + p - 1 - s.  coef[s (D+1) + k] holds the value
// series; coef[2p (D+1) + s D + k] the series of d phi/du.  The degree is the
// smallest meeting the tolerance of the precision on a test grid.
int fit_window_series(const WindowParams &w, int fp32, std::vector<long double> *coef) {
  const int P2 = 2 * w.p;
  const long double tol_v = fp32 ? 1e-8L : 4e-15L, tol_d = fp32 ? 1e-6L : 1e-12L;
  int D = 4;
  for (;; ++D) {
    coef->assign((size_t)P2 * (2 * D + 1), 0.0L);
    long double ev = 0, ed = 0;
    const int n = D + 1;
    for (int s = 0; s < P2; ++s) {
      long double *c = coef->data() + (size_t)s * (D + 1);
      long double *d = coef->data() + (size_t)P2 * (D + 1) + (size_t)s * D;
      std::vector<long double> f(n), dd(D + 1, 0.0L);
      for (int m = 0; m < n; ++m) {
        const long double x = std::cos((long double)M_PI * (m + 0.5L) / n);
        long double v, dv;
        window_exact(w, x / 2 + w.p - 0.5L - s, &v, &dv);
        f[m] = v;
      }
      for (int k = 0; k <= D; ++k) {
        long double acc = 0;
        for (int m = 0; m < n; ++m) acc += f[m] * std::cos((long double)M_PI * k * (m + 0.5L) / n);
        c[k] = 2.0L * acc / n;
      }
      c[0] *= 0.5L;
      // derivative series d/dx, then d/du = 2 d/dx
      if (D >= 1) {
        dd[D - 1] = 2.0L * D * c[D];
        for (int k = D - 1; k >= 1; --k) dd[k - 1] = (k + 1 <= D ? dd[k + 1] : 0.0L) + 2.0L * k * c[k];
        dd[0] *= 0.5L;
      }
      for (int k = 0; k < D; ++k) d[k] = 2.0L * dd[k];
      for (int t = 0; t <= 256; ++t) {
        const long double x = -1.0L + t / 128.0L;
        long double v, dv;
        window_exact(w, x / 2 + w.p - 0.5L - s, &v, &dv);
        long double b1 = 0, b2 = 0;
        for (int k = D; k >= 1; --k) { const long double tt = c[k] + 2 * x * b1 - b2; b2 = b1; b1 = tt; }
        const long double sv = c[0] + x * b1 - b2;
        b1 = b2 = 0;
        for (int k = D - 1; k >= 1; --k) { const long double tt = d[k] + 2 * x * b1 - b2; b2 = b1; b1 = tt; }
        const long double sd = D >= 1 ? d[0] + x * b1 - b2 : 0.0L;
        ev = std::max(ev, std::fabs(sv - v));
        ed = std::max(ed, std::fabs(sd - dv));
      }
    }
    if ((ev < tol_v && ed < tol_d) || D >= kMaxChebDeg) break;
  }
  return D;
}

// The fits depend only on the window (kind, p, shape) and the precision:
// they are computed once per process and reused by every plan.
int cached_window_series(const WindowParams &w, int fp32, std::vector<long double> *coef) {
  struct Fit {
    int D;
    std::vector<long double> coef;
  };
  static std::mutex mu;
  static std::map<std::tuple<int, int, double, double, int>, Fit> cache;
  const auto key = std::make_tuple(w.kind, w.p, w.b, w.inv_bg, fp32);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it == cache.end()) {
    Fit f;
    f.D = fit_window_series(w, fp32, &f.coef);
    it = cache.emplace(key, std::move(f)).first;
  }
  *coef = it->second.coef;
  return it->second.D;
}

// Device layout of the window series for one precision: value series and
// derivative series, both at stride D + 1 (the derivative's last coefficient
// 0).  Returns the degree D.
int window_table(const WindowParams &w, int fp32, std::vector<long double> *coef) {
  std::vector<long double> fit;
  const int D = cached_window_series(w, fp32, &fit);
  const int P2 = 2 * w.p;
  coef->assign((size_t)P2 * 2 * (D + 1), 0.0L);
  for (int s = 0; s < P2; ++s) {
    for (int k = 0; k <= D; ++k) (*coef)[(size_t)s * (D + 1) + k] = fit[(size_t)s * (D + 1) + k];
    for (int k = 0; k < D; ++k)
      (*coef)[(size_t)(P2 + s) * (D + 1) + k] = fit[(size_t)P2 * (D + 1) + (size_t)s * D + k];
  }
  return D;
}

}  // namespace

namespace enuf {

int plan_tables(const ComputeConfig &c, int precision, PlanTables *t) {
  const int Kc = c.mesh.Kc, M = c.mesh.M, nky = 2 * Kc - 1;
  const WindowParams &w = c.mesh.win;
  t->atab.resize(nky);
  const long double aL = (long double)c.alpha * c.L;
  for (int i = 0; i < nky; ++i) {
    const long double k = (long double)(i - (Kc - 1));
    const long double ph = window_hat(w, k / (long double)M);
    t->atab[i] = (double)(std::exp(-(long double)M_PI * (long double)M_PI * k * k / (aL * aL)) / (ph * ph));
  }
  t->tw64.resize(M);
  t->tw32.resize(M);
  for (int m = 0; m < M; ++m) {
    const long double ang = -2.0L * (long double)M_PI * (long double)m / (long double)M;
    t->tw64[m] = make_double2((double)std::cos(ang), (double)std::sin(ang));
    t->tw32[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  std::vector<long double> coef;
  const int fp32 = precision == ENUF_MIXED;
  t->cheb_deg = window_table(w, fp32, &coef);
  t->wcoef64.clear();
  t->wcoef32.clear();
  if (fp32) {
    t->wcoef32.resize(coef.size());
    for (size_t k = 0; k < coef.size(); ++k) t->wcoef32[k] = (float)coef[k];
  } else {
    t->wcoef64.resize(coef.size());
    for (size_t k = 0; k < coef.size(); ++k) t->wcoef64[k] = (double)coef[k];
  }
  return ENUF_OK;
}

}  // namespace enuf

namespace {

int upload_tables(enuf_plan *pl) {
  PlanTables t;
  plan_tables(pl->cfg, pl->precision, &t);
  pl->cfg.mesh.cheb_deg = t.cheb_deg;
  const int M = pl->M, nky = 2 * pl->Kc - 1;
  HIP_OR_RETURN(hipMemcpy(pl->buf.atab, t.atab.data(), nky * sizeof(double), hipMemcpyHostToDevice), ENUF_EDEVICE);
  HIP_OR_RETURN(hipMemcpy(pl->buf.tw64, t.tw64.data(), M * sizeof(double2), hipMemcpyHostToDevice), ENUF_EDEVICE);
  HIP_OR_RETURN(hipMemcpy(pl->buf.tw32, t.tw32.data(), M * sizeof(float2), hipMemcpyHostToDevice), ENUF_EDEVICE);
  if (!t.wcoef32.empty())
    HIP_OR_RETURN(hipMemcpy(pl->buf.wcoef32, t.wcoef32.data(), t.wcoef32.size() * sizeof(float),
                            hipMemcpyHostToDevice), ENUF_EDEVICE);
  if (!t.wcoef64.empty())
    HIP_OR_RETURN(hipMemcpy(pl->buf.wcoef64, t.wcoef64.data(), t.wcoef64.size() * sizeof(double),
                            hipMemcpyHostToDevice), ENUF_EDEVICE);
  return ENUF_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Work-groups per plane of the spread and gather passes: about 128 planes x
// parts, half the CUs of the device, which leaves the other half to the pair
// and real-space kernels that run beside the mesh passes; at most kMaxParts.
// ENUF_MESH_PARTS (1..8) overrides the choice (tuning and testing).
int mesh_parts(int M) {
  if (const char *v = std::getenv("ENUF_MESH_PARTS")) {
    const int n = std::atoi(v);
    if (n >= 1) return std::min(kMaxParts, n);
  }
  return std::max(1, std::min(kMaxParts, 128 / M));
}

// Work-groups per plane of the backward pass: as many as the spread's, or
// ENUF_BWD_PARTS (1..8) (tuning and testing).
int mesh_bparts(int parts) {
  if (const char *v = std::getenv("ENUF_BWD_PARTS")) {
    const int n = std::atoi(v);
    if (n >= 1) return std::min(kMaxParts, n);
  }
  return parts;
}

// Work-groups per ky row of the x pass: about 64 in all, each a range of kz
// lines.  ENUF_X_SPLIT (1..Kc) overrides the choice (tuning and testing).
int mesh_xsplit(int Kc, int nky) {
  if (const char *v = std::getenv("ENUF_X_SPLIT")) {
    const int n = std::atoi(v);
    if (n >= 1) return std::min(Kc, n);
  }
  return std::max(1, std::min(Kc, 64 / nky));
}

// Fixed-point scale of the partial spectra relative to the spread's: the
// spectrum of a plane is bounded by sum |q| (2p)^3, and up to 8 parts add.
double mesh_gscale_factor(int p) {
  int e = 0;
  while ((1 << e) < 2 * p) ++e;
  return std::ldexp(1.0, -(3 * e + 3));
}

}  // namespace

namespace {

// Geometry that fixes the plan's buffer sizes.
struct PlanGeom {
  int ncell = 1, cap = 1, xcap = 1, part_slots = 0, nblk = 1;
};

// Returns false when no row chunking of the plane passes fits in max_lds.
bool plan_geometry(int64_t N, double box, int p, int M, int Kc, double r_cut, size_t max_lds, PlanGeom *g) {
  int ncell = (int)std::floor(box / r_cut);
  ncell = ncell < 1 ? 1 : (ncell > 1024 ? 1024 : ncell);
  const double mean = (double)N / ((double)ncell * ncell * ncell);
  g->ncell = ncell;
  g->cap = (int)std::ceil(mean + 6.0 * std::sqrt(mean) + 16.0);
  const double xmean = (double)N / ((double)M * kXSub);  // charges per x-cell sub-bin, at most
  g->xcap = (int)std::ceil(xmean + 6.0 * std::sqrt(xmean) + 8.0);
  g->nblk = (int)((N + kPrepThreads - 1) / kPrepThreads);
  // the gather partials are sized for the largest series degree in either precision
  MeshParams m{};
  m.M = M; m.Mp = M + 1; m.Mz = M + 1; m.Kc = Kc; m.nky = 2 * Kc - 1;
  m.win.p = p;
  m.cheb_deg = kMaxChebDeg;
  g->part_slots = 0;
  for (int prec = ENUF_FP64; prec <= ENUF_MIXED; ++prec) {
    MeshParams t = m;
    if (mesh_choose_rows(t, prec, max_lds)) g->part_slots = t.nslot > g->part_slots ? t.nslot : g->part_slots;
  }
  return g->part_slots > 0;
}

constexpr int kPlanBuffers = 24;

// Bytes of every device buffer of a plan, in allocation order.
std::array<size_t, kPlanBuffers> plan_buffer_bytes(int64_t N, int p, int M, int Kc, const PlanGeom &g) {
  const size_t n = (size_t)N, nblk = (size_t)g.nblk, P2 = 2 * (size_t)p, nky = 2 * (size_t)Kc - 1;
  const size_t ncell3 = (size_t)g.ncell * g.ncell * g.ncell, cap = (size_t)g.cap;
  return {nblk * sizeof(int),                                 // blk_cnt
          nblk * 3 * sizeof(double),                          // blk_sums
          sizeof(DevScalars),                                 // sc
          n * sizeof(double4),                                // xq
          n * sizeof(int),                                    // idx
          n * sizeof(int),                                    // slot
          2 * ncell3 * sizeof(int),                           // ccnt (two sets)
          ncell3 * cap * sizeof(double4),                     // cgrid
          ncell3 * cap * sizeof(float4),                      // cpre
          n * 3 * sizeof(unsigned long long),                 // freal
          n * 2 * sizeof(unsigned long long),                 // ereal
          nblk * 2 * sizeof(long long),                       // blk_er
          (size_t)(mesh_parts(M) + 1) * M * nky * (size_t)Kc * 16,  // gzy: partial spectra + field
          (size_t)M * nky * (size_t)Kc * sizeof(double2),     // gzx
          nky * (size_t)Kc * sizeof(double),                  // epart: per (ky, kz) line
          n * P2 * (size_t)g.part_slots * sizeof(double4),    // part
          nblk * sizeof(double),                              // blk_eg
          2 * (size_t)M * kXSub * sizeof(int),                // xcnt (two sets)
          (size_t)M * kXSub * (size_t)g.xcap * sizeof(int),   // xslot
          P2 * (2 * kMaxChebDeg + 2) * sizeof(double),        // wcoef64
          P2 * (2 * kMaxChebDeg + 2) * sizeof(float),         // wcoef32
          nky * sizeof(double),                               // atab
          (size_t)M * sizeof(double2),                        // tw64
          (size_t)M * sizeof(float2)};                        // tw32
}

// LDS bytes per block the plans of this device may use: the device's limit
// less a reserve for the kernels' static LDS, or the lower value of
// ENUF_MAX_LDS_BYTES.  0 if the device cannot be queried.
size_t lds_budget(int device) {
  constexpr size_t kStaticLdsReserve = 256;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return 0;
  if ((size_t)lds <= kStaticLdsReserve) return 0;
  size_t v = (size_t)lds - kStaticLdsReserve;
  if (const char *cap = std::getenv("ENUF_MAX_LDS_BYTES")) {
    const long long c = std::atoll(cap);
    if (c > 0 && (size_t)c < v) v = (size_t)c;
  }
  return v;
}

}  // namespace

extern "C" {

const char *enuf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Host-side argument checks of a plan (no device call); the FFT factorisation
// of M in *fp.  ENUF_OK or ENUF_EINVAL with the message set.
int check_plan_args(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc, double r_cut,
                    double lambda, FftPlan *fp) {
  if (N < 1 || N > (int64_t)1 << 28) { set_error("N must be in [1, 2^28]"); return ENUF_EINVAL; }
  if (!finite_pos(box)) { set_error("box must be finite and > 0"); return ENUF_EINVAL; }
  if (!finite_pos(alpha)) { set_error("alpha must be finite and > 0"); return ENUF_EINVAL; }
  if (!(std::isfinite(sigma) && sigma >= 1.0)) { set_error("sigma must be finite and >= 1"); return ENUF_EINVAL; }
  if (p < 1 || p > 15) { set_error("p must be in [1, 15]"); return ENUF_EINVAL; }
  if (M < 4 || M % 2 != 0 || M > 4096) { set_error("M must be even and in [4, 4096]"); return ENUF_EINVAL; }
  *fp = FftPlan{};
  if (!factor_235(M, fp)) { set_error("M must be of the form 2^a 3^b 5^c"); return ENUF_EINVAL; }
  if (fft_max_butterflies(*fp) > kPassThreads) {
    set_error("M = " + std::to_string(M) + " needs more than " + std::to_string(kPassThreads) +
              " butterflies per FFT pass (too few factors 4 and 8)");
    return ENUF_EINVAL;
  }
  if (2 * p > M / 2) { set_error("need 2p <= M/2"); return ENUF_EINVAL; }
  if (Kc < 1 || (double)Kc > (double)M / (2.0 * sigma)) { set_error("need 1 <= Kc <= M/(2 sigma)"); return ENUF_EINVAL; }
  if (!finite_pos(r_cut) || r_cut > 0.5 * box) { set_error("need 0 < r_cut <= box/2"); return ENUF_EINVAL; }
  if (!(std::isfinite(lambda) && lambda >= 0.0)) { set_error("lambda must be finite and >= 0"); return ENUF_EINVAL; }
  return ENUF_OK;
}

// Configuration and buffer geometry of a plan with checked arguments (FP64,
// Kaiser-Bessel window, gradient forces, default parts); the mesh passes'
// row chunking is chosen later for the precision (plan_rows).  False (message
// set) when no row chunking fits the LDS budget.
bool plan_config(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc, double r_cut,
                 double lambda, const FftPlan &fp, size_t max_lds, ComputeConfig *cfg, PlanGeom *g) {
  ComputeConfig &c = *cfg;
  c = ComputeConfig{};
  c.N = N;
  c.nblk = (int)((N + kPrepThreads - 1) / kPrepThreads);
  c.L = box; c.alpha = alpha; c.r_cut = r_cut; c.lambda = lambda;
  c.precision = ENUF_FP64;
  MeshParams &m = c.mesh;
  m.M = M; m.Mp = M + 1; m.Mz = M + 1; m.Kc = Kc; m.nky = 2 * Kc - 1;
  m.L = box; m.m_over_l = (double)M / box;
  m.win = make_window(ENUF_WINDOW_KB, p, sigma);
  m.fft = fp;
  m.parts = mesh_parts(M);
  m.bparts = mesh_bparts(m.parts);
  m.xsplit = mesh_xsplit(Kc, m.nky);
  m.gscale_f = mesh_gscale_factor(p);
  if (!plan_geometry(N, box, p, M, Kc, r_cut, max_lds, g)) {
    set_error("mesh too large: no row chunking of the plane passes fits in " + std::to_string(max_lds) +
              " bytes of LDS");
    return false;
  }
  // the real-space scan numbers cell slots in 32 bits
  if ((double)g->ncell * g->ncell * g->ncell * g->cap >= 2147483648.0) {
    set_error("real-space cell grid too large: ncell^3 x capacity >= 2^31 slots (box / r_cut too large)");
    return false;
  }
  c.cells.ncell = g->ncell;
  c.cells.cap = g->cap;
  c.cells.inv_cell = (double)g->ncell / box;
  m.xcap = g->xcap;
  m.cheb_deg = kMaxChebDeg;
  m.rows = M;
  m.nchunk = 1;
  m.nslot = 1;
  m.stage = kStage;
  mesh_lds_bytes(m, 0, &c.lds_fwd, &c.lds_x, &c.lds_bwd);
  return true;
}

// Row chunking of the mesh passes for a precision (false: it does not fit).
bool plan_rows(ComputeConfig *c, int precision, size_t max_lds, int part_slots) {
  MeshParams &m = c->mesh;
  if (!mesh_choose_rows(m, precision, max_lds) || m.nslot > part_slots) return false;
  mesh_lds_bytes(m, precision, &c->lds_fwd, &c->lds_x, &c->lds_bwd);
  return true;
}

// The plan's buffers at the offsets of one arena (ptr[k]: buffer k of plan_buffer_bytes).
ComputeBuffers carve_buffers(void *const *ptr) {
  ComputeBuffers b{};
  b.blk_cnt = (int *)ptr[0];
  b.blk_sums = (double *)ptr[1];
  b.sc = (DevScalars *)ptr[2];
  b.xq = (double4 *)ptr[3];
  b.idx = (int *)ptr[4];
  b.slot = (int *)ptr[5];
  b.ccnt = (int *)ptr[6];
  b.cgrid = (double4 *)ptr[7];
  b.cpre = (float4 *)ptr[8];
  b.freal = (unsigned long long *)ptr[9];
  b.ereal = (unsigned long long *)ptr[10];
  b.blk_er = (long long *)ptr[11];
  b.gzy = ptr[12];
  b.gzx = ptr[13];
  b.epart = (double *)ptr[14];
  b.part = (double4 *)ptr[15];
  b.blk_eg = (double *)ptr[16];
  b.xcnt = (int *)ptr[17];
  b.xslot = (int *)ptr[18];
  b.wcoef64 = (double *)ptr[19];
  b.wcoef32 = (float *)ptr[20];
  b.atab = (double *)ptr[21];
  b.tw64 = (double2 *)ptr[22];
  b.tw32 = (float2 *)ptr[23];
  return b;
}

// Buffers that must hold zeros before the first evaluation (the kernels keep
// them so between evaluations): (pointer, bytes) pairs, returns their count.
int zeroed_buffers(const ComputeConfig &c, const ComputeBuffers &b, void **ptr, size_t *bytes) {
  const size_t n = (size_t)c.N, nc = (size_t)c.cells.ncell;
  ptr[0] = b.sc;    bytes[0] = sizeof(DevScalars);
  ptr[1] = b.freal; bytes[1] = n * 3 * sizeof(unsigned long long);
  ptr[2] = b.ccnt;  bytes[2] = 2 * nc * nc * nc * sizeof(int);
  ptr[3] = b.xcnt;  bytes[3] = 2 * (size_t)c.mesh.M * kXSub * sizeof(int);
  return 4;
}

// Dynamic-LDS limits of the mesh kernels, raised once per process.
hipError_t configure_once(size_t max_lds) {
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lock(mu);
  if (done) return hipSuccess;
  const hipError_t e = configure_kernels(max_lds);
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

extern "C" {

enuf_plan *enuf_plan_create(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc,
                            double r_cut, double lambda) {
  g_last_error.clear();
  // ---- validation (host only; no device call before it passes) ----
  FftPlan fp{};
  if (check_plan_args(N, box, alpha, p, sigma, M, Kc, r_cut, lambda, &fp) != ENUF_OK) return nullptr;

  enuf_plan *pl = new enuf_plan();
  pl->N = N; pl->L = box; pl->alpha = alpha; pl->sigma = sigma; pl->r_cut = r_cut; pl->lambda = lambda;
  pl->p = p; pl->M = M; pl->Kc = Kc;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    set_error("hipGetDevice failed");
    delete pl;
    return nullptr;
  }
  pl->max_lds = lds_budget(pl->device);
  if (pl->max_lds == 0) {
    set_error("hipDeviceGetAttribute failed");
    delete pl;
    return nullptr;
  }
  PlanGeom g;
  if (!plan_config(N, box, alpha, p, sigma, M, Kc, r_cut, lambda, fp, pl->max_lds, &pl->cfg, &g)) {
    delete pl;
    return nullptr;
  }
  pl->max_parts = pl->cfg.mesh.parts;  // the spectrum buffer holds this many partial spectra
  pl->part_slots = g.part_slots;

  const std::array<size_t, kPlanBuffers> sz = plan_buffer_bytes(N, p, M, Kc, g);
  void *ptr[kPlanBuffers];
  if (!pl->alloc_arena(sz.data(), kPlanBuffers, ptr)) {
    set_error("device allocation failed");
    delete pl;
    return nullptr;
  }
  pl->buf = carve_buffers(ptr);
  void *zp[8];
  size_t zb[8];
  const int nz = zeroed_buffers(pl->cfg, pl->buf, zp, zb);
  for (int k = 0; k < nz; ++k) {
    if (hipMemset(zp[k], 0, zb[k]) != hipSuccess) {
      set_error("hipMemset failed");
      delete pl;
      return nullptr;
    }
  }
  if (upload_tables(pl) != ENUF_OK) {
    delete pl;
    return nullptr;
  }
  if (!plan_rows(&pl->cfg, ENUF_FP64, pl->max_lds, pl->part_slots)) {
    // FP64 does not fit; the plan stays usable after switching to the mixed mode
    MeshParams &m = pl->cfg.mesh;
    m.rows = M;
    m.nchunk = 1;
    m.nslot = 1;
    m.stage = kStage;
    mesh_lds_bytes(m, ENUF_FP64, &pl->cfg.lds_fwd, &pl->cfg.lds_x, &pl->cfg.lds_bwd);
  }
  if (configure_once(pl->max_lds) != hipSuccess) {
    set_error("hipFuncSetAttribute failed");
    delete pl;
    return nullptr;
  }
  if (hipStreamSynchronize(nullptr) != hipSuccess) {
    set_error("device synchronisation after plan setup failed");
    delete pl;
    return nullptr;
  }
  return pl;
}

void enuf_destroy(enuf_plan *plan) {
  if (!plan) return;
  (void)hipStreamSynchronize(plan->stream);
  delete plan;
}

int enuf_plan_set_stream(enuf_plan *plan, void *hip_stream) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  plan->stream = (hipStream_t)hip_stream;
  return ENUF_OK;
}

int enuf_plan_set_options(enuf_plan *plan, int precision, int window) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  if (precision != ENUF_FP64 && precision != ENUF_MIXED) { set_error("unknown precision"); return ENUF_EINVAL; }
  if (window != ENUF_WINDOW_KB && window != ENUF_WINDOW_GAUSS) { set_error("unknown window"); return ENUF_EINVAL; }
  // the stream may still read the old tables
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  const int old_prec = plan->precision, old_win = plan->window;
  plan->precision = precision;
  plan->window = window;
  plan->cfg.precision = precision;
  plan->cfg.mesh.win = make_window(window, plan->p, plan->sigma);
  int rc = upload_tables(plan);
  size_t f = 0, x = 0, bw = 0;
  const MeshParams old_mesh = plan->cfg.mesh;
  if (rc == ENUF_OK) {
    MeshParams &m = plan->cfg.mesh;
    if (!mesh_choose_rows(m, precision, plan->max_lds) || m.nslot > plan->part_slots) {
      set_error("mesh too large for the LDS in this precision (" + std::to_string(plan->max_lds) + " bytes)");
      rc = ENUF_EINVAL;
    } else {
      mesh_lds_bytes(m, precision, &f, &x, &bw);
    }
  }
  if (rc != ENUF_OK) {  // restore the previous, valid configuration
    plan->precision = old_prec;
    plan->window = old_win;
    plan->cfg.precision = old_prec;
    plan->cfg.mesh.win = make_window(old_win, plan->p, plan->sigma);
    (void)upload_tables(plan);
    plan->cfg.mesh.rows = old_mesh.rows;
    plan->cfg.mesh.nchunk = old_mesh.nchunk;
    plan->cfg.mesh.nslot = old_mesh.nslot;
    plan->cfg.mesh.stage = old_mesh.stage;
    return rc;
  }
  plan->cfg.lds_fwd = f;
  plan->cfg.lds_x = x;
  plan->cfg.lds_bwd = bw;
  return ENUF_OK;
}

int enuf_plan_set_parts(enuf_plan *plan, int parts) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  if (parts < 1 || parts > plan->max_parts) {
    set_error("parts must be in [1, " + std::to_string(plan->max_parts) + "]");
    return ENUF_EINVAL;
  }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  plan->cfg.mesh.parts = parts;
  plan->cfg.mesh.bparts = parts;
  return ENUF_OK;
}

int enuf_plan_set_concurrency(enuf_plan *plan, int enable) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  plan->concurrent = enable ? 1 : 0;
  return ENUF_OK;
}

int enuf_plan_set_force_mode(enuf_plan *plan, int mode) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  if (mode != ENUF_FORCE_GRADIENT && mode != ENUF_FORCE_IK) { set_error("unknown force mode"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  MeshParams m = plan->cfg.mesh;
  m.ik = mode == ENUF_FORCE_IK ? 1 : 0;
  if (!mesh_choose_rows(m, plan->precision, plan->max_lds) || m.nslot > plan->part_slots) {
    set_error("mesh too large for the LDS with this force mode and precision");
    return ENUF_EINVAL;
  }
  size_t f = 0, x = 0, bw = 0;
  mesh_lds_bytes(m, plan->precision, &f, &x, &bw);
  plan->cfg.mesh = m;
  plan->cfg.lds_fwd = f;
  plan->cfg.lds_x = x;
  plan->cfg.lds_bwd = bw;
  return ENUF_OK;
}

static int compute_impl(enuf_plan *plan, const double *pos, const double *q, double *forces,
                        double *energy, double *energy5) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  if (!pos || !q || !forces || (!energy && !energy5)) { set_error("NULL buffer"); return ENUF_EINVAL; }
  const ComputeConfig &c = plan->cfg;
  if (c.lds_fwd > plan->max_lds || c.lds_bwd > plan->max_lds || c.lds_x > plan->max_lds) {
    set_error("mesh too large for one LDS plane in this precision");
    return ENUF_EINVAL;
  }
  int dev = -1;
  HIP_OR_RETURN(hipGetDevice(&dev), ENUF_EDEVICE);
  if (dev != plan->device) HIP_OR_RETURN(hipSetDevice(plan->device), ENUF_EDEVICE);
  KernelTimer *tm = plan->timer.active();
  hipStream_t st = plan->stream;
  // the real-space term on the side stream, beside the mesh passes (no
  // cross-stream events inside a capture, and one stream while timing)
  bool fork = plan->concurrent && !tm;
  if (fork) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    fork = hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
  }
  hipError_t e = hipSuccess;
  if (fork && !plan->side) {
    e = hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->join_ev, hipEventDisableTiming);
  }
  if (e == hipSuccess && fork) {
    e = launch_prep(c, plan->buf, pos, q, st, nullptr);
    if (e == hipSuccess) e = hipEventRecord(plan->fork_ev, st);
    if (e == hipSuccess) e = launch_recip(c, plan->buf, c.N, st, nullptr);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->side, plan->fork_ev, 0);
    if (e == hipSuccess) e = launch_real(c, plan->buf, c.N, plan->side, nullptr);
    if (e == hipSuccess) e = hipEventRecord(plan->join_ev, plan->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->join_ev, 0);
    if (e == hipSuccess) e = launch_combine(c, plan->buf, forces, energy, energy5, FinishArgs(), st, nullptr);
  } else if (e == hipSuccess) {
    e = launch_compute(c, plan->buf, pos, q, forces, energy, energy5, st, tm);
  }
  if (dev != plan->device) (void)hipSetDevice(dev);
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return ENUF_EDEVICE;
  }
  return ENUF_OK;
}

int enuf_compute(enuf_plan *plan, const double *pos, const double *q, double *forces, double *energy) {
  return compute_impl(plan, pos, q, forces, energy, nullptr);
}

int enuf_compute_components(enuf_plan *plan, const double *pos, const double *q, double *forces,
                            double *energy5) {
  return compute_impl(plan, pos, q, forces, nullptr, energy5);
}

int enuf_plan_status(enuf_plan *plan, int *status) {
  if (!plan || !status) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  int s = 0;
  HIP_OR_RETURN(hipMemcpy(&s, &plan->buf.sc->status, sizeof(int), hipMemcpyDeviceToHost), ENUF_EDEVICE);
  const int zero = 0;
  HIP_OR_RETURN(hipMemcpy(&plan->buf.sc->status, &zero, sizeof(int), hipMemcpyHostToDevice), ENUF_EDEVICE);
  *status = s;
  return ENUF_OK;
}

size_t enuf_plan_footprint_bytes(const enuf_plan *plan) { return plan ? plan->bytes : 0; }

int enuf_plan_time_kernel(enuf_plan *plan, int kernel, int max_launches) {
  if (!plan) { set_error("NULL plan"); return ENUF_EINVAL; }
  if (!valid_timer_args(kernel, max_launches)) { set_error("invalid kernel id or launch count"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  if (!plan->timer.start(kernel, max_launches)) { set_error("hipEventCreate failed"); return ENUF_EDEVICE; }
  return ENUF_OK;
}

int enuf_plan_kernel_time(enuf_plan *plan, double *total_ms, int *launches) {
  if (!plan || !total_ms || !launches) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(plan->stream), ENUF_EDEVICE);
  HIP_OR_RETURN(plan->timer.total(total_ms, launches), ENUF_EDEVICE);
  return ENUF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One evaluation that allocates nothing: the plan's buffers are carved out of
// a fixed device array instead of a hipMalloc'd arena.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // ENUF_NOALLOC_SCRATCH_BYTES in enuf.h
constexpr int kNoAllocMaxM = 256;
constexpr int kMaxDevices = 64;

// Every device the library runs on holds its own copy until the process ends.
// Host code never names it in a device context: the address each device
// gives for it (scratch_address) is what kernels and copies receive.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of scratch, looked up once per
// device with that device current.
int scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index out of range for the static scratch table");
    return ENUF_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return ENUF_EDEVICE;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return ENUF_OK;
}

// Small host tables reach the device as kernel arguments (no copy from host
// memory, no staging allocation): 500 words per launch.
constexpr int kFillWords = 500;
struct FillChunk {
  uint32_t n;
  uint32_t w[kFillWords];
};

__global__ void k_fill_words(uint32_t *dst, FillChunk c) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.n) dst[i] = c.w[i];
}

__global__ void k_zero_words(uint32_t *dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = 0u;
}

__global__ void k_copy_status(const DevScalars *sc, int *status) { *status = sc->status; }

hipError_t fill_words(void *dst, const void *src, size_t bytes, hipStream_t st) {
  const uint32_t *w = static_cast<const uint32_t *>(src);
  uint32_t *d = static_cast<uint32_t *>(dst);
  const size_t n = bytes / 4;
  for (size_t k0 = 0; k0 < n; k0 += kFillWords) {
    FillChunk c;
    c.n = (uint32_t)std::min<size_t>(kFillWords, n - k0);
    std::memcpy(c.w, w + k0, c.n * 4);
    hipLaunchKernelGGL(k_fill_words, dim3((c.n + 255) / 256), dim3(256), 0, st, d + k0, c);
  }
  return hipGetLastError();
}

hipError_t zero_words(void *dst, size_t bytes, hipStream_t st) {
  const size_t n = (bytes + 3) / 4;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0, st,
                     static_cast<uint32_t *>(dst), n);
  return hipGetLastError();
}

}  // namespace

extern "C" int enuf_compute_noalloc(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc,
                                    double r_cut, double lambda, int precision, const double *pos,
                                    const double *q, double *forces, double *energy5, int *status,
                                    void *hip_stream) {
  g_last_error.clear();
  FftPlan fp{};
  int rc = check_plan_args(N, box, alpha, p, sigma, M, Kc, r_cut, lambda, &fp);
  if (rc != ENUF_OK) return rc;
  if (precision != ENUF_FP64 && precision != ENUF_MIXED) { set_error("unknown precision"); return ENUF_EINVAL; }
  if (M > kNoAllocMaxM) {
    set_error("M must be <= " + std::to_string(kNoAllocMaxM) + " without allocation");
    return ENUF_EINVAL;
  }
  if (!pos || !q || !forces || !energy5) { set_error("NULL buffer"); return ENUF_EINVAL; }
  int dev = 0;
  HIP_OR_RETURN(hipGetDevice(&dev), ENUF_EDEVICE);
  const size_t max_lds = lds_budget(dev);
  if (max_lds == 0) { set_error("hipDeviceGetAttribute failed"); return ENUF_EDEVICE; }
  ComputeConfig cfg;
  PlanGeom g;
  if (!plan_config(N, box, alpha, p, sigma, M, Kc, r_cut, lambda, fp, max_lds, &cfg, &g)) return ENUF_EINVAL;
  cfg.precision = precision;
  PlanTables t;
  plan_tables(cfg, precision, &t);
  cfg.mesh.cheb_deg = t.cheb_deg;
  if (!plan_rows(&cfg, precision, max_lds, g.part_slots)) {
    set_error("mesh too large for the LDS in this precision");
    return ENUF_EINVAL;
  }
  const std::array<size_t, kPlanBuffers> sz = plan_buffer_bytes(N, p, M, Kc, g);
  const size_t need = arena_bytes(sz.data(), kPlanBuffers);
  if (need > kScratchBytes) {
    set_error("these sizes need " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
              std::to_string(kScratchBytes));
    return ENUF_EINVAL;
  }
  void *base = nullptr;
  rc = scratch_address(dev, &base);
  if (rc != ENUF_OK) return rc;
  void *ptr[kPlanBuffers];
  size_t off = 0;
  for (int k = 0; k < kPlanBuffers; ++k) {
    ptr[k] = (char *)base + off;
    off += arena_slot(sz[k]);
  }
  const ComputeBuffers buf = carve_buffers(ptr);
  hipStream_t st = (hipStream_t)hip_stream;
  // the previous call's contents: clear what the kernels expect to start at zero
  void *zp[8];
  size_t zb[8];
  const int nz = zeroed_buffers(cfg, buf, zp, zb);
  for (int k = 0; k < nz; ++k) HIP_OR_RETURN(zero_words(zp[k], zb[k], st), ENUF_EDEVICE);
  const int nky = 2 * Kc - 1;
  HIP_OR_RETURN(fill_words(buf.atab, t.atab.data(), nky * sizeof(double), st), ENUF_EDEVICE);
  HIP_OR_RETURN(fill_words(buf.tw64, t.tw64.data(), M * sizeof(double2), st), ENUF_EDEVICE);
  HIP_OR_RETURN(fill_words(buf.tw32, t.tw32.data(), M * sizeof(float2), st), ENUF_EDEVICE);
  if (precision == ENUF_MIXED)
    HIP_OR_RETURN(fill_words(buf.wcoef32, t.wcoef32.data(), t.wcoef32.size() * sizeof(float), st), ENUF_EDEVICE);
  else
    HIP_OR_RETURN(fill_words(buf.wcoef64, t.wcoef64.data(), t.wcoef64.size() * sizeof(double), st), ENUF_EDEVICE);
  HIP_OR_RETURN(configure_once(max_lds), ENUF_EDEVICE);
  hipError_t e = launch_compute(cfg, buf, pos, q, forces, nullptr, energy5, st);
  if (e == hipSuccess && status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, st, (const DevScalars *)buf.sc, status);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return ENUF_EDEVICE;
  }
  return ENUF_OK;
}

// ---------------------------------------------------------------------------
// DPD integrator
// ---------------------------------------------------------------------------
namespace {

// DPD cell grid: cells per side (edge box / nc >= R_c = 1) and slots per cell.
void dpd_geometry(int64_t N, double box, int *nc_out, int *cap_out) {
  int nc = (int)std::floor(box);
  nc = nc < 1 ? 1 : (nc > 1024 ? 1024 : nc);
  const double mean = (double)N / ((double)nc * nc * nc);
  *nc_out = nc;
  *cap_out = (int)std::ceil(mean + 6.0 * std::sqrt(mean) + 16.0);
}

constexpr int kDpdBuffers = 12;

// Bytes of every device buffer of a DPD integrator, in allocation order.
std::array<size_t, kDpdBuffers> dpd_buffer_bytes(int64_t N, double box, int64_t nbonds) {
  int nc, cap;
  dpd_geometry(N, box, &nc, &cap);
  const size_t n = (size_t)N, nc3 = (size_t)nc * nc * nc;
  return {n * sizeof(double),                                        // q
          3 * n * sizeof(double),                                    // fdpd
          5 * sizeof(double),                                        // e5
          2 * nc3 * sizeof(int),                                     // dcnt (two sets)
          nc3 * (size_t)cap * sizeof(double4),                       // cpos
          nc3 * (size_t)cap * sizeof(double4),                       // cvel
          (n + 1) * sizeof(int),                                     // bond_start
          (size_t)(2 * nbonds > 0 ? 2 * nbonds : 1) * sizeof(int),   // bond_to
          sizeof(int),                                               // status
          n * sizeof(int),                                           // dslot
          sizeof(unsigned long long),                                // step_ctr
          n * sizeof(int)};                                          // species
}

}  // namespace

struct enuf_dpd {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  DpdParams P{};
  enuf_plan *plan = nullptr;  // not owned
  double *q = nullptr;        // [N]
  double *fdpd = nullptr;     // [N * 3] pair + bond forces
  double *e5 = nullptr;       // [5]
  int *dcnt = nullptr;        // [2 ncell^3] two sets, like the plan's bin counts
  double4 *cpos = nullptr;    // [ncell^3 * cap] (x, y, z, index) per cell slot
  double4 *cvel = nullptr;    // [ncell^3 * cap] predicted velocity per cell slot
  int *bond_start = nullptr;  // [N + 1]
  int *bond_to = nullptr;     // [2 nbonds]
  int *status = nullptr;      // [1]
  std::vector<void *> allocations;
  EventTimer timer;  // enuf_dpd_time_kernel
  int *dslot = nullptr;       // [N] static compact slot of each particle (-1: neutral)
  int64_t nq = 0;
  DpdCharges charges{};
  hipStream_t side = nullptr;  // forked stream (pair forces, then real space)
  int concurrent = 1;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  unsigned long long *step_ctr = nullptr;  // [1] next step index when stepped in a batch
  int *species = nullptr;                  // [N] species of each particle (read when P.nspec > 1)
  int batches = 0;                         // batches this integrator is a member of
  size_t bytes = 0;
  // Steps of enuf_dpd_run captured in graphs (no cross-stream events: the
  // fork and join are dependency edges), one per graph length (kGraphLen) and
  // per parity of the first replayed step (the bin-count set a step uses is
  // its index mod 2; a graph of an even number of steps keeps it).  Each is
  // valid for the state buffers and the configuration it was captured with.
  struct GraphSlot {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *key[3] = {nullptr, nullptr, nullptr};
    std::vector<unsigned char> cfg;  // parameters the kernels were captured with
  };
  int use_graph = 1;
  GraphSlot gslot[2][2];  // [length index][parity]

  // Callers synchronise the stream first: an exec may still be queued on it.
  void drop_graph(int len, int par) {
    GraphSlot &g = gslot[len][par];
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
  }
  void drop_graph() {
    for (int l = 0; l < 2; ++l)
      for (int par = 0; par < 2; ++par) drop_graph(l, par);
  }

  // All buffers in one device allocation (one hipMalloc / hipFree per
  // object), each at a 256-byte aligned offset.  False on failure.
  bool alloc_arena(const size_t *sizes, int n, void **ptrs) {
    const size_t total = arena_bytes(sizes, n);
    void *base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) return false;
    allocations.push_back(base);
    bytes += total;
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
      ptrs[k] = (char *)base + off;
      off += arena_slot(sizes[k]);
    }
    return true;
  }
  ~enuf_dpd() {
    drop_graph();
    timer.drop();
    if (side) (void)hipStreamDestroy(side);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (void *ptr : allocations) (void)hipFree(ptr);
  }
};

extern "C" {

enuf_dpd *enuf_dpd_create(int64_t N, double box, const enuf_dpd_params *prm, enuf_plan *plan,
                          const double *q, int64_t nbonds, const int64_t *bonds) {
  g_last_error.clear();
  if (N < 1 || N > (int64_t)1 << 28) { set_error("N must be in [1, 2^28]"); return nullptr; }
  if (!(std::isfinite(box) && box >= 2.0)) { set_error("box must be finite and >= 2 (R_c = 1)"); return nullptr; }
  if (!prm) { set_error("NULL params"); return nullptr; }
  const double vals[8] = {prm->a, prm->gamma, prm->sigma, prm->dt, prm->lam, prm->k_bond, prm->r0_bond, prm->kappa};
  for (double v : vals)
    if (!std::isfinite(v)) { set_error("non-finite DPD parameter"); return nullptr; }
  if (!(prm->dt > 0.0)) { set_error("dt must be > 0"); return nullptr; }
  if (!q) { set_error("NULL charges"); return nullptr; }
  if (nbonds < 0 || (nbonds > 0 && !bonds)) { set_error("invalid bond list"); return nullptr; }
  if (plan && (plan->N != N || plan->L != box)) { set_error("plan N / box differ from the integrator's"); return nullptr; }
  {
    int nc0, cap0;
    dpd_geometry(N, box, &nc0, &cap0);
    if (cap0 > kPairOwn) { set_error("density too high: DPD cells would need more than 128 slots"); return nullptr; }
    // the pair kernels hold cell slots in 32-bit integers
    if ((int64_t)nc0 * nc0 * nc0 * cap0 >= (int64_t)1 << 31) {
      set_error("DPD cell grid too large: ncell^3 x capacity >= 2^31 slots");
      return nullptr;
    }
  }
  std::vector<int> deg(N + 1, 0);
  for (int64_t b = 0; b < nbonds; ++b) {
    const int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= N || j >= N || i == j) { set_error("bond index out of range"); return nullptr; }
    ++deg[i + 1];
    ++deg[j + 1];
  }
  for (int64_t i = 0; i < N; ++i) deg[i + 1] += deg[i];
  std::vector<int> to(2 * nbonds > 0 ? 2 * nbonds : 1), fill(deg.begin(), deg.end() - 1);
  for (int64_t b = 0; b < nbonds; ++b) {
    const int i = (int)bonds[2 * b], j = (int)bonds[2 * b + 1];
    to[fill[i]++] = j;
    to[fill[j]++] = i;
  }

  enuf_dpd *d = new enuf_dpd();
  d->N = N;
  d->plan = plan;
  if (hipGetDevice(&d->device) != hipSuccess) { set_error("hipGetDevice failed"); delete d; return nullptr; }
  if (plan) d->stream = plan->stream;
  DpdParams &P = d->P;
  P.L = box; P.a = prm->a; P.gamma = prm->gamma; P.sigma = prm->sigma; P.dt = prm->dt; P.lam = prm->lam;
  P.k_bond = prm->k_bond; P.r0_bond = prm->r0_bond; P.kappa = prm->kappa; P.seed = prm->seed;
  int nc, cap;
  dpd_geometry(N, box, &nc, &cap);
  P.ncell = nc;
  P.cap = cap;
  P.inv_cell = (double)nc / box;
  pair_segments(nc, kPairSeg, &P.seg_cells, &P.nseg);
  P.pair_stage = kPairStage;
  if (configure_pair_kernels(pair_lds_bytes(P, true)) != hipSuccess) {
    set_error("configuring the pair kernels failed");
    delete d;
    return nullptr;
  }
  const size_t n = (size_t)N, nc3 = (size_t)nc * nc * nc;
  const std::array<size_t, kDpdBuffers> sz = dpd_buffer_bytes(N, box, nbonds);
  void *ptr[kDpdBuffers];
  if (!d->alloc_arena(sz.data(), kDpdBuffers, ptr)) { set_error("device allocation failed"); delete d; return nullptr; }
  d->q = (double *)ptr[0];
  d->fdpd = (double *)ptr[1];
  d->e5 = (double *)ptr[2];
  d->dcnt = (int *)ptr[3];
  d->cpos = (double4 *)ptr[4];
  d->cvel = (double4 *)ptr[5];
  d->bond_start = (int *)ptr[6];
  d->bond_to = (int *)ptr[7];
  d->status = (int *)ptr[8];
  d->dslot = (int *)ptr[9];
  d->step_ctr = (unsigned long long *)ptr[10];
  d->species = (int *)ptr[11];
  P.nspec = 0;
  P.species = d->species;
  if (hipMemcpy(d->q, q, n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(d->bond_start, deg.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d->bond_to, to.data(), to.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(d->dcnt, 0, 2 * nc3 * sizeof(int)) != hipSuccess || hipMemset(d->e5, 0, 5 * sizeof(double)) != hipSuccess ||

      hipMemset(d->status, 0, sizeof(int)) != hipSuccess || hipMemset(d->species, 0, n * sizeof(int)) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess) {
    set_error("device setup of the DPD integrator failed");
    delete d;
    return nullptr;
  }
  // The charges are fixed: compact them once (index order) and precompute the
  // plan scalars the compaction kernels would otherwise produce every step.
  std::vector<double> hq(n);
  if (hipMemcpy(hq.data(), d->q, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("copying the charges failed");
    delete d;
    return nullptr;
  }
  std::vector<int> hslot(n, -1);
  DevScalars st{};
  int nq = 0;
  for (size_t i = 0; i < n; ++i) {
    if (!std::isfinite(hq[i])) { set_error("non-finite charge"); delete d; return nullptr; }
    if (hq[i] != 0.0) hslot[i] = nq++;
    st.sum_q += hq[i];
    st.sum_absq += std::fabs(hq[i]);
    st.sum_q2 += hq[i] * hq[i];
  }
  if (std::fabs(st.sum_q) > 1e-10 * st.sum_absq) { set_error("charges are not neutral"); delete d; return nullptr; }
  st.nq = nq;
  int ex;
  std::frexp(st.sum_absq + 1.0, &ex);
  st.scale = std::ldexp(1.0, 61 - ex);
  st.inv_scale = std::ldexp(1.0, ex - 61);
  d->nq = nq;
  if (hipMemcpy(d->dslot, hslot.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("uploading the charge map failed");
    delete d;
    return nullptr;
  }
  if (plan) {
    DpdCharges &ch = d->charges;
    ch.enabled = 1;
    ch.dslot = d->dslot;
    ch.q = d->q;
    ch.xq = plan->buf.xq;
    ch.slot = plan->buf.slot;
    ch.ccnt = plan->buf.ccnt;
    ch.cgrid = plan->buf.cgrid;
    ch.cpre = plan->buf.cpre;
    ch.cells = plan->cfg.cells;
    ch.xcnt = plan->buf.xcnt;
    ch.xslot = plan->buf.xslot;
    ch.M = plan->cfg.mesh.M;
    ch.xcap = plan->cfg.mesh.xcap;
    ch.m_over_l = plan->cfg.mesh.m_over_l;
    ch.sc = plan->buf.sc;
    ch.stat = st;
  }
  if (hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&d->join_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&d->fork_ev, hipEventDisableTiming) != hipSuccess) {
    set_error("creating the side stream failed");
    delete d;
    return nullptr;
  }
  return d;
}

int enuf_dpd_set_stream(enuf_dpd *d, void *hip_stream) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  d->stream = (hipStream_t)hip_stream;
  if (d->plan) d->plan->stream = d->stream;
  return ENUF_OK;
}

// The plan's buffers with the real-space and mesh bin counts of set `par`
// (a DPD step bins into one set while the combine clears the other).
static ComputeBuffers plan_buffers_set(const enuf_plan *pl, int par) {
  ComputeBuffers b = pl->buf;
  const int nc = pl->cfg.cells.ncell;
  b.ccnt += (size_t)par * nc * nc * nc;
  b.xcnt += (size_t)par * pl->cfg.mesh.M * kXSub;
  return b;
}

// The DPD cell counts of set `par` (with a plan; without one the post kernel
// clears the only set before the next step bins).
static int *dpd_counts_set(const enuf_dpd *d, int par) {
  return d->plan ? d->dcnt + (size_t)par * d->P.ncell * d->P.ncell * d->P.ncell : d->dcnt;
}

static DpdCharges dpd_charges_set(const enuf_dpd *d, int par) {
  DpdCharges ch = d->charges;
  if (ch.enabled && d->plan) {
    const ComputeBuffers b = plan_buffers_set(d->plan, par);
    ch.ccnt = b.ccnt;
    ch.xcnt = b.xcnt;
  }
  return ch;
}

// Steps per graph launch of enuf_dpd_run: long graphs for the body of a run,
// short ones for its remainder (at most one step of the body is then
// launched eagerly, plus the last step with its energy reduction).
constexpr int kGraphLen[2] = {8, 2};
static_assert(kGraphLen[0] % 2 == 0 && kGraphLen[1] % 2 == 0,
              "a replayed graph keeps the parity of the bin-count set");

// The last node captured on a capturing stream (its single dependency)
// (*count = 0 before the first node of the capture.)
static hipError_t capture_tail(hipStream_t st, hipGraphNode_t *node, size_t *count) {
  hipStreamCaptureStatus cs;
  const hipGraphNode_t *deps = nullptr;
  size_t nd = 0;
  hipError_t e = hipStreamGetCaptureInfo_v2(st, &cs, nullptr, nullptr, &deps, &nd);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusActive || nd > 1 || (nd == 1 && !deps)) return hipErrorIllegalState;
  *node = nd == 1 ? deps[0] : nullptr;
  *count = nd;
  return hipSuccess;
}

// One force evaluation (mode 1) or step (mode 0).
//   pre:  launch the pre kernel first (else the previous step's combine ran it)
//   next: fuse the pre kernel of the next step (mode 0) into the combine
//   graph_st: capture for a graph on that stream (the step index is read from
//         and advanced in device memory; the fork and join are dependency
//         edges of the capture instead of events).
// With a plan, the mesh passes (the longest chain) are enqueued first on the
// integrator's stream; the pair forces and then the real-space term run on
// one forked stream beside them (a second forked stream costs more in
// cross-stream waits than it gains); the combine kernel joins the two.  All
// cell and bin counts come in two sets, step k using set k mod 2, so that the
// fused combine can clear step k's set while it bins step k + 1 into the
// other.
// energies: reduce the ENUF energies of this evaluation (enuf_dpd_energy
// reports the last one; steps inside a run other than its last skip it).
constexpr int kDpdXThreads = 256;  // x-pass work-group size beside the pair kernels
static int dpd_eval(enuf_dpd *d, int mode, double *pos, double *vel, double *force, uint64_t step,
                    bool energies, bool pre, bool next, hipStream_t graph_st = nullptr) {
  const int64_t N = d->N;
  const bool graph = graph_st != nullptr;
  KernelTimer *tm = graph ? nullptr : d->timer.active();
  hipStream_t st = graph ? graph_st : d->stream;
  const unsigned long long *step_dev = graph ? d->step_ctr : nullptr;
  // the real-space and mesh bin counts of step k are set k mod 2
  const int par = (int)(step & 1);
  const DpdCharges ch = dpd_charges_set(d, par), ch_next = dpd_charges_set(d, par ^ 1);
  int *dcnt = dpd_counts_set(d, par), *dcnt_next = dpd_counts_set(d, par ^ 1);
  hipError_t e = hipSuccess;
  if (pre)
    e = launch_dpd_pre(N, mode, d->P, pos, vel, force, dcnt, d->cpos, d->cvel, d->status, ch, st, tm);
  if (!d->plan) {
    if (e == hipSuccess)
      e = launch_dpd_pair(N, d->P, step, pos, dcnt, d->cpos, d->cvel, d->bond_start, d->bond_to,
                          d->fdpd, st, tm, step_dev);
    if (e == hipSuccess) e = launch_dpd_post(N, mode, d->P, d->fdpd, nullptr, force, vel, dcnt, st, tm);
    if (graph && e == hipSuccess) e = launch_add_u64(d->step_ctr, st);
    if (next && e == hipSuccess)
      e = launch_dpd_pre(N, 0, d->P, pos, vel, force, dcnt_next, d->cpos, d->cvel, d->status, ch_next,
                         st, tm);
  } else {
    enuf_plan *pl = d->plan;
    const ComputeBuffers bk = plan_buffers_set(pl, par);
    if (!graph) pl->stream = st;
    const bool fork = d->concurrent != 0;
    const bool events = fork && !graph;
    hipStream_t s1 = events ? d->side : st;
    hipGraphNode_t n_pre = nullptr, n_bwd = nullptr;
    size_t c_pre = 0;
    if (events) {
      if (e == hipSuccess) e = hipEventRecord(d->fork_ev, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(s1, d->fork_ev, 0);
    }
    if (graph && fork && e == hipSuccess) e = capture_tail(st, &n_pre, &c_pre);
    // beside the pair and real-space kernels the x pass runs in 256-thread
    // work-groups, which fit on CUs those kernels partly hold (0.5 us less
    // per step at N = 24000; alone it is faster in 512-thread ones)
    if (e == hipSuccess) e = launch_recip(pl->cfg, bk, d->nq, st, tm, fork ? kDpdXThreads : kPassThreads);
    size_t c_bwd = 0;
    if (graph && fork && e == hipSuccess) e = capture_tail(st, &n_bwd, &c_bwd);
    // the pair forces and the real-space term depend on the pre kernel only
    if (graph && fork && e == hipSuccess)
      e = hipStreamUpdateCaptureDependencies(st, &n_pre, c_pre, hipStreamSetCaptureDependencies);
    if (e == hipSuccess)
      e = launch_dpd_pair(N, d->P, step, pos, dcnt, d->cpos, d->cvel, d->bond_start, d->bond_to,
                          d->fdpd, s1, tm, step_dev);
    const int ndcell3 = d->P.ncell * d->P.ncell * d->P.ncell;
    if (e == hipSuccess) e = launch_real(pl->cfg, bk, d->nq, s1, tm);
    if (events && e == hipSuccess) e = hipEventRecord(d->join_ev, s1);
    if (events && e == hipSuccess) e = hipStreamWaitEvent(st, d->join_ev, 0);
    // the combine kernel depends on the mesh passes and the real-space term
    if (graph && fork && e == hipSuccess)
      e = hipStreamUpdateCaptureDependencies(st, &n_bwd, c_bwd, hipStreamAddCaptureDependencies);
    if (e == hipSuccess) {
      FinishArgs fa;
      fa.mode = mode;
      fa.kappa = d->P.kappa;
      fa.dt = d->P.dt;
      fa.fdpd = d->fdpd;
      fa.vel = vel;
      fa.dcnt = dcnt;  // this step's set, cleared while the next is filled
      fa.ndcell3 = ndcell3;
      fa.energies = energies ? 1 : 0;
      fa.step_inc = graph ? d->step_ctr : nullptr;
      if (next && !energies)
        e = launch_combine_pre(pl->cfg, bk, force, fa, d->P, pos, dcnt_next, d->cpos, d->cvel, d->status,
                               ch_next, st, tm);
      else {
        e = launch_combine(pl->cfg, bk, force, nullptr, d->e5, fa, st, tm);
        if (next && e == hipSuccess)
          e = launch_dpd_pre(N, 0, d->P, pos, vel, force, dcnt_next, d->cpos, d->cvel, d->status, ch_next,
                             st, tm);
      }
    }
  }
  if (e != hipSuccess) {
    set_error(std::string("DPD kernel launch failed: ") + hipGetErrorString(e));
    return ENUF_EDEVICE;
  }
  return ENUF_OK;
}

static int dpd_check(enuf_dpd *d, const void *a, const void *b, const void *c) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  if (!a || !b || !c) { set_error("NULL buffer"); return ENUF_EINVAL; }
  if (d->plan) {
    const ComputeConfig &cf = d->plan->cfg;
    if (cf.lds_fwd > d->plan->max_lds || cf.lds_bwd > d->plan->max_lds) {
      set_error("mesh too large for one LDS plane in this precision");
      return ENUF_EINVAL;
    }
  }
  return ENUF_OK;
}

int enuf_dpd_forces(enuf_dpd *d, double *pos, const double *vel, double *force, uint64_t step) {
  int rc = dpd_check(d, pos, vel, force);
  if (rc != ENUF_OK) return rc;
  return dpd_eval(d, 1, pos, const_cast<double *>(vel), force, step, true, true, false);
}

// Bytes of everything the captured kernels take by value: when they change
// (integrator parameters, species, concurrency, the plan's configuration),
// the graph is captured again.
static std::vector<unsigned char> dpd_graph_config(const enuf_dpd *d) {
  std::vector<unsigned char> v;
  auto put = [&v](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    v.insert(v.end(), c, c + n);
  };
  put(&d->P, sizeof(DpdParams));
  put(&d->concurrent, sizeof(int));
  put(&d->charges, sizeof(DpdCharges));
  if (d->plan) {
    put(&d->plan->cfg, sizeof(ComputeConfig));
    put(&d->plan->buf, sizeof(ComputeBuffers));
  }
  return v;
}

// Capture kGraphLen[len] steps (no energy reduction) on the integrator's side
// stream.  False (and no graph) if capture is not available; the caller then
// launches the steps eagerly.  Synchronises the integrator's stream first,
// since the graph it replaces may still be queued there.
static bool dpd_capture(enuf_dpd *d, double *pos, double *vel, double *force, int len, int par) {
  if (hipStreamSynchronize(d->stream) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  d->drop_graph(len, par);
  hipStream_t cs = d->side;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  int rc = ENUF_OK;
  // the step index passed here only selects the bin-count set; the replayed
  // steps read their index from the device counter
  for (int k = 0; k < kGraphLen[len] && rc == ENUF_OK; ++k)
    rc = dpd_eval(d, 0, pos, vel, force, (uint64_t)(par + k), false, false, true, cs);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc != ENUF_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    g_last_error.clear();
    return false;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  enuf_dpd::GraphSlot &gs = d->gslot[len][par];
  gs.graph = g;
  gs.exec = x;
  gs.key[0] = pos;
  gs.key[1] = vel;
  gs.key[2] = force;
  gs.cfg = dpd_graph_config(d);
  return true;
}

// The graph of kGraphLen[len] steps from parity par for these buffers, captured
// now if it is missing or stale; nullptr if capture is not available.
static hipGraphExec_t dpd_graph(enuf_dpd *d, double *pos, double *vel, double *force, int len, int par) {
  const enuf_dpd::GraphSlot &gs = d->gslot[len][par];
  const bool same = gs.exec && gs.key[0] == pos && gs.key[1] == vel && gs.key[2] == force &&
                    gs.cfg == dpd_graph_config(d);
  if (same || dpd_capture(d, pos, vel, force, len, par)) return d->gslot[len][par].exec;
  return nullptr;
}

int enuf_dpd_run(enuf_dpd *d, double *pos, double *vel, double *force, uint64_t first_step, int nsteps) {
  int rc = dpd_check(d, pos, vel, force);
  if (rc != ENUF_OK) return rc;
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return ENUF_EINVAL; }
  if (nsteps == 0) return ENUF_OK;
  const int par = (int)(first_step & 1);
  const int body = nsteps - 1;
  // graphs first: capturing one synchronises the stream, which must not
  // happen between the launches of this run
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  if (d->use_graph && !d->timer.active()) {
    if (body >= kGraphLen[0]) gx[0] = dpd_graph(d, pos, vel, force, 0, par);
    const int rest = body - (gx[0] ? (body / kGraphLen[0]) * kGraphLen[0] : 0);
    if (rest >= kGraphLen[1]) gx[1] = dpd_graph(d, pos, vel, force, 1, par);
  }
  // the first step's pre kernel; each later one runs fused into the combine
  // kernel of the step before
  KernelTimer *tm = d->timer.active();
  HIP_OR_RETURN(launch_dpd_pre(d->N, 0, d->P, pos, vel, force, dpd_counts_set(d, par),
                               d->cpos, d->cvel, d->status, dpd_charges_set(d, par), d->stream, tm),
                ENUF_EDEVICE);
  int s = 0;
  // all but the last step from graphs (long ones, then short ones; every
  // graph holds an even number of steps, so each starts on parity par); the
  // rest, and the last step with its energy reduction, eagerly
  if (gx[0] || gx[1]) {
    HIP_OR_RETURN(launch_set_u64(d->step_ctr, (unsigned long long)first_step, d->stream), ENUF_EDEVICE);
    for (int len = 0; len < 2; ++len) {
      if (!gx[len]) continue;
      for (; s + kGraphLen[len] <= body; s += kGraphLen[len])
        HIP_OR_RETURN(hipGraphLaunch(gx[len], d->stream), ENUF_EDEVICE);
    }
  }
  for (; s < nsteps; ++s) {
    rc = dpd_eval(d, 0, pos, vel, force, first_step + (uint64_t)s, s == nsteps - 1, false, s < nsteps - 1);
    if (rc != ENUF_OK) return rc;
  }
  return ENUF_OK;
}

int enuf_dpd_prepare_graphs(enuf_dpd *d, double *pos, double *vel, double *force) {
  int rc = dpd_check(d, pos, vel, force);
  if (rc != ENUF_OK) return rc;
  if (!d->use_graph) return ENUF_OK;
  for (int len = 0; len < 2; ++len)
    for (int par = 0; par < 2; ++par)
      if (!dpd_graph(d, pos, vel, force, len, par)) {
        set_error("HIP graph capture of the DPD step failed");
        return ENUF_EDEVICE;
      }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  return ENUF_OK;
}

int enuf_dpd_set_graphs(enuf_dpd *d, int enable) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  d->use_graph = enable ? 1 : 0;
  d->drop_graph();
  return ENUF_OK;
}

int enuf_dpd_set_concurrency(enuf_dpd *d, int enable) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  d->concurrent = enable ? 1 : 0;
  return ENUF_OK;
}

int enuf_dpd_energy(enuf_dpd *d, double *energy5) {
  if (!d || !energy5) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipMemcpyAsync(energy5, d->e5, 5 * sizeof(double), hipMemcpyDeviceToDevice, d->stream), ENUF_EDEVICE);
  return ENUF_OK;
}

int enuf_dpd_status(enuf_dpd *d, int *status) {
  if (!d || !status) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  int s = 0;
  HIP_OR_RETURN(hipMemcpy(&s, d->status, sizeof(int), hipMemcpyDeviceToHost), ENUF_EDEVICE);
  const int zero = 0;
  HIP_OR_RETURN(hipMemcpy(d->status, &zero, sizeof(int), hipMemcpyHostToDevice), ENUF_EDEVICE);
  if (s == 0 && d->plan) return enuf_plan_status(d->plan, status);
  if (d->plan) {
    int ps = 0;
    (void)enuf_plan_status(d->plan, &ps);
  }
  *status = s;
  return ENUF_OK;
}

int enuf_dpd_time_kernel(enuf_dpd *d, int kernel, int max_launches) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  if (!valid_timer_args(kernel, max_launches)) { set_error("invalid kernel id or launch count"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  if (!d->timer.start(kernel, max_launches)) { set_error("hipEventCreate failed"); return ENUF_EDEVICE; }
  return ENUF_OK;
}

int enuf_dpd_kernel_time(enuf_dpd *d, double *total_ms, int *launches) {
  if (!d || !total_ms || !launches) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  HIP_OR_RETURN(d->timer.total(total_ms, launches), ENUF_EDEVICE);
  return ENUF_OK;
}

void enuf_dpd_destroy(enuf_dpd *d) {
  if (!d) return;
  (void)hipStreamSynchronize(d->stream);
  delete d;
}

size_t enuf_dpd_footprint_bytes(const enuf_dpd *d) {
  if (!d) return 0;
  return d->bytes + (d->plan ? d->plan->bytes : 0);
}

size_t enuf_plan_footprint_estimate(int64_t N, double box, int p, int M, int Kc, double r_cut) {
  if (N < 1 || !finite_pos(box) || p < 1 || M < 4 || Kc < 1 || !finite_pos(r_cut)) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const size_t lds = lds_budget(dev);
  PlanGeom g;
  if (lds == 0 || !plan_geometry(N, box, p, M, Kc, r_cut, lds, &g)) return 0;
  const auto sz = plan_buffer_bytes(N, p, M, Kc, g);
  return arena_bytes(sz.data(), kPlanBuffers);
}

size_t enuf_dpd_footprint_estimate(int64_t N, double box, int64_t nbonds) {
  if (N < 1 || !finite_pos(box) || nbonds < 0) return 0;
  const auto sz = dpd_buffer_bytes(N, box, nbonds);
  return arena_bytes(sz.data(), kDpdBuffers);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched DPD steps: one launch per stage for every member of the batch.
// ---------------------------------------------------------------------------
struct enuf_batch {
  struct Member {
    int id;
    enuf_dpd *d;
    double *pos, *vel, *force;
  };
  int device = 0;
  int precision = ENUF_MIXED;
  hipStream_t stream = nullptr;   // the caller's stream: runs are ordered after its work and before its later work
  hipStream_t own = nullptr;      // the batch's stream (graph capture needs a non-null stream)
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
  hipEvent_t in_ev = nullptr, out_ev = nullptr;
  int concurrent = 1;
  int use_graph = 1;
  int ik = -1;       // force mode of the members (all alike; -1 while empty)
  std::vector<Member> members;
  int next_id = 0;
  // device copies of the member table and the work maps (rebuilt when the
  // membership changes), staged through pinned host buffers
  BatchMember *dmem = nullptr;
  int2 *dmap = nullptr;
  size_t mem_cap = 0, map_cap = 0;
  BatchMember *hmem = nullptr;
  int2 *hmap = nullptr;
  int off[8] = {0};  // map offsets: pre, pair, real, fwd, x, bwd, comb, end
  int nmem = 0;      // members in the device table
  size_t lds_fwd = 0, lds_x = 0, lds_bwd = 0;
  int pass_threads = kBatchPassThreads, x_threads = kBatchXThreads;  // work-group sizes of the mesh passes
  // launch parameters (enuf_batch_set_tuning; none changes a result bit)
  struct Tuning {
    int pass_threads = kBatchPassThreads;  // spread / gather work-groups (raised to the members' FFT needs)
    int x_threads = kBatchXThreads;        // x-pass work-groups (likewise)
    int stage = kBatchStage;               // most charges staged per mesh work-group (at most the plan's)
    int pair_steps = 4;                    // candidate steps in flight per lane of the pair kernel
    int x_split_mul = 1;                   // x-pass work-groups per ky row: the plan's times this (<= Kc)
    int pair_seg = kBatchPairSeg;          // cells per column segment of the pair kernel, about
  } tune;
  bool dirty = true;
  // step graphs: [0][par] a step of table par that ends with the fused
  // combine + pre kernel (binning the next step into the other set), [1][par]
  // a run's last step (combine and energy reduction)
  hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  EventTimer timer;  // enuf_batch_time_kernel: eager single-stream steps while active

  bool captured() const {
    for (int k = 0; k < 2; ++k)
      for (int p = 0; p < 2; ++p)
        if (exec[k][p]) return true;
    return false;
  }
  void drop_graph() {
    for (int k = 0; k < 2; ++k)
      for (int p = 0; p < 2; ++p) {
        if (exec[k][p]) (void)hipGraphExecDestroy(exec[k][p]);
        if (graph[k][p]) (void)hipGraphDestroy(graph[k][p]);
        exec[k][p] = nullptr;
        graph[k][p] = nullptr;
      }
  }
  ~enuf_batch() {
    drop_graph();
    for (int k = 0; k < 2; ++k) {
      if (side[k]) (void)hipStreamDestroy(side[k]);
      if (join_ev[k]) (void)hipEventDestroy(join_ev[k]);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (in_ev) (void)hipEventDestroy(in_ev);
    if (out_ev) (void)hipEventDestroy(out_ev);
    if (own) (void)hipStreamDestroy(own);
    if (dmem) (void)hipFree(dmem);
    if (dmap) (void)hipFree(dmap);
    if (hmem) (void)hipHostFree(hmem);
    if (hmap) (void)hipHostFree(hmap);
  }
};

namespace {

// The member as table par sees it: bin-count set par (and the other set as
// the next step's, for the fused combine + pre kernel).
BatchMember member_view(const enuf_batch::Member &mb, const enuf_batch::Tuning &t, int par) {
  const enuf_dpd *d = mb.d;
  const enuf_plan *pl = d->plan;
  BatchMember m{};
  m.cfg = pl->cfg;
  if (m.cfg.mesh.stage > t.stage) {  // the batch's smaller stage (less LDS per work-group)
    m.cfg.mesh.stage = t.stage;
    mesh_lds_bytes(m.cfg.mesh, pl->cfg.precision, &m.cfg.lds_fwd, &m.cfg.lds_x, &m.cfg.lds_bwd);
  }
  // more x-pass work-groups per ky row (each a range of kz lines; the energy
  // is kept per line, so the grouping does not change it)
  m.cfg.mesh.xsplit = std::min(m.cfg.mesh.Kc, m.cfg.mesh.xsplit * t.x_split_mul);
  m.buf = plan_buffers_set(pl, par);
  m.nq = (int)d->nq;
  m.nblk = pl->cfg.nblk;
  const int64_t g = (d->nq + 3) / 4;
  m.real_blocks = (int)(g < 1 ? 1 : (g < 2048 ? g : 2048));
  m.fscale = pl->cfg.mesh.ik ? 2.0 / (pl->cfg.L * pl->cfg.L) : (double)pl->cfg.mesh.M / (M_PI * pl->cfg.L * pl->cfg.L);
  m.inv2piL = 1.0 / (2.0 * M_PI * pl->cfg.L);
  m.N = d->N;
  m.P = d->P;
  // the batch's segments and stage (the pair kernel reads velocities from
  // their cell slots, so the stage holds more particles in less LDS)
  pair_segments(m.P.ncell, t.pair_seg, &m.P.seg_cells, &m.P.nseg);
  m.P.pair_stage = kBatchPairStage;
  m.pair_blocks = pair_blocks(m.P);
  m.pos = mb.pos;
  m.vel = mb.vel;
  m.force = mb.force;
  m.fdpd = d->fdpd;
  m.e5 = d->e5;
  m.dcnt = dpd_counts_set(d, par);
  m.dcnt_next = dpd_counts_set(d, par ^ 1);
  m.cpos = d->cpos;
  m.cvel = d->cvel;
  m.bond_start = d->bond_start;
  m.bond_to = d->bond_to;
  m.status = d->status;
  m.ch = dpd_charges_set(d, par);
  m.ch_next = dpd_charges_set(d, par ^ 1);
  m.step = d->step_ctr;
  return m;
}

// Member table and work maps.  Members are ordered by decreasing N so that
// the blocks of the largest systems are dispatched first in every stage.
int batch_rebuild(enuf_batch *b) {
  std::vector<int> order(b->members.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->members[x].d->N > b->members[y].d->N; });
  std::vector<BatchMember> mem, mem1;  // tables of bin-count sets 0 and 1
  std::vector<int2> map[7];
  size_t lf = 0, lx = 0, lb = 0;
  int tp = b->tune.pass_threads, tx = b->tune.x_threads;  // enough threads for every member's FFT passes
  for (int k : order) {
    const BatchMember m = member_view(b->members[k], b->tune, 0);
    const int id = (int)mem.size();
    mem.push_back(m);
    mem1.push_back(member_view(b->members[k], b->tune, 1));
    const int planes = m.cfg.mesh.M * m.cfg.mesh.parts;     // work-groups of the spread pass
    const int bplanes = m.cfg.mesh.M * m.cfg.mesh.bparts;   // and of the gather pass
    const int counts[7] = {m.nblk,  m.pair_blocks, m.real_blocks, planes, m.cfg.mesh.nky * m.cfg.mesh.xsplit,
                           bplanes, m.nblk};
    for (int s = 0; s < 7; ++s)
      for (int i = 0; i < counts[s]; ++i) map[s].push_back(make_int2(id, i));
    lf = std::max(lf, m.cfg.lds_fwd);
    lx = std::max(lx, m.cfg.lds_x);
    lb = std::max(lb, m.cfg.lds_bwd);
    const int nbf = fft_max_butterflies(m.cfg.mesh.fft);
    while (tp < nbf) tp *= 2;
    while (tx < nbf) tx *= 2;
  }
  size_t nmap = 0;
  for (int s = 0; s < 7; ++s) {
    b->off[s] = (int)nmap;
    nmap += map[s].size();
  }
  b->off[7] = (int)nmap;
  // the previous table may still be read by queued work
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  if (mem.size() > b->mem_cap) {
    const size_t cap = std::max<size_t>(mem.size(), 2 * b->mem_cap);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->hmem) (void)hipHostFree(b->hmem);
    b->dmem = nullptr;
    b->hmem = nullptr;
    b->mem_cap = 0;
    HIP_OR_RETURN(hipMalloc(&b->dmem, 2 * cap * sizeof(BatchMember)), ENUF_ENOMEM);
    HIP_OR_RETURN(hipHostMalloc((void **)&b->hmem, 2 * cap * sizeof(BatchMember), hipHostMallocDefault),
                  ENUF_ENOMEM);
    b->mem_cap = cap;
  }
  if (nmap > b->map_cap) {
    const size_t cap = std::max<size_t>(nmap, 2 * b->map_cap);
    if (b->dmap) (void)hipFree(b->dmap);
    if (b->hmap) (void)hipHostFree(b->hmap);
    b->dmap = nullptr;
    b->hmap = nullptr;
    b->map_cap = 0;
    HIP_OR_RETURN(hipMalloc(&b->dmap, cap * sizeof(int2)), ENUF_ENOMEM);
    HIP_OR_RETURN(hipHostMalloc((void **)&b->hmap, cap * sizeof(int2), hipHostMallocDefault), ENUF_ENOMEM);
    b->map_cap = cap;
  }
  if (!mem.empty()) {
    std::memcpy(b->hmem, mem.data(), mem.size() * sizeof(BatchMember));
    std::memcpy(b->hmem + mem.size(), mem1.data(), mem1.size() * sizeof(BatchMember));
    for (int s = 0; s < 7; ++s)
      if (!map[s].empty()) std::memcpy(b->hmap + b->off[s], map[s].data(), map[s].size() * sizeof(int2));
    HIP_OR_RETURN(hipMemcpyAsync(b->dmem, b->hmem, 2 * mem.size() * sizeof(BatchMember), hipMemcpyHostToDevice,
                                 b->own), ENUF_EDEVICE);
    HIP_OR_RETURN(hipMemcpyAsync(b->dmap, b->hmap, nmap * sizeof(int2), hipMemcpyHostToDevice, b->own),
                  ENUF_EDEVICE);
  }
  b->nmem = (int)mem.size();
  b->lds_fwd = lf;
  b->lds_x = lx;
  b->lds_bwd = lb;
  b->pass_threads = tp;
  b->x_threads = tx;
  b->drop_graph();
  b->dirty = false;
  return ENUF_OK;
}

// Member table par (bin-count set par) on the device.
const BatchMember *batch_table(const enuf_batch *b, int par) { return b->dmem + (size_t)par * b->nmem; }

// The forces of one step of every member, after its pre kernel: pair forces
// and real space forked onto two side streams (fork = true) or kept on the
// batch stream, the mesh passes on the batch stream, joined before return.
// tm (eager single-stream steps only) brackets one stage with events.
hipError_t batch_forces(enuf_batch *b, const BatchMember *mt, bool fork, KernelTimer *tm) {
  const int *o = b->off;
  const int2 *mp = b->dmap;
  hipStream_t st = b->own;
  hipStream_t s0 = fork ? b->side[0] : st, s1 = fork ? b->side[1] : st;
  hipError_t e = hipSuccess;
  if (fork) {
    e = hipEventRecord(b->fork_ev, st);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->fork_ev, 0);
  }
  if (tm) tm->before(ENUF_K_DPD_PAIR, s0);
  if (e == hipSuccess) e = launch_batch_pair(mt, mp + o[1], o[2] - o[1], b->tune.pair_steps, s0);
  if (tm) tm->after(ENUF_K_DPD_PAIR, s0);
  if (fork && e == hipSuccess) e = hipEventRecord(b->join_ev[0], s0);
  if (tm) tm->before(ENUF_K_REAL, s1);
  if (e == hipSuccess) e = launch_batch_real(mt, mp + o[2], o[3] - o[2], s1);
  if (tm) tm->after(ENUF_K_REAL, s1);
  if (fork && e == hipSuccess) e = hipEventRecord(b->join_ev[1], s1);
  if (e == hipSuccess)
    e = launch_batch_recip(mt, b->precision, b->ik, mp + o[3], o[4] - o[3], mp + o[4], o[5] - o[4],
                           mp + o[5], o[6] - o[5], b->lds_fwd, b->lds_x, b->lds_bwd, b->pass_threads,
                           b->x_threads, st, tm);
  if (fork)
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(st, b->join_ev[k], 0);
  return e;
}

// One whole step of every member with table 0 (eager runs): pre, forces,
// combine and the energy reduction.
hipError_t batch_step(enuf_batch *b, bool fork, KernelTimer *tm = nullptr) {
  const int *o = b->off;
  const int2 *mp = b->dmap;
  hipStream_t st = b->own;
  const BatchMember *mt = batch_table(b, 0);
  if (tm) tm->before(ENUF_K_DPD_PRE, st);
  hipError_t e = launch_batch_pre(mt, mp + o[0], o[1] - o[0], 0, st);
  if (tm) tm->after(ENUF_K_DPD_PRE, st);
  if (e == hipSuccess) e = batch_forces(b, mt, fork, tm);
  if (tm) tm->before(ENUF_K_COMBINE, st);
  if (e == hipSuccess) e = launch_batch_combine(mt, b->nmem, mp + o[6], o[7] - o[6], 0, st);
  if (tm) tm->after(ENUF_K_COMBINE, st);
  return e;
}

// The step graph [kind][par] (captured on first use): the forces of table
// par, then (kind 0) the fused combine + pre kernel that bins the next step
// into the other set, or (kind 1, a run's last step) the combine and the
// energy reduction.  Single stream: no cross-stream event in a capture.
int batch_capture(enuf_batch *b, int kind, int par) {
  if (b->exec[kind][par]) return ENUF_OK;
  const int *o = b->off;
  const int2 *mp = b->dmap;
  const BatchMember *mt = batch_table(b, par);
  HIP_OR_RETURN(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal), ENUF_EDEVICE);
  hipError_t e = batch_forces(b, mt, false, nullptr);
  if (e == hipSuccess)
    e = kind == 0 ? launch_batch_combine_pre(mt, mp + o[6], o[7] - o[6], b->own)
                  : launch_batch_combine(mt, b->nmem, mp + o[6], o[7] - o[6], 0, b->own);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->own, &g);
  if (e != hipSuccess || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    set_error(std::string("capturing the batched step failed: ") + hipGetErrorString(e != hipSuccess ? e : ec));
    return ENUF_EDEVICE;
  }
  b->graph[kind][par] = g;
  if (hipGraphInstantiate(&b->exec[kind][par], g, nullptr, nullptr, 0) != hipSuccess) {
    b->exec[kind][par] = nullptr;
    b->drop_graph();
    set_error("instantiating the batched step graph failed");
    return ENUF_EDEVICE;
  }
  return ENUF_OK;
}

}  // namespace

extern "C" {

enuf_batch *enuf_batch_create(int precision) {
  g_last_error.clear();
  if (precision != ENUF_FP64 && precision != ENUF_MIXED) { set_error("unknown precision"); return nullptr; }
  enuf_batch *b = new enuf_batch();
  b->precision = precision;
  if (hipGetDevice(&b->device) != hipSuccess) { set_error("hipGetDevice failed"); delete b; return nullptr; }
  for (int k = 0; k < 2; ++k) {
    if (hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join_ev[k], hipEventDisableTiming) != hipSuccess) {
      set_error("creating the side streams failed");
      delete b;
      return nullptr;
    }
  }
  if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->in_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->out_ev, hipEventDisableTiming) != hipSuccess) {
    set_error("creating the batch stream or events failed");
    delete b;
    return nullptr;
  }
  return b;
}

void enuf_batch_destroy(enuf_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->own);
  (void)hipStreamSynchronize(b->stream);
  for (auto &mb : b->members) --mb.d->batches;
  delete b;
}

int enuf_batch_set_stream(enuf_batch *b, void *hip_stream) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  if ((hipStream_t)hip_stream == b->stream) return ENUF_OK;  // keeps the captured graph
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  HIP_OR_RETURN(hipStreamSynchronize(b->stream), ENUF_EDEVICE);
  b->stream = (hipStream_t)hip_stream;
  for (auto &mb : b->members) {
    mb.d->stream = b->stream;
    mb.d->plan->stream = b->stream;
  }
  b->drop_graph();
  return ENUF_OK;
}

int enuf_batch_set_options(enuf_batch *b, int use_graph, int concurrent) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  if (use_graph < 0 || use_graph > ENUF_GRAPH_AUTO) { set_error("use_graph must be 0, 1 or ENUF_GRAPH_AUTO"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  b->use_graph = use_graph;
  b->concurrent = concurrent ? 1 : 0;
  b->drop_graph();
  return ENUF_OK;
}

int enuf_batch_set_tuning(enuf_batch *b, int pass_threads, int x_threads, int stage, int pair_steps,
                          int x_split_mul, int pair_seg) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  enuf_batch::Tuning t = b->tune;
  if (pass_threads) t.pass_threads = pass_threads;
  if (x_threads) t.x_threads = x_threads;
  if (stage) t.stage = stage;
  if (pair_steps) t.pair_steps = pair_steps;
  if (x_split_mul) t.x_split_mul = x_split_mul;
  if (pair_seg) t.pair_seg = pair_seg;
  if (t.pass_threads != 256 && t.pass_threads != 512) { set_error("pass_threads must be 256 or 512"); return ENUF_EINVAL; }
  if (t.x_threads != 128 && t.x_threads != 256 && t.x_threads != 512) {
    set_error("x_threads must be 128, 256 or 512");
    return ENUF_EINVAL;
  }
  if (t.stage < 32 || t.stage > kStage) { set_error("stage must be in [32, " + std::to_string(kStage) + "]"); return ENUF_EINVAL; }
  if (t.pair_steps != 4 && t.pair_steps != 8) { set_error("pair_steps must be 4 or 8"); return ENUF_EINVAL; }
  if (t.x_split_mul < 1 || t.x_split_mul > 8) { set_error("x_split_mul must be in [1, 8]"); return ENUF_EINVAL; }
  if (t.pair_seg < 1 || t.pair_seg > kPairSegMax) {
    set_error("pair_seg must be in [1, " + std::to_string(kPairSegMax) + "]");
    return ENUF_EINVAL;
  }
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  b->tune = t;
  b->dirty = true;  // rebuilt (and the graph dropped) at the next run
  return ENUF_OK;
}

int enuf_batch_add(enuf_batch *b, enuf_dpd *d, double *pos, double *vel, double *force, uint64_t first_step) {
  if (!b || !d) { set_error("NULL batch or integrator"); return ENUF_EINVAL; }
  if (!pos || !vel || !force) { set_error("NULL buffer"); return ENUF_EINVAL; }
  if (!d->plan) { set_error("batched integrators need an ENUF plan"); return ENUF_EINVAL; }
  if (d->plan->precision != b->precision) { set_error("integrator precision differs from the batch's"); return ENUF_EINVAL; }
  if (d->device != b->device || d->plan->device != b->device) { set_error("integrator on another device"); return ENUF_EINVAL; }
  const ComputeConfig &cf = d->plan->cfg;
  if (cf.lds_fwd > d->plan->max_lds || cf.lds_bwd > d->plan->max_lds || cf.lds_x > d->plan->max_lds) {
    set_error("mesh too large for the LDS in this precision");
    return ENUF_EINVAL;
  }
  for (const auto &mb : b->members)
    if (mb.d == d) { set_error("integrator is already a member"); return ENUF_EINVAL; }
  if (!b->members.empty() && cf.mesh.ik != b->ik) {
    set_error("integrator force mode differs from the other members'");
    return ENUF_EINVAL;
  }
  // the member's own stream may still be working on it
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  d->stream = b->stream;
  d->plan->stream = b->stream;
  HIP_OR_RETURN(launch_set_u64(d->step_ctr, (unsigned long long)first_step, b->stream), ENUF_EDEVICE);
  enuf_batch::Member mb{b->next_id++, d, pos, vel, force};
  b->members.push_back(mb);
  ++d->batches;
  b->ik = cf.mesh.ik;
  b->dirty = true;
  return mb.id;
}

int enuf_batch_remove(enuf_batch *b, int id) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  for (size_t k = 0; k < b->members.size(); ++k) {
    if (b->members[k].id == id) {
      HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
      HIP_OR_RETURN(hipStreamSynchronize(b->stream), ENUF_EDEVICE);
      --b->members[k].d->batches;
      b->members.erase(b->members.begin() + (long)k);
      b->dirty = true;
      return ENUF_OK;
    }
  }
  set_error("no member with this id");
  return ENUF_EINVAL;
}

int enuf_batch_size(const enuf_batch *b) { return b ? (int)b->members.size() : 0; }

int enuf_batch_run(enuf_batch *b, int nsteps) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return ENUF_EINVAL; }
  if (b->members.empty() || nsteps == 0) return ENUF_OK;
  int dev = -1;
  HIP_OR_RETURN(hipGetDevice(&dev), ENUF_EDEVICE);
  if (dev != b->device) { set_error("the batch's device is not current"); return ENUF_EINVAL; }
  if (b->dirty) {
    const int rc = batch_rebuild(b);
    if (rc != ENUF_OK) return rc;
  }
  // Replayed runs: the first pre kernel, then steps whose combine is fused
  // with the next step's pre kernel, alternating the two bin-count sets (step
  // s of the run uses set s mod 2), and the last step with its energy
  // reduction; every set is clear again at the end.  Eager and timed runs
  // launch whole steps with set 0.
  KernelTimer *tm = b->timer.active();
  const bool graph = !tm && (b->use_graph == 1 ||
                             (b->use_graph == ENUF_GRAPH_AUTO && (b->captured() || nsteps >= ENUF_GRAPH_AUTO_STEPS)));
  if (graph) {
    for (int s = 0; s < nsteps - 1 && s < 2; ++s) {
      const int rc = batch_capture(b, 0, s & 1);
      if (rc != ENUF_OK) return rc;
    }
    const int rc = batch_capture(b, 1, (nsteps - 1) & 1);
    if (rc != ENUF_OK) return rc;
  }
  // order after the caller's stream, run on the batch stream, order the
  // caller's later work after the run
  HIP_OR_RETURN(hipEventRecord(b->in_ev, b->stream), ENUF_EDEVICE);
  HIP_OR_RETURN(hipStreamWaitEvent(b->own, b->in_ev, 0), ENUF_EDEVICE);
  if (graph) {
    hipError_t e = launch_batch_pre(batch_table(b, 0), b->dmap + b->off[0], b->off[1] - b->off[0], 0, b->own);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s)
      e = hipGraphLaunch(b->exec[s == nsteps - 1 ? 1 : 0][s & 1], b->own);
    if (e != hipSuccess) {
      set_error(std::string("batched step launch failed: ") + hipGetErrorString(e));
      return ENUF_EDEVICE;
    }
  } else {
    for (int s = 0; s < nsteps; ++s) {
      const hipError_t e = batch_step(b, !tm && b->concurrent != 0, tm);
      if (e != hipSuccess) {
        set_error(std::string("batched step launch failed: ") + hipGetErrorString(e));
        return ENUF_EDEVICE;
      }
    }
  }
  HIP_OR_RETURN(hipEventRecord(b->out_ev, b->own), ENUF_EDEVICE);
  HIP_OR_RETURN(hipStreamWaitEvent(b->stream, b->out_ev, 0), ENUF_EDEVICE);
  return ENUF_OK;
}

int enuf_dpd_set_species(enuf_dpd *d, int nspecies, const int *species, const double *a_table) {
  if (!d) { set_error("NULL integrator"); return ENUF_EINVAL; }
  if (nspecies < 1 || nspecies > 4) { set_error("nspecies must be in [1, 4]"); return ENUF_EINVAL; }
  if (!a_table || (nspecies > 1 && !species)) { set_error("NULL species or amplitude table"); return ENUF_EINVAL; }
  if (d->batches > 0) { set_error("the integrator is a member of a batch"); return ENUF_EINVAL; }
  for (int s = 0; s < nspecies; ++s)
    for (int t = 0; t < nspecies; ++t) {
      const double v = a_table[s * nspecies + t];
      if (!std::isfinite(v)) { set_error("non-finite amplitude"); return ENUF_EINVAL; }
      if (v != a_table[t * nspecies + s]) { set_error("the amplitude table must be symmetric"); return ENUF_EINVAL; }
    }
  const size_t n = (size_t)d->N;
  if (nspecies > 1)
    for (size_t i = 0; i < n; ++i)
      if (species[i] < 0 || species[i] >= nspecies) { set_error("species out of range"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  DpdParams &P = d->P;
  if (nspecies == 1) {
    P.a = a_table[0];
    P.nspec = 0;
    return ENUF_OK;
  }
  HIP_OR_RETURN(hipMemcpy(d->species, species, n * sizeof(int), hipMemcpyHostToDevice), ENUF_EDEVICE);
  for (int k = 0; k < 16; ++k) P.atab[k] = 0.0;
  for (int s = 0; s < nspecies; ++s)
    for (int t = 0; t < nspecies; ++t) P.atab[4 * s + t] = a_table[s * nspecies + t];
  P.nspec = nspecies;
  return ENUF_OK;
}

int enuf_batch_time_kernel(enuf_batch *b, int kernel, int max_launches) {
  if (!b) { set_error("NULL batch"); return ENUF_EINVAL; }
  if (!valid_timer_args(kernel, max_launches)) { set_error("invalid kernel id or launch count"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  if (!b->timer.start(kernel, max_launches)) { set_error("hipEventCreate failed"); return ENUF_EDEVICE; }
  return ENUF_OK;
}

int enuf_batch_kernel_time(enuf_batch *b, double *total_ms, int *launches) {
  if (!b || !total_ms || !launches) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(b->own), ENUF_EDEVICE);
  HIP_OR_RETURN(b->timer.total(total_ms, launches), ENUF_EDEVICE);
  return ENUF_OK;
}

size_t enuf_batch_footprint_bytes(const enuf_batch *b) {
  if (!b) return 0;
  size_t t = 2 * b->mem_cap * sizeof(BatchMember) + b->map_cap * sizeof(int2);
  for (const auto &mb : b->members) t += enuf_dpd_footprint_bytes(mb.d);
  return t;
}

int enuf_pair_histogram(const double *pos, int64_t n, int64_t nsel, const int64_t *sel, const int *cls, int ncls,
                        double box, double r_max, int nbins, unsigned long long *hist, void *hip_stream) {
  if (n < 0 || nsel < 0 || ncls < 1 || nbins < 1) { set_error("invalid sizes"); return ENUF_EINVAL; }
  if ((int64_t)ncls * ncls * nbins > kHistMaxBins) { set_error("classes^2 x bins exceeds 12288"); return ENUF_EINVAL; }
  if (nsel > kHistMaxSel) { set_error("too many selected particles"); return ENUF_EINVAL; }
  if (!(std::isfinite(box) && box > 0.0) || !(std::isfinite(r_max) && r_max > 0.0)) {
    set_error("box and r_max must be finite and > 0");
    return ENUF_EINVAL;
  }
  if (!hist || (nsel > 0 && (!pos || !sel || !cls))) { set_error("NULL buffer"); return ENUF_EINVAL; }
  HIP_OR_RETURN(launch_pair_histogram(pos, n, nsel, sel, cls, ncls, box, r_max, nbins, hist,
                                      (hipStream_t)hip_stream),
                ENUF_EDEVICE);
  return ENUF_OK;
}

int enuf_chain_rg2(const double *pos, int64_t n, int nchains, int len, const int64_t *beads, double box, double *out,
                   void *hip_stream) {
  if (n < 0 || nchains < 0 || len < 1) { set_error("invalid sizes"); return ENUF_EINVAL; }
  if (!(std::isfinite(box) && box > 0.0)) { set_error("box must be finite and > 0"); return ENUF_EINVAL; }
  if (nchains > 0 && (!pos || !beads || !out)) { set_error("NULL buffer"); return ENUF_EINVAL; }
  HIP_OR_RETURN(launch_chain_rg2(pos, n, nchains, len, beads, box, out, (hipStream_t)hip_stream), ENUF_EDEVICE);
  return ENUF_OK;
}

}  // extern "C"
