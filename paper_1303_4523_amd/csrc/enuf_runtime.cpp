// enuf_runtime.cpp -- host side of the ENUF C ABI: argument validation, window
// and influence tables, FFT factorisation, device buffers and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
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
  const int order[4] = {4, 2, 3, 5};
  for (int oi = 0; oi < 4; ++oi) {
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

struct enuf_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  double L = 0, alpha = 0, sigma = 0, r_cut = 0, lambda = 0;
  int p = 0, M = 0, Kc = 0;
  int precision = ENUF_FP64, window = ENUF_WINDOW_KB;
  size_t max_lds = 0;
  int part_slots = 1;      // gather partial slots allocated per (charge, x offset)
  ComputeConfig cfg{};
  ComputeBuffers buf{};
  std::vector<void *> allocations;
  size_t bytes = 0;

  void *alloc(size_t n) {
    void *ptr = nullptr;
    if (n == 0) n = 16;
    if (hipMalloc(&ptr, n) != hipSuccess) return nullptr;
    allocations.push_back(ptr);
    bytes += n;
    return ptr;
  }
  ~enuf_plan() {
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

int upload_window_series(enuf_plan *pl) {
  std::vector<long double> coef;
  const int fp32 = pl->precision == ENUF_MIXED;
  const int D = fit_window_series(pl->cfg.mesh.win, fp32, &coef);
  pl->cfg.mesh.cheb_deg = D;
  const size_t n = coef.size();
  if (fp32) {
    std::vector<float> h(n);
    for (size_t k = 0; k < n; ++k) h[k] = (float)coef[k];
    HIP_OR_RETURN(hipMemcpy(pl->buf.wcoef32, h.data(), n * sizeof(float), hipMemcpyHostToDevice), ENUF_EDEVICE);
  } else {
    std::vector<double> h(n);
    for (size_t k = 0; k < n; ++k) h[k] = (double)coef[k];
    HIP_OR_RETURN(hipMemcpy(pl->buf.wcoef64, h.data(), n * sizeof(double), hipMemcpyHostToDevice), ENUF_EDEVICE);
  }
  return ENUF_OK;
}

int upload_tables(enuf_plan *pl) {
  const int Kc = pl->Kc, M = pl->M, nky = 2 * Kc - 1;
  const WindowParams &w = pl->cfg.mesh.win;
  std::vector<double> atab(nky);
  const long double aL = (long double)pl->alpha * pl->L;
  for (int i = 0; i < nky; ++i) {
    const long double k = (long double)(i - (Kc - 1));
    const long double ph = window_hat(w, k / (long double)M);
    atab[i] = (double)(std::exp(-(long double)M_PI * (long double)M_PI * k * k / (aL * aL)) / (ph * ph));
  }
  std::vector<double2> tw64(M);
  std::vector<float2> tw32(M);
  for (int m = 0; m < M; ++m) {
    const long double ang = -2.0L * (long double)M_PI * (long double)m / (long double)M;
    tw64[m] = make_double2((double)std::cos(ang), (double)std::sin(ang));
    tw32[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  HIP_OR_RETURN(hipMemcpy(pl->buf.atab, atab.data(), nky * sizeof(double), hipMemcpyHostToDevice), ENUF_EDEVICE);
  HIP_OR_RETURN(hipMemcpy(pl->buf.tw64, tw64.data(), M * sizeof(double2), hipMemcpyHostToDevice), ENUF_EDEVICE);
  HIP_OR_RETURN(hipMemcpy(pl->buf.tw32, tw32.data(), M * sizeof(float2), hipMemcpyHostToDevice), ENUF_EDEVICE);
  return upload_window_series(pl);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" {

const char *enuf_last_error(void) { return g_last_error.c_str(); }

enuf_plan *enuf_plan_create(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc,
                            double r_cut, double lambda) {
  g_last_error.clear();
  // ---- validation (host only; no device call before it passes) ----
  if (N < 1 || N > (int64_t)1 << 28) { set_error("N must be in [1, 2^28]"); return nullptr; }
  if (!finite_pos(box)) { set_error("box must be finite and > 0"); return nullptr; }
  if (!finite_pos(alpha)) { set_error("alpha must be finite and > 0"); return nullptr; }
  if (!(std::isfinite(sigma) && sigma >= 1.0)) { set_error("sigma must be finite and >= 1"); return nullptr; }
  if (p < 1 || p > 15) { set_error("p must be in [1, 15]"); return nullptr; }
  if (M < 4 || M % 2 != 0 || M > 4096) { set_error("M must be even and in [4, 4096]"); return nullptr; }
  FftPlan fp{};
  if (!factor_235(M, &fp)) { set_error("M must be of the form 2^a 3^b 5^c"); return nullptr; }
  if (2 * p > M / 2) { set_error("need 2p <= M/2"); return nullptr; }
  if (Kc < 1 || (double)Kc > (double)M / (2.0 * sigma)) { set_error("need 1 <= Kc <= M/(2 sigma)"); return nullptr; }
  if (!finite_pos(r_cut) || r_cut > 0.5 * box) { set_error("need 0 < r_cut <= box/2"); return nullptr; }
  if (!(std::isfinite(lambda) && lambda >= 0.0)) { set_error("lambda must be finite and >= 0"); return nullptr; }

  enuf_plan *pl = new enuf_plan();
  pl->N = N; pl->L = box; pl->alpha = alpha; pl->sigma = sigma; pl->r_cut = r_cut; pl->lambda = lambda;
  pl->p = p; pl->M = M; pl->Kc = Kc;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    set_error("hipGetDevice failed");
    delete pl;
    return nullptr;
  }
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device) != hipSuccess) {
    set_error("hipDeviceGetAttribute failed");
    delete pl;
    return nullptr;
  }
  pl->max_lds = (size_t)lds;
  // optional lower LDS budget per block: forces the row-chunked plane passes
  if (const char *cap = std::getenv("ENUF_MAX_LDS_BYTES")) {
    const long long v = std::atoll(cap);
    if (v > 0 && (size_t)v < pl->max_lds) pl->max_lds = (size_t)v;
  }

  ComputeConfig &c = pl->cfg;
  c.N = N;
  c.nblk = (int)((N + kPrepThreads - 1) / kPrepThreads);
  c.L = box; c.alpha = alpha; c.r_cut = r_cut; c.lambda = lambda;
  c.precision = ENUF_FP64;
  MeshParams &m = c.mesh;
  m.M = M; m.Mp = M + 1; m.Mz = M + 1; m.Kc = Kc; m.nky = 2 * Kc - 1;
  m.L = box; m.m_over_l = (double)M / box;
  m.win = make_window(ENUF_WINDOW_KB, p, sigma);
  m.fft = fp;
  int ncell = (int)std::floor(box / r_cut);
  ncell = ncell < 1 ? 1 : (ncell > 1024 ? 1024 : ncell);
  const double mean = (double)N / ((double)ncell * ncell * ncell);
  c.cells.ncell = ncell;
  c.cells.cap = (int)std::ceil(mean + 6.0 * std::sqrt(mean) + 16.0);
  c.cells.inv_cell = (double)ncell / box;
  const double xmean = (double)N / (double)M;
  m.xcap = (int)std::ceil(xmean + 6.0 * std::sqrt(xmean) + 16.0);
  // Row chunking of the plane passes; the gather partials are sized for the
  // largest series degree in either precision.
  m.cheb_deg = kMaxChebDeg;
  int part_slots = 0;
  for (int prec = ENUF_FP64; prec <= ENUF_MIXED; ++prec) {
    MeshParams t = m;
    if (mesh_choose_rows(t, prec, pl->max_lds)) part_slots = t.nslot > part_slots ? t.nslot : part_slots;
  }
  if (part_slots == 0) {
    set_error("mesh too large: no row chunking of the plane passes fits in " + std::to_string(pl->max_lds) +
              " bytes of LDS");
    delete pl;
    return nullptr;
  }
  pl->part_slots = part_slots;
  m.rows = M;
  m.nchunk = 1;
  m.nslot = 1;
  mesh_lds_bytes(m, 0, &c.lds_fwd, &c.lds_x, &c.lds_bwd);

  ComputeBuffers &b = pl->buf;
  const size_t nblk = c.nblk, n = (size_t)N, ncell3 = (size_t)ncell * ncell * ncell;
  const size_t P2 = 2 * (size_t)p;
  b.blk_cnt = (int *)pl->alloc(nblk * sizeof(int));
  b.blk_sums = (double *)pl->alloc(nblk * 3 * sizeof(double));
  b.done = (unsigned *)pl->alloc(4 * sizeof(unsigned));
  b.sc = (DevScalars *)pl->alloc(sizeof(DevScalars));
  b.xq = (double4 *)pl->alloc(n * sizeof(double4));
  b.idx = (int *)pl->alloc(n * sizeof(int));
  b.slot = (int *)pl->alloc(n * sizeof(int));
  b.ccnt = (int *)pl->alloc(ncell3 * sizeof(int));
  b.cgrid = (double4 *)pl->alloc(ncell3 * (size_t)c.cells.cap * sizeof(double4));
  b.cidx = (int *)pl->alloc(ncell3 * (size_t)c.cells.cap * sizeof(int));
  b.freal = (unsigned long long *)pl->alloc(n * 3 * sizeof(unsigned long long));
  b.eacc = (unsigned long long *)pl->alloc(4 * sizeof(unsigned long long));
  b.gzy = pl->alloc((size_t)M * m.nky * Kc * sizeof(double2));
  b.epart = (double *)pl->alloc((size_t)m.nky * sizeof(double));
  b.part = (double4 *)pl->alloc(n * P2 * (size_t)part_slots * sizeof(double4));
  b.blk_eg = (double *)pl->alloc(nblk * sizeof(double));
  b.xcnt = (int *)pl->alloc((size_t)M * sizeof(int));
  b.xslot = (int *)pl->alloc((size_t)M * (size_t)m.xcap * sizeof(int));
  b.wcoef64 = (double *)pl->alloc(P2 * (2 * kMaxChebDeg + 1) * sizeof(double));
  b.wcoef32 = (float *)pl->alloc(P2 * (2 * kMaxChebDeg + 1) * sizeof(float));
  b.atab = (double *)pl->alloc((size_t)m.nky * sizeof(double));
  b.tw64 = (double2 *)pl->alloc((size_t)M * sizeof(double2));
  b.tw32 = (float2 *)pl->alloc((size_t)M * sizeof(float2));
  if (pl->allocations.size() != 23) {  // alloc() records successful allocations only
    set_error("device allocation failed");
    delete pl;
    return nullptr;
  }
  if (hipMemset(b.done, 0, 4 * sizeof(unsigned)) != hipSuccess ||
      hipMemset(b.sc, 0, sizeof(DevScalars)) != hipSuccess ||
      hipMemset(b.freal, 0, n * 3 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(b.ccnt, 0, ncell3 * sizeof(int)) != hipSuccess ||
      hipMemset(b.xcnt, 0, (size_t)M * sizeof(int)) != hipSuccess) {
    set_error("hipMemset failed");
    delete pl;
    return nullptr;
  }
  if (upload_tables(pl) != ENUF_OK) {
    delete pl;
    return nullptr;
  }
  if (!mesh_choose_rows(m, ENUF_FP64, pl->max_lds) || m.nslot > pl->part_slots) {
    // FP64 does not fit; the plan stays usable after switching to the mixed mode
    m.rows = M;
    m.nchunk = 1;
    m.nslot = 1;
  }
  mesh_lds_bytes(m, ENUF_FP64, &c.lds_fwd, &c.lds_x, &c.lds_bwd);
  static bool configured = false;
  if (!configured) {
    if (configure_kernels(pl->max_lds) != hipSuccess) {
      set_error("hipFuncSetAttribute failed");
      delete pl;
      return nullptr;
    }
    configured = true;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
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
    return rc;
  }
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
  hipError_t e = launch_compute(c, plan->buf, pos, q, forces, energy, energy5, plan->stream);
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

}  // extern "C"

// ---------------------------------------------------------------------------
// DPD integrator
// ---------------------------------------------------------------------------
struct enuf_dpd {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  DpdParams P{};
  enuf_plan *plan = nullptr;  // not owned
  double *q = nullptr;        // [N]
  double *v0 = nullptr;       // [N * 3] predicted velocities
  double *fdpd = nullptr;     // [N * 3] pair + bond forces
  double *felec = nullptr;    // [N * 3]
  double *e5 = nullptr;       // [5]
  int *dcnt = nullptr;        // [ncell^3]
  double4 *cpos = nullptr;    // [ncell^3 * cap] (x, y, z, index) per cell slot
  double4 *cvel = nullptr;    // [ncell^3 * cap] predicted velocity per cell slot
  int *bond_start = nullptr;  // [N + 1]
  int *bond_to = nullptr;     // [2 nbonds]
  int *status = nullptr;      // [1]
  std::vector<void *> allocations;
  KernelTimer timer;
  std::vector<hipEvent_t> events;
  int *dslot = nullptr;       // [N] static compact slot of each particle (-1: neutral)
  int64_t nq = 0;
  DpdCharges charges{};
  hipStream_t side[2] = {nullptr, nullptr};  // forked streams (pair forces, real space)
  int concurrent = 1;
  hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};

  void *alloc(size_t n) {
    void *ptr = nullptr;
    if (n == 0) n = 16;
    if (hipMalloc(&ptr, n) != hipSuccess) return nullptr;
    allocations.push_back(ptr);
    return ptr;
  }
  void drop_events() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    timer = KernelTimer();
  }
  ~enuf_dpd() {
    drop_events();
    for (int k = 0; k < 2; ++k) {
      if (side[k]) (void)hipStreamDestroy(side[k]);
      if (join_ev[k]) (void)hipEventDestroy(join_ev[k]);
    }
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
  int nc = (int)std::floor(box);  // cell edge box / nc >= 1 = R_c
  nc = nc < 1 ? 1 : (nc > 1024 ? 1024 : nc);
  P.ncell = nc;
  const double mean = (double)N / ((double)nc * nc * nc);
  P.cap = (int)std::ceil(mean + 6.0 * std::sqrt(mean) + 16.0);
  P.inv_cell = (double)nc / box;
  const size_t n = (size_t)N, nc3 = (size_t)nc * nc * nc;
  d->q = (double *)d->alloc(n * sizeof(double));
  d->v0 = (double *)d->alloc(3 * n * sizeof(double));
  d->fdpd = (double *)d->alloc(3 * n * sizeof(double));
  d->felec = (double *)d->alloc(3 * n * sizeof(double));
  d->e5 = (double *)d->alloc(5 * sizeof(double));
  d->dcnt = (int *)d->alloc(nc3 * sizeof(int));
  d->cpos = (double4 *)d->alloc(nc3 * (size_t)P.cap * sizeof(double4));
  d->cvel = (double4 *)d->alloc(nc3 * (size_t)P.cap * sizeof(double4));
  d->bond_start = (int *)d->alloc((n + 1) * sizeof(int));
  d->bond_to = (int *)d->alloc(to.size() * sizeof(int));
  d->status = (int *)d->alloc(sizeof(int));
  d->dslot = (int *)d->alloc(n * sizeof(int));
  if (d->allocations.size() != 12) { set_error("device allocation failed"); delete d; return nullptr; }
  if (hipMemcpy(d->q, q, n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(d->bond_start, deg.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d->bond_to, to.data(), to.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(d->dcnt, 0, nc3 * sizeof(int)) != hipSuccess || hipMemset(d->e5, 0, 5 * sizeof(double)) != hipSuccess ||

      hipMemset(d->status, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
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
    ch.cidx = plan->buf.cidx;
    ch.cells = plan->cfg.cells;
    ch.xcnt = plan->buf.xcnt;
    ch.xslot = plan->buf.xslot;
    ch.M = plan->cfg.mesh.M;
    ch.xcap = plan->cfg.mesh.xcap;
    ch.m_over_l = plan->cfg.mesh.m_over_l;
    ch.sc = plan->buf.sc;
    ch.eacc = plan->buf.eacc;
    ch.stat = st;
  }
  for (int k = 0; k < 2; ++k) {
    if (hipStreamCreateWithFlags(&d->side[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&d->join_ev[k], hipEventDisableTiming) != hipSuccess) {
      set_error("creating the side streams failed");
      delete d;
      return nullptr;
    }
  }
  if (hipEventCreateWithFlags(&d->fork_ev, hipEventDisableTiming) != hipSuccess) {
    set_error("creating the fork event failed");
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

// One force evaluation (mode 1) or step (mode 0).  With a plan the pair
// forces and the real-space term run on two forked streams while the mesh
// passes run on the integrator's stream; the combine kernel joins them.
static int dpd_eval(enuf_dpd *d, int mode, double *pos, double *vel, double *force, uint64_t step) {
  const int64_t N = d->N;
  KernelTimer *tm = d->timer.kernel >= 0 ? &d->timer : nullptr;
  hipStream_t st = d->stream;
  hipError_t e = launch_dpd_pre(N, mode, d->P, pos, vel, force, d->v0, d->dcnt, d->cpos, d->cvel, d->status,
                                d->charges, st, tm);
  if (!d->plan) {
    if (e == hipSuccess)
      e = launch_dpd_pair(N, d->P, step, pos, d->v0, d->dcnt, d->cpos, d->cvel, d->bond_start, d->bond_to,
                          d->fdpd, st, tm);
    if (e == hipSuccess) e = launch_dpd_post(N, mode, d->P, d->fdpd, nullptr, force, vel, d->dcnt, st, tm);
  } else {
    enuf_plan *pl = d->plan;
    pl->stream = st;
    const bool fork = d->concurrent != 0;
    hipStream_t s0 = fork ? d->side[0] : st, s1 = fork ? d->side[1] : st;
    if (fork) {
      if (e == hipSuccess) e = hipEventRecord(d->fork_ev, st);
      for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(d->side[k], d->fork_ev, 0);
    }
    if (e == hipSuccess)
      e = launch_dpd_pair(N, d->P, step, pos, d->v0, d->dcnt, d->cpos, d->cvel, d->bond_start, d->bond_to,
                          d->fdpd, s0, tm);
    if (fork && e == hipSuccess) e = hipEventRecord(d->join_ev[0], s0);
    if (e == hipSuccess) e = launch_real(pl->cfg, pl->buf, d->nq, s1, tm);
    if (fork && e == hipSuccess) e = hipEventRecord(d->join_ev[1], s1);
    if (e == hipSuccess) e = launch_recip(pl->cfg, pl->buf, d->nq, st, tm);
    if (fork)
      for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(st, d->join_ev[k], 0);
    if (e == hipSuccess) {
      FinishArgs fa;
      fa.mode = mode;
      fa.kappa = d->P.kappa;
      fa.dt = d->P.dt;
      fa.fdpd = d->fdpd;
      fa.vel = vel;
      fa.dcnt = d->dcnt;
      fa.ndcell3 = d->P.ncell * d->P.ncell * d->P.ncell;
      e = launch_combine(pl->cfg, pl->buf, force, nullptr, d->e5, fa, st, tm);
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
  return dpd_eval(d, 1, pos, const_cast<double *>(vel), force, step);
}

int enuf_dpd_run(enuf_dpd *d, double *pos, double *vel, double *force, uint64_t first_step, int nsteps) {
  int rc = dpd_check(d, pos, vel, force);
  if (rc != ENUF_OK) return rc;
  if (nsteps < 0) { set_error("nsteps must be >= 0"); return ENUF_EINVAL; }
  for (int s = 0; s < nsteps; ++s) {
    rc = dpd_eval(d, 0, pos, vel, force, first_step + (uint64_t)s);
    if (rc != ENUF_OK) return rc;
  }
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
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  d->drop_events();
  if (kernel < 0) return ENUF_OK;
  if (kernel > ENUF_K_DPD_POST || max_launches < 1 || max_launches > (1 << 20)) {
    set_error("invalid kernel id or launch count");
    return ENUF_EINVAL;
  }
  d->events.resize(2 * (size_t)max_launches);
  for (size_t k = 0; k < d->events.size(); ++k) {
    if (hipEventCreate(&d->events[k]) != hipSuccess) {
      d->events.resize(k);
      d->drop_events();
      set_error("hipEventCreate failed");
      return ENUF_EDEVICE;
    }
  }
  d->timer.kernel = kernel;
  d->timer.cap = max_launches;
  d->timer.count = 0;
  d->timer.ev = d->events.data();
  return ENUF_OK;
}

int enuf_dpd_kernel_time(enuf_dpd *d, double *total_ms, int *launches) {
  if (!d || !total_ms || !launches) { set_error("NULL argument"); return ENUF_EINVAL; }
  HIP_OR_RETURN(hipStreamSynchronize(d->stream), ENUF_EDEVICE);
  double t = 0.0;
  for (int k = 0; k < d->timer.count; ++k) {
    float ms = 0.0f;
    HIP_OR_RETURN(hipEventElapsedTime(&ms, d->events[2 * k], d->events[2 * k + 1]), ENUF_EDEVICE);
    t += ms;
  }
  *total_ms = t;
  *launches = d->timer.count;
  return ENUF_OK;
}

void enuf_dpd_destroy(enuf_dpd *d) {
  if (!d) return;
  (void)hipStreamSynchronize(d->stream);
  delete d;
}

}  // extern "C"
