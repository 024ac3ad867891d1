// enuf_internal.h -- definitions shared by the library's host runtime and its
// HIP kernels (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace enuf {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kPrepThreads = 256;  // threads per block of the particle-parallel kernels
constexpr int kPassThreads = 512;  // threads per block of the mesh-plane kernels
constexpr int kMaxRadixPasses = 16;

// Device-resident scalars produced by the preparation kernels of one compute.
struct DevScalars {
  int nq;               // number of charged particles (compacted prefix of xq)
  int status;           // sticky ENUF_* data error (0 = OK), cleared by the host
  double scale;         // fixed-point scale of the mesh accumulator (power of 2)
  double inv_scale;
  double sum_q;         // sum q, sum |q|, sum q^2 (fixed-order reductions)
  double sum_absq;
  double sum_q2;
};

// Mixed-radix factorisation of an FFT length, radices in {2, 3, 4, 5}.
struct FftPlan {
  int n;
  int npass;
  int radix[kMaxRadixPasses];
};

// NFFT window, normalised to phi(0) = 1.  u is the offset t - l in mesh cells.
struct WindowParams {
  int kind;        // ENUF_WINDOW_KB or ENUF_WINDOW_GAUSS
  int p;           // half-width; 2p stencil points per axis
  double b;        // Kaiser-Bessel shape pi (2 - 1/sigma)
  double c1;       // 1 / (1 - exp(-2 b p))
  double inv_sinh_bp;  // 1 / sinh(b p)
  double inv_bg;   // Gaussian: 1 / b_G, b_G = 2 sigma p / ((2 sigma - 1) pi)
};

// Geometry shared by the mesh kernels.
struct MeshParams {
  int M;           // mesh points per side
  int Mp;          // padded row stride of LDS planes (elements)
  int Mz;          // padded line stride of LDS spectrum buffers (elements)
  int Kc;          // reciprocal cutoff: 0 < |k| < Kc
  int nky;         // 2 Kc - 1 stored ky values (ky = idx - (Kc - 1))
  double L;
  double m_over_l; // M / L: mesh coordinate t = x * m_over_l
  WindowParams win;
  FftPlan fft;
};

// Real-space cell grid of the charges (cell edge >= r_cut).
struct CellParams {
  int ncell;       // cells per side
  int cap;         // slots per cell
  double inv_cell; // ncell / L
};

// Status codes mirrored from enuf.h for device code.
constexpr int kOK = 0;
constexpr int kENonNeutral = -4;
constexpr int kENonFinite = -5;
constexpr int kECoincident = -7;
constexpr int kEOverflow = -8;

// Fixed-point scale of the real-space force / energy accumulators.  Pair terms
// are rounded to 2^-36 (1.5e-11) and summed exactly in int64, which makes the
// sums independent of the order in which pairs are visited.
constexpr double kRealFxScale = 68719476736.0;  // 2^36
constexpr double kRealFxInv = 1.0 / 68719476736.0;
constexpr double kFxLimit = 4.0e18;             // |value * scale| beyond this overflows

// ---------------------------------------------------------------------------
// Host-side launchers (defined in enuf_kernels.hip).
// ---------------------------------------------------------------------------
struct ComputeBuffers {
  // preparation
  int *blk_cnt;          // [nblk]
  double *blk_sums;      // [nblk * 3]
  unsigned *done;        // [2] last-block tickets (prep, combine)
  DevScalars *sc;
  double4 *xq;           // [N] compacted (x, y, z, q), wrapped into [0, L)
  int *idx;              // [N] particle index of compact slot j
  int *slot;             // [N] compact slot of particle i, or -1
  // real-space cell grid
  int *ccnt;             // [ncell^3]
  double4 *cgrid;        // [ncell^3 * cap] (x, y, z, q) per cell slot
  int *cidx;             // [ncell^3 * cap] compact index per cell slot
  unsigned long long *freal;  // [N * 3] fixed-point real-space forces per slot (zero between calls)
  unsigned long long *eacc;  // [2] fixed-point E_real (whole), E_slater
  // reciprocal
  void *gzy;             // [M * nky * Kc] complex (double2 or float2)
  double *epart;         // [nky] k-space energy per ky row
  double4 *part;         // [N * 2p] gather partials (dwx A, wx By, wx Bz, wx A)
  void *winv;            // [N * 3 * 2p] window values per charge, axis, offset (double or float)
  void *wind;            // [N * 3 * 2p] window derivatives
  int *mbase;            // [N * 4] first stencil index per axis
  double *blk_eg;        // [nblk] per-block sums of q * A
  // tables
  double *atab;          // [nky] exp(-pi^2 k^2/(alpha L)^2) / Phi(k/M)^2
  double2 *tw64;         // [M] exp(-2 pi i m / M)
  float2 *tw32;          // [M]
};

struct ComputeConfig {
  int64_t N;
  int nblk;              // ceil(N / kPrepThreads)
  double L;
  double alpha;
  double r_cut;
  double lambda;
  int precision;         // ENUF_FP64 / ENUF_MIXED
  MeshParams mesh;
  CellParams cells;
  size_t lds_fwd, lds_x, lds_bwd;  // dynamic LDS bytes of the three mesh passes
};

// Optional event timing of one kernel class (kernel ids as ENUF_K_* in enuf.h).
struct KernelTimer {
  int kernel = -1;
  int cap = 0;
  int count = 0;
  hipEvent_t *ev = nullptr;  // 2 * cap events
  void before(int k, hipStream_t s) {
    if (k == kernel && count < cap) (void)hipEventRecord(ev[2 * count], s);
  }
  void after(int k, hipStream_t s) {
    if (k == kernel && count < cap) {
      (void)hipEventRecord(ev[2 * count + 1], s);
      ++count;
    }
  }
};

hipError_t launch_compute(const ComputeConfig &cfg, const ComputeBuffers &b,
                          const double *pos, const double *q, double *forces,
                          double *energy_total, double *energy5, hipStream_t stream,
                          KernelTimer *timer = nullptr);

// LDS bytes the three mesh passes need for the given geometry and precision.
void mesh_lds_bytes(const MeshParams &m, int precision, size_t *fwd, size_t *x, size_t *bwd);

// Raise the per-kernel dynamic LDS limit where needed (once per process).
hipError_t configure_kernels(size_t max_lds);

}  // namespace enuf
