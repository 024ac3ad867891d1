// enuf_internal.h -- definitions shared by the library's host runtime and its
// HIP kernels (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace enuf {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kPrepThreads = 256;  // threads per block of the particle-parallel kernels
constexpr int kPassThreads = 512;  // threads per block of the mesh-plane kernels
constexpr int kXSub = 8;           // sub-bins of a mesh x-cell (by compact index mod 8): the binning's
                                   // slot counters are shared by 8 times fewer charges
constexpr int kMaxRadixPasses = 16;
constexpr int kMaxChebDeg = 24;    // highest degree of the window series
constexpr int kStage = 512;        // most charges of a plane staged in LDS at a time by the mesh passes
// Batched mesh passes: work-groups of kBatchPassThreads threads staging at most
// kBatchStage charges, so that two work-groups share a CU (the passes need
// about 200-256 VGPRs per lane, two waves per SIMD): one work-group's waits on
// memory and barriers overlap the other's work.
constexpr int kBatchPassThreads = 256;
constexpr int kBatchStage = 256;
// The batched x pass (no charges, little LDS) in work-groups of 128 threads:
// four share a CU.
constexpr int kBatchXThreads = 128;
constexpr int kMaxParts = 8;       // most work-groups per plane in the spread and gather passes

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

// Mixed-radix factorisation of an FFT length, radices in {2, 3, 4, 5, 8}.
struct FftPlan {
  int n;
  int npass;
  int radix[kMaxRadixPasses];
};

// Most butterflies per line of any radix pass of a plan: the LDS transforms
// give each butterfly of a line its own thread, so a work-group needs at least
// this many threads.
inline int fft_max_butterflies(const FftPlan &f) {
  int b = 0;
  for (int k = 0; k < f.npass; ++k) b = f.n / f.radix[k] > b ? f.n / f.radix[k] : b;
  return b;
}

// NFFT window, normalised to phi(0) = 1.  u is the offset t - l in mesh cells.
struct WindowParams {
  int kind;        // ENUF_WINDOW_KB or ENUF_WINDOW_GAUSS
  int p;           // half-width; 2p stencil points per axis
  double b;        // Kaiser-Bessel shape pi (2 - 1/sigma)
  double c1;       // 1 / (1 - exp(-2 b p))
  double inv_sinh_bp;  // 1 / sinh(b p)
  double inv_bg;   // Gaussian: 1 / b_G, b_G = 2 sigma p / ((2 sigma - 1) pi)
};

// Geometry shared by the mesh kernels.  The window is evaluated from
// piecewise Chebyshev series: on stencil offset s the window at
// u = frac + p - 1 - s (frac in [0, 1)) is sum_k c_{s,k} T_k(2 frac - 1),
// and its u-derivative a series of degree cheb_deg - 1.  Table layout:
// [2p][cheb_deg + 1] value series, then [2p][cheb_deg + 1] derivative series
// (last coefficient 0), so that both kinds evaluate in one recurrence.
struct MeshParams {
  int cheb_deg;    // degree of the value series (derivative: cheb_deg - 1)
  int xcap;        // slots per x-cell sub-bin of the charge binning
  int M;           // mesh points per side
  int Mp;          // padded row stride of LDS planes (elements)
  int Mz;          // padded line stride of LDS spectrum buffers (elements)
  int Kc;          // reciprocal cutoff: 0 < |k| < Kc
  int nky;         // 2 Kc - 1 stored ky values (ky = idx - (Kc - 1))
  int rows;        // mesh rows (y) per LDS chunk of a plane pass; even, >= 2p when < M
  int nchunk;      // ceil(M / rows)
  int nslot;       // gather partials per (charge, x offset): 1, or 2 when a
                   // charge's 2p rows can straddle two chunks
  int ik;          // forces: 0 window gradient, 1 ik-differentiation (eq. 24-25)
  int stage;       // charges of a plane staged in LDS at a time (<= kStage)
  int parts;       // work-groups per plane in the spread and gather passes, each
                   // taking a contiguous share of the plane's charges (<= kMaxParts)
  int bparts;      // work-groups per plane in the backward (gather) pass, each taking
                   // the charges j with j mod bparts equal to its index (<= kMaxParts)
  int xsplit;      // work-groups per ky row in the x pass, each a contiguous range of kz
  double gscale_f; // fixed-point scale of the partial spectra, relative to the
                   // spread's scale: 2^-(3 ceil(log2 2p) + 3)
  double L;
  double m_over_l; // M / L: mesh coordinate t = x * m_over_l
  WindowParams win;
  FftPlan fft;
};

// Byte offset of the field spectrum h within the gzy buffer (after the
// fixed-point partial spectra of the plane parts).
__host__ __device__ inline size_t spectrum_h_offset(const MeshParams &m) {
  return (size_t)m.parts * m.M * m.nky * m.Kc * 16;
}

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
  DevScalars *sc;
  double4 *xq;           // [N] compacted (x, y, z, q), wrapped into [0, L)
  int *idx;              // [N] particle index of compact slot j
  int *slot;             // [N] compact slot of particle i, or -1
  // real-space cell grid
  int *ccnt;             // [2 ncell^3] two sets: a DPD step bins into one while the other is cleared
  double4 *cgrid;        // [ncell^3 * cap] (x, y, z, q) per cell slot
  float4 *cpre;          // [ncell^3 * cap] FP32 (x, y, z) and the compact index (bits in w) per cell
                         // slot: what the real-space scan's pre-test reads
  unsigned long long *freal;  // [N * 3] fixed-point real-space force per compact slot
  unsigned long long *ereal; // [2 N] fixed-point (E_real whole, E_slater) of the pairs (j, k > j), per compact slot j
  long long *blk_er;         // [2 nblk] per-block sums of ereal over the particles of the block
  // reciprocal
  void *gzy;             // [(parts + 1) * M * nky * Kc] 16-byte entries: the partial spectra
                         // G[part][x][ky][kz] as fixed-point int64 pairs, then the field
                         // spectrum h[x][ky][kz] as complex T (double2 or float2)
  void *gzx;             // [M * nky * Kc] complex: i kx h for the ik forces
  double *epart;         // [nky * Kc] k-space energy per (ky, kz) line
  double4 *part;         // [N * 2p * nslot] gather partials (dwx A, wx By, wx Bz, wx A)
  int *xcnt;             // [2 M kXSub] charges per mesh x-cell sub-bin (zero between calls; two sets like ccnt)
  int *xslot;            // [M kXSub xcap] compact indices of the charges of each x-cell sub-bin
  double *wcoef64;       // [2p (D+1) + 2p D] window series coefficients (value, then derivative)
  float *wcoef32;
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

// What the closing kernel does besides the electrostatic force.
struct FinishArgs {
  int mode = -1;                     // -1: plain ENUF evaluation (forces = F_elec)
                                     //  0: DPD step: F = F_pair + kappa F_elec, v += dt F / 2
                                     //  1: DPD forces only: F = F_pair + kappa F_elec
  double kappa = 0.0, dt = 0.0;
  const double *fdpd = nullptr;      // DPD pair + bond forces
  double *vel = nullptr;
  int *dcnt = nullptr;               // DPD cell counts, cleared for the next step
  int ndcell3 = 0;
  int energies = 1;                  // 0: skip the energy reduction (a step whose energies no one reads)
  unsigned long long *step_inc = nullptr;  // device step index, advanced by one (steps replayed from a graph)
};

// Scale of the gathered mesh field in the combine kernel: 2 / L^2 for ik
// forces, M / (pi L^2) for the window-gradient forces.
inline double combine_fscale(const ComputeConfig &cfg) {
  const double L = cfg.L;
  return cfg.mesh.ik ? 2.0 / (L * L) : (double)cfg.mesh.M / (3.14159265358979323846 * L * L);
}

// The ENUF evaluation in four phases (launch_compute runs them in order on
// one stream; the DPD step forks the real-space phase onto another stream).
hipError_t launch_prep(const ComputeConfig &cfg, const ComputeBuffers &b, const double *pos,
                       const double *q, hipStream_t st, KernelTimer *tm);
hipError_t launch_real(const ComputeConfig &cfg, const ComputeBuffers &b, int64_t nq_max, hipStream_t st,
                       KernelTimer *tm);
// x_threads: work-group size of the x pass (at least fft_max_butterflies of
// the mesh, at most kPassThreads; others are raised or clamped to fit).
hipError_t launch_recip(const ComputeConfig &cfg, const ComputeBuffers &b, int64_t nq_max, hipStream_t st,
                        KernelTimer *tm, int x_threads = kPassThreads);
hipError_t launch_combine(const ComputeConfig &cfg, const ComputeBuffers &b, double *forces,
                          double *energy_total, double *energy5, const FinishArgs &fa, hipStream_t st,
                          KernelTimer *tm);

hipError_t launch_compute(const ComputeConfig &cfg, const ComputeBuffers &b,
                          const double *pos, const double *q, double *forces,
                          double *energy_total, double *energy5, hipStream_t stream,
                          KernelTimer *timer = nullptr);

// Host-computed tables of a plan: influence factors per wave number
// (exp(-pi^2 k^2/(alpha L)^2) / Phi(k/M)^2), FFT twiddles, and the window
// series of the given precision (cheb_deg its degree).
struct PlanTables {
  std::vector<double> atab;
  std::vector<double2> tw64;
  std::vector<float2> tw32;
  std::vector<double> wcoef64;  // filled for ENUF_FP64
  std::vector<float> wcoef32;   // filled for ENUF_MIXED
  int cheb_deg = 0;
};
int plan_tables(const ComputeConfig &c, int precision, PlanTables *t);

// LDS bytes the three mesh passes need for the given geometry, precision and
// m.rows.
void mesh_lds_bytes(const MeshParams &m, int precision, size_t *fwd, size_t *x, size_t *bwd);

// Choose m.rows / m.nchunk / m.nslot: the fewest row chunks whose passes fit
// in max_lds bytes.  Returns false when no chunking fits.
bool mesh_choose_rows(MeshParams &m, int precision, size_t max_lds);

// Raise the per-kernel dynamic LDS limit where needed (once per process).
hipError_t configure_kernels(size_t max_lds);

// Structure observables (enuf_observables.hip).  Pair-distance histogram by
// class: at most kHistMaxBins = classes^2 x bins counters (LDS-resident).
constexpr int kHistMaxBins = 12288;
constexpr int64_t kHistMaxSel = (int64_t)65535 * 256;
hipError_t launch_pair_histogram(const double *pos, int64_t n, int64_t nsel, const int64_t *sel, const int *cls,
                                 int ncls, double box, double r_max, int nbins, unsigned long long *hist,
                                 hipStream_t st);
hipError_t launch_chain_rg2(const double *pos, int64_t n, int nchains, int len, const int64_t *beads, double box,
                            double *out, hipStream_t st);

}  // namespace enuf
