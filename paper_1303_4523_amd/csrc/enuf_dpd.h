// enuf_dpd.h -- internal definitions of the DPD step (not part of the ABI).
#pragma once

#include "enuf_internal.h"

namespace enuf {

struct DpdParams {
  double L;
  double a, gamma, sigma, dt, lam;  // DPD amplitudes, time step, VV prediction parameter
  double k_bond, r0_bond;
  double kappa;                     // electrostatic coupling
  uint64_t seed;
  int ncell;                        // DPD cells per side (edge >= R_c = 1)
  int cap;                          // slots per cell
  double inv_cell;
  int seg_cells, nseg;              // pair kernel: cells per column segment, segments per column
  int pair_stage;                   // particles the pair kernel stages in LDS per segment
  int nspec;                        // > 1: the conservative amplitude depends on the pair's species
  const int *species;               // [N] species of each particle (device; read when nspec > 1)
  double atab[16];                  // a_ij = atab[4 s_i + s_j], symmetric (nspec <= 4)
};

// Charges of a DPD system are fixed, so their compaction into an ENUF plan is
// computed once; the pre kernel then writes the compacted, wrapped charges,
// bins them into the plan's real-space cell grid and sets the plan scalars.
struct DpdCharges {
  int enabled = 0;
  const int *dslot = nullptr;   // [N] compact slot of particle i or -1 (static)
  const double *q = nullptr;    // [N]
  double4 *xq = nullptr;        // plan: compacted charges
  int *slot = nullptr;          // plan: slot map read by the combine kernel
  int *ccnt = nullptr;          // plan: charge cell grid
  double4 *cgrid = nullptr;
  float4 *cpre = nullptr;
  CellParams cells{};
  int *xcnt = nullptr;          // plan: charges binned by mesh x-cell
  int *xslot = nullptr;
  int M = 0, xcap = 0;
  double m_over_l = 0.0;
  DevScalars *sc = nullptr;     // plan scalars, rewritten every step
  DevScalars stat{};            // nq, sums and fixed-point scale of the fixed charges
};

// One member system of a batched DPD step (one launch per stage for all
// members): the geometry and scratch of its ENUF plan, its integrator state
// and its device step counter.  Kept in device memory; every block of a
// batched launch reads the member its work-map entry names.
struct BatchMember {
  ComputeConfig cfg;
  ComputeBuffers buf;
  int nq;                       // charged particles (static compaction)
  int nblk;                     // blocks of 256 particles (pre, combine)
  int pair_blocks;              // blocks of the pair kernel
  int real_blocks;              // blocks of the real-space kernel (one wave per charge)
  double fscale, inv2piL;       // M / (pi L^2), 1 / (2 pi L)
  int64_t N;
  DpdParams P;
  double *pos, *vel, *force;    // caller-owned state
  double *fdpd, *e5;
  int *dcnt;
  double4 *cpos, *cvel;
  const int *bond_start, *bond_to;
  int *status;
  DpdCharges ch;
  unsigned long long *step;     // index of the member's next step
  // the other set of bin counts: a fused combine + pre step clears this
  // table's set (buf, dcnt) while it bins the next step into these
  int *dcnt_next;
  DpdCharges ch_next;
};

// Batched launches: map[b] = (member, block of that member) for block b.
hipError_t launch_batch_pre(const BatchMember *mem, const int2 *map, int nmap, int mode, hipStream_t st);
// Step k's combine (mode 0, no energy partials, the step index advanced) and
// step k + 1's pre kernel in one launch, over the combine map (blocks of
// 256 particles).
hipError_t launch_batch_combine_pre(const BatchMember *mem, const int2 *map, int nmap, hipStream_t st);
// steps: candidate steps in flight per lane (4 or 8, else hipErrorInvalidValue).
hipError_t launch_batch_pair(const BatchMember *mem, const int2 *map, int nmap, int steps, hipStream_t st);
// Column segments of the pair kernel for a grid of n cells per side, about
// target cells each (1 .. kPairSegMax).
void pair_segments(int n, int target, int *seg_cells, int *nseg);
constexpr int kPairSeg = 10;      // cells per column segment, about: one system
constexpr int kBatchPairSeg = 26; // batches (default of enuf_batch_set_tuning)
constexpr int kPairSegMax = 26;   // longest segment the kernel's tables allow
// Dynamic LDS bytes of the pair kernel (its staged particles; vlds: with their
// velocities, as one system stages them).
size_t pair_lds_bytes(const DpdParams &P, bool vlds);
constexpr int kPairStage = 384;   // particles staged per segment, one system (30 KB of LDS with velocities)
constexpr int kBatchPairStage = 600;  // batches (28 KB without velocities)
constexpr int kPairStageMax = 1024;  // largest stage the kernel's tables allow
constexpr int kPairOwn = 128;     // own particles of a chunk (LDS force accumulators); cell capacity limit
// Allow the pair kernels the dynamic LDS of their staged particles.
hipError_t configure_pair_kernels(size_t lds_bytes);
// Blocks of the pair kernel (one per column segment), a multiple of 8 (whole
// rounds over the XCDs).
int pair_blocks(const DpdParams &P);
hipError_t launch_batch_real(const BatchMember *mem, const int2 *map, int nmap, hipStream_t st);
// pass_threads, x_threads: work-group sizes of the spread/gather passes and of
// the x pass (at least fft_max_butterflies of every member).
hipError_t launch_batch_recip(const BatchMember *mem, int precision, int ik, const int2 *fwd, int nfwd,
                              const int2 *x, int nx, const int2 *bwd, int nbwd, size_t lds_fwd, size_t lds_x,
                              size_t lds_bwd, int pass_threads, int x_threads, hipStream_t st,
                              KernelTimer *tm = nullptr);
// Combine for every member, then the final energies (one block per member).
hipError_t launch_batch_combine(const BatchMember *mem, int nmem, const int2 *map, int nmap, int mode,
                                hipStream_t st);
hipError_t launch_set_u64(unsigned long long *dst, unsigned long long value, hipStream_t st);
hipError_t launch_add_u64(unsigned long long *dst, hipStream_t st);  // *dst += 1

// The predicted velocity v0 = v + lam dt F is kept only in the cell slots
// (the pair kernel reads it there).
hipError_t launch_dpd_pre(int64_t N, int mode, const DpdParams &P, double *pos, double *vel,
                          const double *force, int *dcnt, double4 *cpos, double4 *cvel, int *status,
                          const DpdCharges &ch, hipStream_t st, KernelTimer *tm = nullptr);
hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos, const int *dcnt,
                           const double4 *cpos, const double4 *cvel, const int *bond_start, const int *bond_to,
                           double *fdpd, hipStream_t st, KernelTimer *tm = nullptr,
                           const unsigned long long *step_dev = nullptr);
// The combine kernel of a DPD step fused with the next step's pre kernel
// (no energy reduction: fa.energies must be 0, else hipErrorInvalidValue).
hipError_t launch_combine_pre(const ComputeConfig &cfg, const ComputeBuffers &b, double *forces,
                              const FinishArgs &fa, const DpdParams &P, double *pos, int *dcnt, double4 *cpos,
                              double4 *cvel, int *status, const DpdCharges &ch, hipStream_t st,
                              KernelTimer *tm = nullptr);
hipError_t launch_dpd_post(int64_t N, int mode, const DpdParams &P, const double *fdpd,
                           const double *felec, double *force, double *vel, int *dcnt, hipStream_t st,
                           KernelTimer *tm = nullptr);

}  // namespace enuf
