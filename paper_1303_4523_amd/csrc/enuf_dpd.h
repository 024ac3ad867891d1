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
  int *cidx = nullptr;
  CellParams cells{};
  int *xcnt = nullptr;          // plan: charges binned by mesh x-cell
  int *xslot = nullptr;
  int M = 0, xcap = 0;
  double m_over_l = 0.0;
  DevScalars *sc = nullptr;     // plan scalars, rewritten every step
  unsigned long long *eacc = nullptr;  // plan: real-space energy accumulators (cleared)
  DevScalars stat{};            // nq, sums and fixed-point scale of the fixed charges
};

hipError_t launch_dpd_pre(int64_t N, int mode, const DpdParams &P, double *pos, double *vel,
                          const double *force, double *v0, int *dcnt, double4 *cpos, double4 *cvel,
                          int *status, const DpdCharges &ch, hipStream_t st, KernelTimer *tm = nullptr);
hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos,
                           const double *v0, const int *dcnt, const double4 *cpos, const double4 *cvel,
                           const int *bond_start, const int *bond_to, double *fdpd,
                           hipStream_t st, KernelTimer *tm = nullptr);
hipError_t launch_dpd_post(int64_t N, int mode, const DpdParams &P, const double *fdpd,
                           const double *felec, double *force, double *vel, int *dcnt, hipStream_t st,
                           KernelTimer *tm = nullptr);

}  // namespace enuf
