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

hipError_t launch_dpd_pre(int64_t N, int mode, const DpdParams &P, double *pos, double *vel,
                          const double *force, double *v0, int *dcnt, double4 *cpos, double4 *cvel,
                          int *status, hipStream_t st, KernelTimer *tm = nullptr);
hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos,
                           const double *v0, const int *dcnt, const double4 *cpos, const double4 *cvel,
                           const int *bond_start, const int *bond_to, unsigned long long *facc,
                           hipStream_t st, KernelTimer *tm = nullptr);
hipError_t launch_dpd_post(int64_t N, int mode, const DpdParams &P, unsigned long long *facc,
                           const double *felec, double *force, double *vel, int *dcnt, hipStream_t st,
                           KernelTimer *tm = nullptr);

}  // namespace enuf
