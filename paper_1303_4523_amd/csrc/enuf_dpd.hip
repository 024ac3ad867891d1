// enuf_dpd.hip -- HIP kernels (gfx950) of one DPD step with ENUF electrostatics
// (modified velocity Verlet of Table 2):
//   k_dpd_pre    (0) v0 = v + lam dt F, (1) v += dt F / 2, (2) r += dt v (wrapped);
//                bin particles into the DPD cell grid (cell edge >= R_c = 1)
//   k_dpd_pair   (3) conservative, dissipative and random pair forces (eq. 2-7)
//                with theta_ij from Philox4x64-10, plus harmonic bonds
//   [enuf_compute (4): electrostatic forces and energy]
//   k_dpd_post   (5) F = F_dpd + kappa F_elec, (6) v += dt F / 2; clear the grid
#include "enuf_device.h"
#include "enuf_dpd.h"

namespace enuf {

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl constants between rounds.
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// theta_ij: uniform on [-sqrt 3, sqrt 3) (zero mean, unit variance), keyed by
// the unordered pair, the step and the seed; 53 bits of the first word.
__device__ inline double dpd_theta(uint64_t seed, uint64_t step, int i, int j) {
  uint64_t c[4] = {(uint64_t)(i < j ? i : j), (uint64_t)(i < j ? j : i), step, 0ull};
  philox4x64_10(c, seed, 0ull);
  const double u = (double)(c[0] >> 11) * (1.0 / 9007199254740992.0);
  return 1.7320508075688772935 * (2.0 * u - 1.0);
}

__device__ inline double wrap_box(double x, double L) {
  double y = x - L * floor(x / L);
  if (!(y < L) || y < 0.0) y = 0.0;
  return y;
}

__device__ inline int dpd_cell_of(double x, double inv_cell, int n) {
  int c = (int)(x * inv_cell);
  return c < n ? (c < 0 ? 0 : c) : n - 1;
}

// mode 0: full predictor / half kick / drift; mode 1: forces only (v0 = v).
__global__ void __launch_bounds__(256)
k_dpd_pre(int64_t N, int mode, DpdParams P, double *__restrict__ pos, double *__restrict__ vel,
          const double *__restrict__ force, double *__restrict__ v0, int *dcnt, int *dgrid,
          int *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double r[3], v[3], f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = pos[3 * i + a];
    v[a] = vel[3 * i + a];
    f[a] = force[3 * i + a];
  }
  if (mode == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v0[3 * i + a] = v[a] + P.lam * P.dt * f[a];
      v[a] += 0.5 * P.dt * f[a];
      r[a] = wrap_box(r[a] + P.dt * v[a], P.L);
      vel[3 * i + a] = v[a];
      pos[3 * i + a] = r[a];
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v0[3 * i + a] = v[a];
      r[a] = wrap_box(r[a], P.L);
      pos[3 * i + a] = r[a];
    }
  }
  const int n = P.ncell;
  const int cell = (dpd_cell_of(r[0], P.inv_cell, n) * n + dpd_cell_of(r[1], P.inv_cell, n)) * n +
                   dpd_cell_of(r[2], P.inv_cell, n);
  const int s = atomicAdd(&dcnt[cell], 1);
  if (s < P.cap)
    dgrid[(size_t)cell * P.cap + s] = (int)i;
  else
    atomicCAS(status, 0, kEOverflow);
}

__device__ inline bool dpd_offset_valid(int o, int n) {
  return n >= 3 || (n == 2 && o >= 0) || (n == 1 && o == 0);
}

// One thread per particle; every pair is evaluated from both sides (the
// random number is symmetric in i, j).  Sums are exact int64 fixed point so
// that the visiting order inside a cell does not change the result.
__global__ void __launch_bounds__(256)
k_dpd_pair(int64_t N, DpdParams P, uint64_t step, const double *__restrict__ pos,
           const double *__restrict__ v0, const int *__restrict__ dcnt, const int *__restrict__ dgrid,
           const int *__restrict__ bond_start, const int *__restrict__ bond_to,
           double *__restrict__ fdpd) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= N) return;
  const int i = (int)i64;
  const double L = P.L, invL = 1.0 / L, isdt = 1.0 / sqrt(P.dt);
  const double rx = pos[3 * i], ry = pos[3 * i + 1], rz = pos[3 * i + 2];
  const double vx = v0[3 * i], vy = v0[3 * i + 1], vz = v0[3 * i + 2];
  const int n = P.ncell;
  const int cx = dpd_cell_of(rx, P.inv_cell, n), cy = dpd_cell_of(ry, P.inv_cell, n),
            cz = dpd_cell_of(rz, P.inv_cell, n);
  long long fx = 0, fy = 0, fz = 0;
  for (int o = 0; o < 27; ++o) {
    const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
    if (!(dpd_offset_valid(ox, n) && dpd_offset_valid(oy, n) && dpd_offset_valid(oz, n))) continue;
    const int c = (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + mod_pos(cz + oz, n);
    int cnt = dcnt[c];
    cnt = cnt < P.cap ? cnt : P.cap;
    for (int s = 0; s < cnt; ++s) {
      const int j = dgrid[(size_t)c * P.cap + s];
      if (j == i) continue;
      double dx = rx - pos[3 * j], dy = ry - pos[3 * j + 1], dz = rz - pos[3 * j + 2];
      dx -= L * rint(dx * invL);
      dy -= L * rint(dy * invL);
      dz -= L * rint(dz * invL);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < 1.0) || r2 == 0.0) continue;
      const double r = sqrt(r2), ir = 1.0 / r;
      const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
      const double wr = 1.0 - r;
      const double vdot = (vx - v0[3 * j]) * ex + (vy - v0[3 * j + 1]) * ey + (vz - v0[3 * j + 2]) * ez;
      const double th = dpd_theta(P.seed, step, i, j);
      const double mag = P.a * wr - P.gamma * wr * wr * vdot + P.sigma * wr * th * isdt;
      fx += to_fixed(mag * ex, kRealFxScale);
      fy += to_fixed(mag * ey, kRealFxScale);
      fz += to_fixed(mag * ez, kRealFxScale);
    }
  }
  double gx = (double)fx * kRealFxInv, gy = (double)fy * kRealFxInv, gz = (double)fz * kRealFxInv;
  // harmonic bonds, F_i = -K (r - r0) rhat_ij, in the order the bonds were given
  for (int b = bond_start[i]; b < bond_start[i + 1]; ++b) {
    const int j = bond_to[b];
    double dx = rx - pos[3 * j], dy = ry - pos[3 * j + 1], dz = rz - pos[3 * j + 2];
    dx -= L * rint(dx * invL);
    dy -= L * rint(dy * invL);
    dz -= L * rint(dz * invL);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r == 0.0) continue;
    const double mag = -P.k_bond * (r - P.r0_bond) / r;
    gx += mag * dx;
    gy += mag * dy;
    gz += mag * dz;
  }
  fdpd[3 * i] = gx;
  fdpd[3 * i + 1] = gy;
  fdpd[3 * i + 2] = gz;
}

// mode 0: F = F_dpd + kappa F_elec and the closing half kick; mode 1: forces only.
__global__ void __launch_bounds__(256)
k_dpd_post(int64_t N, int mode, DpdParams P, const double *__restrict__ fdpd,
           const double *__restrict__ felec, double *__restrict__ force, double *__restrict__ vel,
           int *dcnt, int ncell3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = i; c < ncell3; c += stride) dcnt[c] = 0;
  if (i >= N) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f = fdpd[3 * i + a];
    if (felec) f += P.kappa * felec[3 * i + a];
    force[3 * i + a] = f;
    if (mode == 0) vel[3 * i + a] += 0.5 * P.dt * f;
  }
}

hipError_t launch_dpd_pre(int64_t N, int mode, const DpdParams &P, double *pos, double *vel,
                          const double *force, double *v0, int *dcnt, int *dgrid, int *status,
                          hipStream_t st, KernelTimer *tm) {
  const int nb = (int)((N + 255) / 256);
  if (tm) tm->before(0, st);
  hipLaunchKernelGGL(k_dpd_pre, dim3(nb), dim3(256), 0, st, N, mode, P, pos, vel, force, v0, dcnt, dgrid,
                     status);
  if (tm) tm->after(0, st);
  return hipGetLastError();
}

hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos,
                           const double *v0, const int *dcnt, const int *dgrid, const int *bond_start,
                           const int *bond_to, double *fdpd, hipStream_t st, KernelTimer *tm) {
  const int nb = (int)((N + 255) / 256);
  if (tm) tm->before(1, st);
  hipLaunchKernelGGL(k_dpd_pair, dim3(nb), dim3(256), 0, st, N, P, step, pos, v0, dcnt, dgrid, bond_start,
                     bond_to, fdpd);
  if (tm) tm->after(1, st);
  return hipGetLastError();
}

hipError_t launch_dpd_post(int64_t N, int mode, const DpdParams &P, const double *fdpd,
                           const double *felec, double *force, double *vel, int *dcnt, hipStream_t st,
                           KernelTimer *tm) {
  const int nb = (int)((N + 255) / 256);
  const int ncell3 = P.ncell * P.ncell * P.ncell;
  if (tm) tm->before(9, st);
  hipLaunchKernelGGL(k_dpd_post, dim3(nb), dim3(256), 0, st, N, mode, P, fdpd, felec, force, vel, dcnt,
                     ncell3);
  if (tm) tm->after(9, st);
  return hipGetLastError();
}

}  // namespace enuf
