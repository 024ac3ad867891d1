// enuf_dpd.hip -- HIP kernels (gfx950) of one DPD step with ENUF electrostatics
// (modified velocity Verlet of Table 2):
//   k_dpd_pre    (0) v0 = v + lam dt F, (1) v += dt F / 2, (2) r += dt v (wrapped);
//                bin particles into the DPD cell grid (cell edge >= R_c = 1)
//   k_dpd_pair   (3) conservative, dissipative and random pair forces (eq. 2-7)
//                with theta_ij from Philox4x32-10, plus harmonic bonds
//   [enuf_compute (4): electrostatic forces and energy]
//   k_dpd_post   (5) F = F_dpd + kappa F_elec, (6) v += dt F / 2; clear the grid
#include "enuf_device.h"
#include "enuf_dpd.h"

namespace enuf {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
    const uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// theta_ij: uniform on [-sqrt 3, sqrt 3) (zero mean, unit variance), keyed by
// the unordered pair, the step and the seed; 53 bits of the first two words.
__device__ inline double dpd_theta(uint64_t seed, uint64_t step, int i, int j) {
  uint32_t c[4] = {(uint32_t)(i < j ? i : j), (uint32_t)(i < j ? j : i), (uint32_t)step,
                   (uint32_t)(step >> 32)};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t bits = ((uint64_t)c[0] << 21) | (uint64_t)(c[1] >> 11);
  const double u = (double)bits * (1.0 / 9007199254740992.0);
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
// Each particle is binned into a slot of its DPD cell together with its
// position (and index) and predicted velocity, so that the pair kernel reads
// neighbour data contiguously.
__global__ void __launch_bounds__(256)
k_dpd_pre(int64_t N, int mode, DpdParams P, double *__restrict__ pos, double *__restrict__ vel,
          const double *__restrict__ force, double *__restrict__ v0, int *dcnt, double4 *cpos,
          double4 *cvel, int *status, DpdCharges ch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ch.enabled && i == 0) {
    ch.sc->nq = ch.stat.nq;
    ch.sc->scale = ch.stat.scale;
    ch.sc->inv_scale = ch.stat.inv_scale;
    ch.sc->sum_q = ch.stat.sum_q;
    ch.sc->sum_absq = ch.stat.sum_absq;
    ch.sc->sum_q2 = ch.stat.sum_q2;
    ch.eacc[0] = 0ull;
    ch.eacc[1] = 0ull;
  }
  if (i >= N) return;
  double r[3], v[3], f[3], w[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = pos[3 * i + a];
    v[a] = vel[3 * i + a];
    f[a] = force[3 * i + a];
  }
  if (mode == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      w[a] = v[a] + P.lam * P.dt * f[a];
      v[a] += 0.5 * P.dt * f[a];
      r[a] = wrap_box(r[a] + P.dt * v[a], P.L);
      vel[3 * i + a] = v[a];
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      w[a] = v[a];
      r[a] = wrap_box(r[a], P.L);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    pos[3 * i + a] = r[a];
    v0[3 * i + a] = w[a];
  }
  const int n = P.ncell;
  const int cell = (dpd_cell_of(r[0], P.inv_cell, n) * n + dpd_cell_of(r[1], P.inv_cell, n)) * n +
                   dpd_cell_of(r[2], P.inv_cell, n);
  const int s = atomicAdd(&dcnt[cell], 1);
  if (s < P.cap) {
    cpos[(size_t)cell * P.cap + s] = make_double4(r[0], r[1], r[2], (double)i);
    cvel[(size_t)cell * P.cap + s] = make_double4(w[0], w[1], w[2], 0.0);
  } else {
    atomicCAS(status, 0, kEOverflow);
  }
  if (ch.enabled) {
    const int j = ch.dslot[i];
    ch.slot[i] = j;
    if (j >= 0) {
      const double qi = ch.q[i];
      ch.xq[j] = make_double4(r[0], r[1], r[2], qi);
      const CellParams &cp = ch.cells;
      int cx = (int)(r[0] * cp.inv_cell), cy = (int)(r[1] * cp.inv_cell), cz = (int)(r[2] * cp.inv_cell);
      cx = cx < cp.ncell ? cx : cp.ncell - 1;
      cy = cy < cp.ncell ? cy : cp.ncell - 1;
      cz = cz < cp.ncell ? cz : cp.ncell - 1;
      const int c = (cx * cp.ncell + cy) * cp.ncell + cz;
      const int sl = atomicAdd(&ch.ccnt[c], 1);
      if (sl < cp.cap) {
        ch.cgrid[(size_t)c * cp.cap + sl] = make_double4(r[0], r[1], r[2], qi);
        ch.cidx[(size_t)c * cp.cap + sl] = j;
      } else {
        atomicCAS(&ch.sc->status, 0, kEOverflow);
      }
      double t;
      const int xc = mesh_cell(r[0], ch.m_over_l, ch.M, &t);
      const int xs = atomicAdd(&ch.xcnt[xc], 1);
      if (xs < ch.xcap)
        ch.xslot[(size_t)xc * ch.xcap + xs] = j;
      else
        atomicCAS(&ch.sc->status, 0, kEOverflow);
    }
  }
}

__device__ inline bool dpd_offset_valid(int o, int n) {
  return n >= 3 || (n == 2 && o >= 0) || (n == 1 && o == 0);
}

// Four lanes per particle i split the 27 neighbour cells; every pair is
// evaluated from both of its particles (theta_ij = theta_ji keeps the pair
// forces antisymmetric), so no thread writes another particle's force.  Sums
// are exact int64 fixed point (2^-36): the result does not depend on the order
// in which the pairs are visited.
__global__ void __launch_bounds__(256)
k_dpd_pair(int64_t N, DpdParams P, uint64_t step, const double *__restrict__ pos,
           const double *__restrict__ v0, const int *__restrict__ dcnt,
           const double4 *__restrict__ cpos, const double4 *__restrict__ cvel,
           const int *__restrict__ bond_start, const int *__restrict__ bond_to,
           double *__restrict__ fdpd) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i64 = g >> 2;
  const int quad = (int)(g & 3);
  if (i64 >= N) return;  // whole quads leave together
  const int i = (int)i64;
  const double L = P.L, invL = 1.0 / L, isdt = 1.0 / sqrt(P.dt);
  const double rx = pos[3 * i], ry = pos[3 * i + 1], rz = pos[3 * i + 2];
  const double vx = v0[3 * i], vy = v0[3 * i + 1], vz = v0[3 * i + 2];
  const int n = P.ncell;
  const int cx = dpd_cell_of(rx, P.inv_cell, n), cy = dpd_cell_of(ry, P.inv_cell, n),
            cz = dpd_cell_of(rz, P.inv_cell, n);
  long long fx = 0, fy = 0, fz = 0;
  for (int o = quad; o < 27; o += 4) {
    const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
    if (!(dpd_offset_valid(ox, n) && dpd_offset_valid(oy, n) && dpd_offset_valid(oz, n))) continue;
    const int c = (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + mod_pos(cz + oz, n);
    int cnt = dcnt[c];
    cnt = cnt < P.cap ? cnt : P.cap;
    const double4 *cp = cpos + (size_t)c * P.cap;
    for (int s = 0; s < cnt; ++s) {
      const double4 e = cp[s];
      const int j = (int)e.w;
      if (j == i) continue;
      double dx = rx - e.x, dy = ry - e.y, dz = rz - e.z;
      dx -= L * rint(dx * invL);
      dy -= L * rint(dy * invL);
      dz -= L * rint(dz * invL);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < 1.0) || r2 == 0.0) continue;
      const double4 vj = cvel[(size_t)c * P.cap + s];
      const double r = sqrt(r2), ir = 1.0 / r;
      const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
      const double wr = 1.0 - r;
      const double vdot = (vx - vj.x) * ex + (vy - vj.y) * ey + (vz - vj.z) * ez;
      const double th = dpd_theta(P.seed, step, i, j);
      const double mag = P.a * wr - P.gamma * wr * wr * vdot + P.sigma * wr * th * isdt;
      fx += to_fixed(mag * ex, kRealFxScale);
      fy += to_fixed(mag * ey, kRealFxScale);
      fz += to_fixed(mag * ez, kRealFxScale);
    }
  }
  // harmonic bonds of i, F_i = -K (r - r0) rhat_ij
  if (quad == 0) {
    for (int b = bond_start[i]; b < bond_start[i + 1]; ++b) {
      const int j = bond_to[b];
      double dx = rx - pos[3 * j], dy = ry - pos[3 * j + 1], dz = rz - pos[3 * j + 2];
      dx -= L * rint(dx * invL);
      dy -= L * rint(dy * invL);
      dz -= L * rint(dz * invL);
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r == 0.0) continue;
      const double mag = -P.k_bond * (r - P.r0_bond) / r;
      fx += to_fixed(mag * dx, kRealFxScale);
      fy += to_fixed(mag * dy, kRealFxScale);
      fz += to_fixed(mag * dz, kRealFxScale);
    }
  }
  fx += __shfl_xor(fx, 1, kWave);
  fy += __shfl_xor(fy, 1, kWave);
  fz += __shfl_xor(fz, 1, kWave);
  fx += __shfl_xor(fx, 2, kWave);
  fy += __shfl_xor(fy, 2, kWave);
  fz += __shfl_xor(fz, 2, kWave);
  if (quad == 0) {
    fdpd[3 * i] = (double)fx * kRealFxInv;
    fdpd[3 * i + 1] = (double)fy * kRealFxInv;
    fdpd[3 * i + 2] = (double)fz * kRealFxInv;
  }
}

// mode 0: F = F_dpd + kappa F_elec and the closing half kick; mode 1: forces
// only.  Clears the cell counts for the next step.
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
                          const double *force, double *v0, int *dcnt, double4 *cpos, double4 *cvel,
                          int *status, const DpdCharges &ch, hipStream_t st, KernelTimer *tm) {
  const int nb = (int)((N + 255) / 256);
  if (tm) tm->before(0, st);
  hipLaunchKernelGGL(k_dpd_pre, dim3(nb), dim3(256), 0, st, N, mode, P, pos, vel, force, v0, dcnt, cpos,
                     cvel, status, ch);
  if (tm) tm->after(0, st);
  return hipGetLastError();
}

hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos,
                           const double *v0, const int *dcnt, const double4 *cpos, const double4 *cvel,
                           const int *bond_start, const int *bond_to, double *fdpd,
                           hipStream_t st, KernelTimer *tm) {
  const int nb = (int)((4 * N + 255) / 256);
  if (tm) tm->before(1, st);
  hipLaunchKernelGGL(k_dpd_pair, dim3(nb), dim3(256), 0, st, N, P, step, pos, v0, dcnt, cpos, cvel,
                     bond_start, bond_to, fdpd);
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
