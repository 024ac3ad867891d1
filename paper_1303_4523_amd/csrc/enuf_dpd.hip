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
__device__ __forceinline__ void
dpd_pre_body(int64_t N, int mode, const DpdParams &P, double *__restrict__ pos, double *__restrict__ vel,
             const double *__restrict__ force, double *__restrict__ v0, int *dcnt, double4 *cpos,
             double4 *cvel, int *status, const DpdCharges &ch, int bid) {
  const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
  if (ch.enabled && i == 0) {
    ch.sc->nq = ch.stat.nq;
    ch.sc->scale = ch.stat.scale;
    ch.sc->inv_scale = ch.stat.inv_scale;
    ch.sc->sum_q = ch.stat.sum_q;
    ch.sc->sum_absq = ch.stat.sum_absq;
    ch.sc->sum_q2 = ch.stat.sum_q2;
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
    const double sp = P.nspec > 1 ? (double)P.species[i] : 0.0;
    cvel[(size_t)cell * P.cap + s] = make_double4(w[0], w[1], w[2], sp);
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

__global__ void __launch_bounds__(256)
k_dpd_pre(int64_t N, int mode, DpdParams P, double *__restrict__ pos, double *__restrict__ vel,
          const double *__restrict__ force, double *__restrict__ v0, int *dcnt, double4 *cpos,
          double4 *cvel, int *status, DpdCharges ch) {
  dpd_pre_body(N, mode, P, pos, vel, force, v0, dcnt, cpos, cvel, status, ch, blockIdx.x);
}

__device__ inline bool dpd_offset_valid(int o, int n) {
  return n >= 3 || (n == 2 && o >= 0) || (n == 1 && o == 0);
}

// Pair forces in cell order.  A wavefront takes a group of consecutive DPD
// cells (z fastest) and their particles, 64/Q at a time with Q = 4 or 8 lanes
// per particle; the particles of one wavefront are neighbours, so they read
// the same neighbour cells.  Blocks are mapped so that each of the 8 XCDs
// (which take the blocks of a launch round-robin) works on one contiguous
// slab of cells, keeping its L2 working set to that slab and its halo.
// Scan: each lane walks the slots of its share of the 27 neighbour cells and
// the pairs with r < R_c = 1 are appended to a wavefront queue in LDS.
// Evaluation: the whole wavefront takes the queued pairs 64 at a time (so the
// Philox draw and the pair force run with full lanes however sparse the
// neighbours are) and adds each pair force to i's int64 fixed-point
// accumulator in LDS.  Every pair is evaluated from both of its particles
// (theta_ij = theta_ji keeps the pair forces antisymmetric), so no thread
// writes another particle's force; the fixed-point sums (2^-36) are exact, so
// the result does not depend on the order in which pairs are visited.  With
// species, the cell slot's predicted velocity carries the species in w and
// the amplitude a_ij is read from the symmetric table in the parameters.
// Particles beyond a full cell's capacity (reported as ENUF_EOVERFLOW by the
// binning) get no force.
constexpr int kPairThreads = 256;
constexpr int kPairQueue = 128;  // queued pairs per wavefront (flushed at > 64)
constexpr int kXcds = 8;         // MI355X: blocks of a launch are dealt round-robin to 8 XCDs

template <int Q>
__device__ __forceinline__ void
dpd_pair_body(const DpdParams &P, uint64_t step, gptr<const double> __restrict__ pos,
              gptr<const int> __restrict__ dcnt, gptr<const double4> __restrict__ cpos,
              gptr<const double4> __restrict__ cvel, gptr<const int> __restrict__ bond_start,
              gptr<const int> __restrict__ bond_to, gptr<double> __restrict__ fdpd, int pb, int nb) {
  constexpr int PPW = kWave / Q;
  constexpr int NW = kPairThreads / kWave;
  __shared__ int s_qs[NW][kPairQueue];
  __shared__ int s_ql[NW][kPairQueue];
  __shared__ double s_rv[NW][PPW][6];
  __shared__ int s_id[NW][PPW];
  __shared__ int s_sp[NW][PPW];
  __shared__ unsigned long long s_f[NW][PPW][3];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int lb = (pb % kXcds) * (nb / kXcds) + pb / kXcds;  // XCD-contiguous logical block
  const int n = P.ncell, cap = P.cap;
  const int G = Q == 8 ? P.group8 : P.group4;
  const int64_t nc3 = (int64_t)n * n * n;
  const int64_t c0 = ((int64_t)lb * NW + w) * G;
  if (c0 >= nc3) return;  // whole wavefronts leave together
  const int ng = (int)((nc3 - c0) < G ? (nc3 - c0) : G);
  int total = 0;
  for (int k = 0; k < ng; ++k) {
    const int ck = dcnt[c0 + k];
    total += ck < cap ? ck : cap;
  }
  const int lp = lane / Q, quad = lane % Q;
  const double L = P.L, invL = 1.0 / L, isdt = 1.0 / sqrt(P.dt);
  int *qs = s_qs[w], *ql = s_ql[w];

  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  auto flush = [&](int qn) {
    wave_sync();
    for (int e = lane; e < qn; e += kWave) {
      const int l = ql[e];
      const int slot = qs[e];
      const int ii = s_id[w][l];
      const double4 ej = gload(cpos + slot);
      const double4 vj = gload(cvel + slot);
      const int j = (int)ej.w;
      double dx = s_rv[w][l][0] - ej.x, dy = s_rv[w][l][1] - ej.y, dz = s_rv[w][l][2] - ej.z;
      dx -= L * rint(dx * invL);
      dy -= L * rint(dy * invL);
      dz -= L * rint(dz * invL);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double r = sqrt(r2), ir = 1.0 / r;
      const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
      const double wr = 1.0 - r;
      const double vdot = (s_rv[w][l][3] - vj.x) * ex + (s_rv[w][l][4] - vj.y) * ey + (s_rv[w][l][5] - vj.z) * ez;
      const double th = dpd_theta(P.seed, step, ii, j);
      const double aij = P.nspec > 1 ? P.atab[4 * s_sp[w][l] + (int)vj.w] : P.a;
      const double mag = aij * wr - P.gamma * wr * wr * vdot + P.sigma * wr * th * isdt;
      atomicAdd(&s_f[w][l][0], (unsigned long long)to_fixed(mag * ex, kRealFxScale));
      atomicAdd(&s_f[w][l][1], (unsigned long long)to_fixed(mag * ey, kRealFxScale));
      atomicAdd(&s_f[w][l][2], (unsigned long long)to_fixed(mag * ez, kRealFxScale));
    }
    wave_sync();
  };

  for (int r0 = 0; r0 < total; r0 += PPW) {
    // particle r0 + lp of the group: cell ci, slot sl
    const int pidx = r0 + lp;
    const bool has = pidx < total;
    int ci = 0, own = 0, i = -1;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (has) {
      int k = 0, rem = pidx;
      for (; k < ng - 1; ++k) {
        int ck = dcnt[c0 + k];
        ck = ck < cap ? ck : cap;
        if (rem < ck) break;
        rem -= ck;
      }
      ci = (int)(c0 + k);
      own = ci * cap + rem;
      const double4 e = gload(cpos + own);
      rx = e.x;
      ry = e.y;
      rz = e.z;
      i = (int)e.w;
      if (quad < 3) s_f[w][lp][quad] = 0ull;
      if (quad == 0) {
        const double4 v = gload(cvel + own);
        s_rv[w][lp][0] = rx;
        s_rv[w][lp][1] = ry;
        s_rv[w][lp][2] = rz;
        s_rv[w][lp][3] = v.x;
        s_rv[w][lp][4] = v.y;
        s_rv[w][lp][5] = v.z;
        s_id[w][lp] = i;
        s_sp[w][lp] = (int)v.w;
      }
    }
    const int cx = ci / (n * n), cy = (ci / n) % n, cz = ci % n;
    // The lane's share of the 27 neighbour cells (o = quad, quad + Q, ...):
    // their counts are loaded together up front, and the lane's candidates
    // t = 0 .. T-1 (cell by cell, slot by slot) are then fetched kB at a time,
    // so that kB loads are in flight instead of one.
    constexpr int KC = (27 + Q - 1) / Q;
    constexpr int kB = 4;
    int cb[KC], cnk[KC], pre[KC];
    int T = 0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int o = quad + k * Q;
      const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
      const bool ok = has && o < 27 && dpd_offset_valid(ox, n) && dpd_offset_valid(oy, n) &&
                      dpd_offset_valid(oz, n);
      const int c = ok ? (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + mod_pos(cz + oz, n) : 0;
      int ck = ok ? dcnt[c] : 0;
      cnk[k] = ck < cap ? ck : cap;
      cb[k] = c * cap;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      pre[k] = T;
      T += cnk[k];
    }
    int qn = 0;  // wavefront-uniform queue length
    for (int t0 = 0;; t0 += kB) {
      if (__ballot(t0 < T) == 0ull) break;
      int slot[kB];
      double4 e[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int t = t0 + u;
        int sl = -1;
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (t >= pre[k] && t < pre[k] + cnk[k]) sl = cb[k] + (t - pre[k]);
        slot[u] = sl;
      }
#pragma unroll
      for (int u = 0; u < kB; ++u)
        if (slot[u] >= 0) e[u] = gload(cpos + slot[u]);
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        bool take = false;
        if (slot[u] >= 0) {
          const int j = (int)e[u].w;
          double dx = rx - e[u].x, dy = ry - e[u].y, dz = rz - e[u].z;
          dx -= L * rint(dx * invL);
          dy -= L * rint(dy * invL);
          dz -= L * rint(dz * invL);
          const double r2 = dx * dx + dy * dy + dz * dz;
          take = (j != i) && (r2 < 1.0) && (r2 != 0.0);
        }
        const unsigned long long m = __ballot(take);
        if (take) {
          const int at = qn + (int)__popcll(m & __lanemask_lt());
          qs[at] = slot[u];
          ql[at] = lp;
        }
        qn += (int)__popcll(m);
        if (qn > kPairQueue - kWave) {
          flush(qn);
          qn = 0;
        }
      }
    }
    flush(qn);

    // harmonic bonds of i, F_i = -K (r - r0) rhat_ij
    if (has && quad == 0) {
      long long fx = (long long)s_f[w][lp][0], fy = (long long)s_f[w][lp][1], fz = (long long)s_f[w][lp][2];
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
      fdpd[3 * i] = (double)fx * kRealFxInv;
      fdpd[3 * i + 1] = (double)fy * kRealFxInv;
      fdpd[3 * i + 2] = (double)fz * kRealFxInv;
    }
    wave_sync();  // the next round reuses the LDS rows of this one
  }
}

template <int Q>
__global__ void __launch_bounds__(kPairThreads)
k_dpd_pair(DpdParams P, uint64_t step, const double *__restrict__ pos, const int *__restrict__ dcnt,
           const double4 *__restrict__ cpos, const double4 *__restrict__ cvel,
           const int *__restrict__ bond_start, const int *__restrict__ bond_to, double *__restrict__ fdpd) {
  dpd_pair_body<Q>(P, step, to_g(pos), to_g(dcnt), to_g(cpos), to_g(cvel), to_g(bond_start), to_g(bond_to),
                   to_g(fdpd), blockIdx.x, gridDim.x);
}

int pair_group_cells(double cell_mean, int lanes) {
  const double per_round = 0.75 * (double)(kWave / lanes);
  int g = (int)(per_round / (cell_mean > 0.0 ? cell_mean : 1.0));
  return g < 1 ? 1 : (g > 64 ? 64 : g);
}

int pair_blocks(const DpdParams &P, int lanes) {
  const int64_t G = lanes == 8 ? P.group8 : P.group4;
  const int64_t nc3 = (int64_t)P.ncell * P.ncell * P.ncell;
  const int64_t waves = (nc3 + G - 1) / G;
  const int64_t nw = kPairThreads / kWave;
  int64_t blocks = (waves + nw - 1) / nw;
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  return (int)blocks;
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

// ---------------------------------------------------------------------------
// Batched DPD kernels: one launch covers every member of a batch.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
kb_dpd_pre(const BatchMember *__restrict__ mem, const int2 *__restrict__ map, int mode) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  dpd_pre_body(m.N, mode, m.P, m.pos, m.vel, m.force, m.v0, m.dcnt, m.cpos, m.cvel, m.status, m.ch, w.y);
}

template <int Q>
__global__ void __launch_bounds__(kPairThreads)
kb_dpd_pair(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  dpd_pair_body<Q>(m.P, *m.step, to_g(m.pos), to_g(m.dcnt), to_g(m.cpos), to_g(m.cvel), to_g(m.bond_start),
                   to_g(m.bond_to), to_g(m.fdpd), w.y, m.pair_blocks);
}

__global__ void k_set_u64(unsigned long long *dst, unsigned long long value) {
  if (threadIdx.x == 0) dst[0] = value;
}

hipError_t launch_batch_pre(const BatchMember *mem, const int2 *map, int nmap, int mode, hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_dpd_pre, dim3(nmap), dim3(256), 0, st, mem, map, mode);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const BatchMember *mem, const int2 *map, int nmap, int lanes, hipStream_t st) {
  if (nmap > 0) {
    if (lanes == 8)
      hipLaunchKernelGGL(kb_dpd_pair<8>, dim3(nmap), dim3(kPairThreads), 0, st, mem, map);
    else
      hipLaunchKernelGGL(kb_dpd_pair<4>, dim3(nmap), dim3(kPairThreads), 0, st, mem, map);
  }
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long *dst, unsigned long long value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, dst, value);
  return hipGetLastError();
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
                           const int *bond_start, const int *bond_to, double *fdpd, int lanes,
                           hipStream_t st, KernelTimer *tm) {
  (void)N;
  (void)v0;
  const int nb = pair_blocks(P, lanes);
  if (tm) tm->before(1, st);
  if (lanes == 8)
    hipLaunchKernelGGL(k_dpd_pair<8>, dim3(nb), dim3(kPairThreads), 0, st, P, step, pos, dcnt, cpos, cvel,
                       bond_start, bond_to, fdpd);
  else
    hipLaunchKernelGGL(k_dpd_pair<4>, dim3(nb), dim3(kPairThreads), 0, st, P, step, pos, dcnt, cpos, cvel,
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
