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
  // the static compaction slot and charge are loaded with the state
  const int j = ch.enabled ? ch.dslot[i] : -1;
  const double qi = j >= 0 ? ch.q[i] : 0.0;
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
  // cells of a charge: real-space grid and mesh x-bin
  int c = 0, xc = 0;
  if (j >= 0) {
    const CellParams &cp = ch.cells;
    int cx = (int)(r[0] * cp.inv_cell), cy = (int)(r[1] * cp.inv_cell), cz = (int)(r[2] * cp.inv_cell);
    cx = cx < cp.ncell ? cx : cp.ncell - 1;
    cy = cy < cp.ncell ? cy : cp.ncell - 1;
    cz = cz < cp.ncell ? cz : cp.ncell - 1;
    c = (cx * cp.ncell + cy) * cp.ncell + cz;
    double t;
    xc = mesh_cell(r[0], ch.m_over_l, ch.M, &t);
  }
  // the slot claims are independent: all are in flight together
  const int s = atomicAdd(&dcnt[cell], 1);
  int sl = 0, xs = 0;
  if (j >= 0) {
    sl = atomicAdd(&ch.ccnt[c], 1);
    xs = atomicAdd(&ch.xcnt[xc], 1);
  }
  if (s < P.cap) {
    cpos[(size_t)cell * P.cap + s] = make_double4(r[0], r[1], r[2], (double)i);
    const double sp = P.nspec > 1 ? (double)P.species[i] : 0.0;
    cvel[(size_t)cell * P.cap + s] = make_double4(w[0], w[1], w[2], sp);
  } else {
    atomicCAS(status, 0, kEOverflow);
  }
  if (ch.enabled) {
    ch.slot[i] = j;
    if (j >= 0) {
      ch.xq[j] = make_double4(r[0], r[1], r[2], qi);
      const CellParams &cp = ch.cells;
      if (sl < cp.cap) {
        ch.cgrid[(size_t)c * cp.cap + sl] = make_double4(r[0], r[1], r[2], qi);
        ch.cidx[(size_t)c * cp.cap + sl] = j;
      } else {
        atomicCAS(&ch.sc->status, 0, kEOverflow);
      }
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

// Pair forces by column segment.  A block takes a segment of seg_cells
// consecutive cells of one z-column of the DPD cell grid (the whole column
// when it has at most kSegWhole cells).  It first stages in LDS every
// particle of the 9 neighbouring columns over the segment's z-range plus one
// cell on each side (the whole column: no halo): the cell counts are read and
// prefix-summed, then the positions are copied with all loads in flight
// together (predicted velocities are read from global memory by the pair
// evaluation, which keeps the block small enough for three per CU).  The segment's own particles form one contiguous
// range of the staged set; each wavefront takes 64/Q of them at a time with Q
// = 4 or 8 lanes per particle.
// Scan: each lane walks the staged particles of its share of the particle's
// 27 neighbour cells (LDS reads, kB at a time) and appends the pairs with
// r < R_c = 1 to a wavefront queue in LDS.  Evaluation: the whole wavefront
// takes the queued pairs 64 at a time (so the Philox draw and the pair force
// run with full lanes however sparse the neighbours are) and adds each pair
// force to i's int64 fixed-point accumulator in LDS.  Every pair is evaluated
// from both of its particles (theta_ij = theta_ji keeps the pair forces
// antisymmetric), so no thread writes another particle's force; the
// fixed-point sums (2^-36) are exact, so the result does not depend on the
// order in which pairs are visited.  With species, the cell slot's predicted
// velocity carries the species in w and the amplitude a_ij is read from the
// symmetric table in the parameters.  A segment whose neighbourhood holds
// more than kPairStage particles (dense cells) runs the same algorithm with
// the candidates read from global memory instead.  Blocks are mapped so that
// each of the 8 XCDs (which take the blocks of a launch round-robin) works on
// one contiguous slab of columns.  Particles beyond a full cell's capacity
// (reported as ENUF_EOVERFLOW by the binning) get no force.
constexpr int kPairThreads = 256;
constexpr int kPairQueue = 128;   // queued pairs per wavefront (flushed at > 64)
constexpr int kXcds = 8;          // MI355X: blocks of a launch are dealt round-robin to 8 XCDs
constexpr int kPairCells = 256;   // staged cells: 9 columns x at most 28 z-cells
constexpr int kSegWhole = 24;     // columns of at most this many cells are one segment
constexpr int kSegCells = 16;     // segment length of longer columns

// Per-wavefront LDS of the pair evaluation: the pair queue and the rows of
// the particles of the current round.
template <int Q>
struct PairScratch {
  static constexpr int PPW = kWave / Q;
  static constexpr int NW = kPairThreads / kWave;
  int qs[NW][kPairQueue];
  int ql[NW][kPairQueue];
  double rv[NW][PPW][6];
  int id[NW][PPW];
  int sp[NW][PPW];
  unsigned long long f[NW][PPW][3];
};

template <int Q, bool STAGED>
__device__ __forceinline__ void
dpd_pair_segment(const DpdParams &P, uint64_t step, gptr<const double> __restrict__ pos,
                 gptr<const double4> __restrict__ cpos, gptr<const double4> __restrict__ cvel,
                 gptr<const int> __restrict__ bond_start, gptr<const int> __restrict__ bond_to,
                 gptr<double> __restrict__ fdpd, PairScratch<Q> &sh, const int *s_cnt, const int *s_off,
                 const int *s_gcell, const double4 *s_pos, const int *s_gs, const int *s_pc, int Sz, int zlo,
                 int zhi) {
  constexpr int PPW = kWave / Q;
  constexpr int NW = kPairThreads / kWave;
  auto &s_qs = sh.qs;
  auto &s_ql = sh.ql;
  auto &s_rv = sh.rv;
  auto &s_id = sh.id;
  auto &s_sp = sh.sp;
  auto &s_f = sh.f;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int n = P.ncell, cap = P.cap;
  const int lp = lane / Q, quad = lane % Q;
  const double L = P.L, invL = 1.0 / L, isdt = 1.0 / sqrt(P.dt);
  int *qs = s_qs[w], *ql = s_ql[w];
  const bool whole = P.seg_whole != 0;
  // staged index of particle s of staged cell k (STAGED) or its global slot
  auto where = [&](int k, int sl) { return STAGED ? s_off[k] + sl : s_gcell[k] * cap + sl; };
  auto cand = [&](int q) -> double4 { return STAGED ? s_pos[q] : gload(cpos + q); };
  auto cvel_of = [&](int q) -> double4 { return gload(cvel + (STAGED ? s_gs[q] : q)); };

  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  auto flush = [&](int qn) {
    wave_sync();
    for (int e = lane; e < qn; e += kWave) {
      const int l = ql[e];
      const int q = qs[e];
      const int ii = s_id[w][l];
      const double4 ej = cand(q);
      const double4 vj = cvel_of(q);
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

  // own particles: staged cells 4 Sz + zlo .. 4 Sz + zhi - 1 (column (0, 0)), contiguous
  const int own0 = 4 * Sz;
  const int plo = s_off[own0 + zlo], phi = s_off[own0 + zhi];
  for (int r0 = plo + w * PPW; r0 < phi; r0 += NW * PPW) {
    const int pidx = r0 + lp;
    const bool has = pidx < phi;
    int zi = 0, i = -1;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (has) {
      int k;
      if (STAGED) {
        k = s_pc[pidx];
      } else {
        k = own0 + zlo;
        while (k < own0 + zhi - 1 && pidx >= s_off[k + 1]) ++k;
      }
      zi = k - own0;
      const int q = where(k, pidx - s_off[k]);
      const double4 e = cand(q);
      rx = e.x;
      ry = e.y;
      rz = e.z;
      i = (int)e.w;
      if (quad < 3) s_f[w][lp][quad] = 0ull;
      if (quad == 0) {
        const double4 v = cvel_of(q);
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
    // The lane's share of the 27 neighbour cells (o = quad, quad + Q, ...),
    // as staged cells; its candidates t = 0 .. T-1 (cell by cell, slot by
    // slot) are read kB at a time.
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
      int z = zi + oz;
      if (whole) z = z < 0 ? z + Sz : (z >= Sz ? z - Sz : z);
      const int kc = ((ox + 1) * 3 + (oy + 1)) * Sz + z;
      cnk[k] = ok ? s_cnt[kc] : 0;
      cb[k] = ok ? where(kc, 0) : 0;
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
        if (slot[u] >= 0) e[u] = cand(slot[u]);
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
__device__ __forceinline__ void
dpd_pair_body(const DpdParams &P, uint64_t step, gptr<const double> __restrict__ pos,
              gptr<const int> __restrict__ dcnt, gptr<const double4> __restrict__ cpos,
              gptr<const double4> __restrict__ cvel, gptr<const int> __restrict__ bond_start,
              gptr<const int> __restrict__ bond_to, gptr<double> __restrict__ fdpd, int pb, int nb) {
  extern __shared__ __align__(16) unsigned char pair_smem[];
  __shared__ PairScratch<Q> sh;
  __shared__ int s_cnt[kPairCells], s_off[kPairCells + 1], s_gcell[kPairCells];
  __shared__ int s_wsum[kPairThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int lb = (pb % kXcds) * (nb / kXcds) + pb / kXcds;  // XCD-contiguous logical block
  const int n = P.ncell, cap = P.cap;
  const int col = lb / P.nseg, seg = lb % P.nseg;
  if (col >= n * n) return;  // whole block leaves together
  const int cx = col / n, cy = col % n;
  const bool whole = P.seg_whole != 0;
  const int z0 = seg * P.seg_cells;
  const int zn = (n - z0) < P.seg_cells ? (n - z0) : P.seg_cells;  // own cells of the segment
  const int Sz = whole ? n : P.seg_cells + 2;                         // staged z-cells per column
  const int zlo = whole ? 0 : 1, zhi = zlo + zn;
  const int ncells = 9 * Sz;
  // counts of the staged cells (invalid aliasing columns of tiny grids count 0)
  for (int k = threadIdx.x; k < ncells; k += kPairThreads) {
    const int c9 = k / Sz, zs = k % Sz;
    const int ox = c9 / 3 - 1, oy = c9 % 3 - 1;
    int c = 0, cnt = 0;
    if (dpd_offset_valid(ox, n) && dpd_offset_valid(oy, n)) {
      const int z = whole ? zs : mod_pos(z0 - 1 + zs, n);
      c = (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + z;
      cnt = dcnt[c];
      cnt = cnt < cap ? cnt : cap;
    }
    s_cnt[k] = cnt;
    s_gcell[k] = c;
  }
  __syncthreads();
  // exclusive prefix sum over at most 256 cells: one per thread, wavefront scans
  {
    const int k = threadIdx.x;
    const int v = k < ncells ? s_cnt[k] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wsum[w] = x;
    __syncthreads();
    int base = 0;
    for (int q = 0; q < w; ++q) base += s_wsum[q];
    if (k < ncells) s_off[k] = base + x - v;
    if (k == ncells - 1) s_off[ncells] = base + x;
    __syncthreads();
  }
  const int S = s_off[ncells];
  const int stage_cap = P.pair_stage;
  double4 *s_pos = reinterpret_cast<double4 *>(pair_smem);
  int *s_gs = reinterpret_cast<int *>(s_pos + stage_cap);  // global slot of each staged particle
  int *s_pc = s_gs + stage_cap;                             // its staged cell
  if (S <= stage_cap) {
    // copy the staged particles: particle p of staged cell k (binary search over the offsets)
    for (int p = threadIdx.x; p < S; p += kPairThreads) {
      int lo = 0, hi = ncells;  // s_off[lo] <= p < s_off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= p) lo = mid; else hi = mid;
      }
      const int g = s_gcell[lo] * cap + (p - s_off[lo]);
      s_pos[p] = gload(cpos + g);
      s_gs[p] = g;
      s_pc[p] = lo;
    }
    __syncthreads();
    dpd_pair_segment<Q, true>(P, step, pos, cpos, cvel, bond_start, bond_to, fdpd, sh, s_cnt, s_off, s_gcell,
                              s_pos, s_gs, s_pc, Sz, zlo, zhi);
  } else {
    dpd_pair_segment<Q, false>(P, step, pos, cpos, cvel, bond_start, bond_to, fdpd, sh, s_cnt, s_off, s_gcell,
                               s_pos, s_gs, s_pc, Sz, zlo, zhi);
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

void pair_segments(int n, int *seg_cells, int *nseg, int *whole) {
  if (n <= kSegWhole) {
    *seg_cells = n;
    *nseg = 1;
    *whole = 1;
  } else {
    *seg_cells = kSegCells;
    *nseg = (n + kSegCells - 1) / kSegCells;
    *whole = 0;
  }
}

int pair_blocks(const DpdParams &P, int lanes) {
  (void)lanes;
  int64_t blocks = (int64_t)P.ncell * P.ncell * P.nseg;
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  return (int)blocks;
}

size_t pair_lds_bytes(const DpdParams &P) {
  return (size_t)P.pair_stage * (sizeof(double4) + 2 * sizeof(int));
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

// every member stages kPairStage particles
constexpr size_t kPairLdsBytes = (size_t)kPairStage * (sizeof(double4) + 2 * sizeof(int));

hipError_t configure_pair_kernels(size_t lds_bytes) {
  const int v = (int)(lds_bytes > kPairLdsBytes ? lds_bytes : kPairLdsBytes);
  const void *k[] = {(const void *)k_dpd_pair<4>, (const void *)k_dpd_pair<8>, (const void *)kb_dpd_pair<4>,
                     (const void *)kb_dpd_pair<8>};
  for (const void *f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch_pre(const BatchMember *mem, const int2 *map, int nmap, int mode, hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_dpd_pre, dim3(nmap), dim3(256), 0, st, mem, map, mode);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const BatchMember *mem, const int2 *map, int nmap, int lanes, hipStream_t st) {
  if (nmap > 0) {
    if (lanes == 8)
      hipLaunchKernelGGL(kb_dpd_pair<8>, dim3(nmap), dim3(kPairThreads), kPairLdsBytes, st, mem, map);
    else
      hipLaunchKernelGGL(kb_dpd_pair<4>, dim3(nmap), dim3(kPairThreads), kPairLdsBytes, st, mem, map);
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
    hipLaunchKernelGGL(k_dpd_pair<8>, dim3(nb), dim3(kPairThreads), pair_lds_bytes(P), st, P, step, pos, dcnt, cpos, cvel,
                       bond_start, bond_to, fdpd);
  else
    hipLaunchKernelGGL(k_dpd_pair<4>, dim3(nb), dim3(kPairThreads), pair_lds_bytes(P), st, P, step, pos, dcnt, cpos, cvel,
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
