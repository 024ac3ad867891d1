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
#include "enuf_combine.h"

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
    // one 32 x 32 -> 64-bit product gives both halves (a single multiply-add instruction)
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// The update arithmetic below (wrap, predictor, kicks, drift) states its
// fused multiply-adds (no contraction left to the compiler): it is inlined
// into several kernels (one system, batches, fused with the combine), which
// must round alike.
__device__ inline double wrap_box(double x, double L) {
#pragma clang fp contract(off)
  double y = fma(-L, floor(x / L), x);
  if (!(y < L) || y < 0.0) y = 0.0;
  return y;
}

__device__ inline int dpd_cell_of(double x, double inv_cell, int n) {
  int c = (int)(x * inv_cell);
  return c < n ? (c < 0 ? 0 : c) : n - 1;
}

// The plan scalars of the charges (static for a DPD system), written by
// particle 0's thread.
__device__ __forceinline__ void dpd_pre_scalars(const DpdCharges &ch, int64_t i) {
  if (ch.enabled && i == 0) {
    ch.sc->nq = ch.stat.nq;
    ch.sc->scale = ch.stat.scale;
    ch.sc->inv_scale = ch.stat.inv_scale;
    ch.sc->sum_q = ch.stat.sum_q;
    ch.sc->sum_absq = ch.stat.sum_absq;
    ch.sc->sum_q2 = ch.stat.sum_q2;
  }
}

// Compaction slot j of particle i (-1: neutral) and its charge.
__device__ __forceinline__ int dpd_pre_slot(const DpdCharges &ch, int64_t i, double *qi) {
  const int j = ch.enabled ? ch.dslot[i] : -1;
  *qi = j >= 0 ? ch.q[i] : 0.0;
  return j;
}

// The pre step of particle i < N from its position r, velocity v and force f.
// mode 0: full predictor / half kick / drift; mode 1: forces only (v0 = v).
// Each particle is binned into a slot of its DPD cell together with its
// position (and index) and predicted velocity, so that the pair kernel reads
// neighbour data contiguously.
__device__ __forceinline__ void
dpd_pre_particle(int64_t i, int mode, const DpdParams &P, double *r, double *v, const double *f, int j, double qi,
                 double *__restrict__ pos, double *__restrict__ vel, int *dcnt, double4 *cpos, double4 *cvel,
                 int *status, const DpdCharges &ch) {
  double w[3];
  if (mode == 0) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      w[a] = fma(P.lam * P.dt, f[a], v[a]);
      v[a] = fma(0.5 * P.dt, f[a], v[a]);
      r[a] = wrap_box(fma(P.dt, v[a], r[a]), P.L);
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
  for (int a = 0; a < 3; ++a) pos[3 * i + a] = r[a];
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
    xc = mesh_cell(r[0], ch.m_over_l, ch.M, &t) * kXSub + (j & (kXSub - 1));  // x-cell sub-bin
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
        ch.cpre[(size_t)c * cp.cap + sl] = make_float4((float)r[0], (float)r[1], (float)r[2], __int_as_float(j));
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

__device__ __forceinline__ void
dpd_pre_body(int64_t N, int mode, const DpdParams &P, double *__restrict__ pos, double *__restrict__ vel,
             const double *__restrict__ force, int *dcnt, double4 *cpos, double4 *cvel, int *status,
             const DpdCharges &ch, int bid) {
  const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
  dpd_pre_scalars(ch, i);
  if (i >= N) return;
  // the static compaction slot and charge are loaded with the state
  double qi;
  const int j = dpd_pre_slot(ch, i, &qi);
  double r[3], v[3], f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = pos[3 * i + a];
    v[a] = vel[3 * i + a];
    f[a] = force[3 * i + a];
  }
  dpd_pre_particle(i, mode, P, r, v, f, j, qi, pos, vel, dcnt, cpos, cvel, status, ch);
}

__global__ void __launch_bounds__(256)
k_dpd_pre(int64_t N, int mode, DpdParams P, double *__restrict__ pos, double *__restrict__ vel,
          const double *__restrict__ force, int *dcnt, double4 *cpos, double4 *cvel, int *status,
          DpdCharges ch) {
  dpd_pre_body(N, mode, P, pos, vel, force, dcnt, cpos, cvel, status, ch, blockIdx.x);
}

// Minimum-image separation d = a - b and |d|^2, with the rounding written
// out (explicit fused multiply-adds, no contraction left to the compiler): the
// scan's FP64 test and the evaluation agree, and every instantiation of the
// pair kernels rounds alike, so a system's forces are bitwise the same alone
// and in a batch.
__device__ __forceinline__ double dpd_sep(const double4 &a, const double4 &b, double L, double invL, double &dx,
                                          double &dy, double &dz) {
#pragma clang fp contract(off)
  dx = a.x - b.x;
  dy = a.y - b.y;
  dz = a.z - b.z;
  dx = fma(-L, rint(dx * invL), dx);
  dy = fma(-L, rint(dy * invL), dy);
  dz = fma(-L, rint(dz * invL), dz);
  return fma(dx, dx, fma(dy, dy, dz * dz));
}

__device__ inline bool dpd_offset_valid(int o, int n) {
  return n >= 3 || (n == 2 && o >= 0) || (n == 1 && o == 0);
}

// Pair forces by column segment.  A block takes a segment of consecutive
// cells of one z-column of the DPD cell grid: about kPairSeg for one system
// (small blocks leave room on every CU for the mesh passes that run beside
// this kernel, and spread the work evenly), longer in batches, which fill the
// chip by themselves (the per-block counting and staging is then paid over
// more cells).  It stages in LDS every particle of
// the 9 neighbouring columns over the segment's z-range plus one cell on each
// side (periodic images in a whole column), ordered by z-slice first and
// column second: then the 27 neighbour cells of any cell of the segment are
// three consecutive z-slices, so the candidates of all particles of that cell
// form ONE contiguous range of the staged set.  Each staged particle keeps its
// position (with its index), an FP32 position relative to the segment,
// shifted to the periodic image next to it, with its cell slot, and (one
// system) its predicted velocity (with its species).  Batches read the
// velocity from the cell slot when a pair is evaluated: 48 instead of 80 bytes
// of LDS per staged particle let a 600-particle stage (longer segments) fit
// four blocks per CU.
// Scan: a wavefront takes the segment's cells one at a time (a shared
// counter deals them out); its 64 lanes take (particle, candidate) pairs of
// the cell, g particles x 64/g candidates per step, and append the pairs that
// pass the FP32 test r^2 < 1 + kPairMargin to a wavefront queue.
// Evaluation: the wavefront takes the queue 64 pairs at a time (full lanes
// however sparse the neighbours are), re-tests r < R_c = 1 exactly in FP64
// with the minimum image, and adds each pair force to i's int64 fixed-point
// accumulator in LDS.  Every pair is evaluated from both of its particles
// (theta_ij = theta_ji keeps the pair forces antisymmetric), so no thread
// writes another particle's force; the fixed-point sums (2^-36) are exact, so
// the result does not depend on the order in which pairs are visited.  The
// bonds of each particle are added last, and its force written once.
// A segment whose staged set exceeds the LDS stage (dense cells) is taken in
// chunks of whole z-cells that fit; a single z-cell that does not fit is
// taken with every candidate read from global memory instead.  Blocks are
// mapped so that each of the 8 XCDs (which take the blocks of a launch
// round-robin) works on one contiguous slab of columns.  Particles beyond a
// full cell's capacity (reported as ENUF_EOVERFLOW by the binning) get no
// force.  Grids of fewer than 3 cells per side (where a cell is its own
// neighbour more than once) test every staged particle of the column set.
constexpr int kPairThreads = 256;
constexpr int kPairWaves = kPairThreads / kWave;
constexpr int kPairQueue = 128;   // queued pairs per wavefront (64 evaluated at a time)
constexpr int kXcds = 8;          // MI355X: blocks of a launch are dealt round-robin to 8 XCDs
constexpr int kPairZ = kPairSegMax + 2;  // staged z-slices at most
constexpr int kPairCells = 9 * kPairZ;   // staged cells at most
static_assert(kPairCells <= kPairThreads, "the prefix sum takes one staged cell per thread");
static_assert(kPairCells <= 256, "staged cells are numbered in a byte");
// candidate steps in flight per lane: 8 for one system (153 VGPRs, 3 waves
// per SIMD; 4.5 % less step time than 4 at N = 24000, where the kernel runs
// beside the mesh passes); batches take 4 (122 VGPRs, 4 waves per SIMD; 8 %
// less batch step time than 8, the batch filling the chip) or 8
// (enuf_batch_set_tuning)
constexpr int kPairU = 8;
constexpr int kPairPer = (kPairStage + kPairThreads - 1) / kPairThreads;  // staged particles copied per thread and pass
constexpr float kPairMargin = 1.0e-3f;

struct PairShared {
  int cnt[kPairCells];    // counts of the staged cells (cell zslice * 9 + column)
  int off[kPairCells + 1];
  int gcell[kPairCells];  // grid cell of each staged cell
  int ownoff[kPairZ + 1]; // prefix over z-slices of the own column's counts
  unsigned char cellof[kPairStageMax];  // staged cell (from the chunk's first) of each staged particle
  int wsum[kPairWaves];
  int next;               // next own z-cell of the chunk (wavefront work counter)
  int qj[kPairWaves][kPairQueue];  // queued pairs: j, i (staged index or grid slot), i's accumulator
  int qi[kPairWaves][kPairQueue];
  unsigned char qa[kPairWaves][kPairQueue];
  unsigned long long acc[kPairOwn][3];
};

// Scan and evaluation over the own z-cells [zs, ze) of a chunk.  STAGED:
// candidates are staged indices (virtual index - base); otherwise grid slots.
// VLDS: the staged velocities are in LDS; otherwise they are read from their
// cell slots when a pair is evaluated.
template <int U, bool STAGED, bool VLDS>
__device__ __forceinline__ void
dpd_pair_cells(const DpdParams &P, uint64_t step, gptr<const double4> __restrict__ cpos,
               gptr<const double4> __restrict__ cvel, PairShared &sh, const double4 *s_pos,
               const double4 *s_vel, const float4 *s_rel, int base, int zs, int ze, int nz, bool tiny) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int cap = P.cap;
  const double L = P.L, invL = 1.0 / L, isdt = 1.0 / sqrt(P.dt);
  int *qj = sh.qj[w], *qi = sh.qi[w];
  unsigned char *qa = sh.qa[w];
  const int own0 = sh.ownoff[zs];

  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // grid slot of virtual staged index q, s_off[k0] <= q < s_off[k1]
  auto slot_of = [&](int q, int k0, int k1) -> int {
    int lo = k0, hi = k1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sh.off[mid] <= q) lo = mid; else hi = mid;
    }
    return sh.gcell[lo] * cap + (q - sh.off[lo]);
  };
  // evaluate queue entries [0, n) (n <= 64: one per lane)
  auto evaluate = [&](int n) {
    wave_sync();
    if (lane < n) {
#pragma clang fp contract(off)
      const int jq = qj[lane], iq = qi[lane], ia = qa[lane];
      const double4 pi = STAGED ? s_pos[iq] : gload(cpos + iq);
      const double4 pj = STAGED ? s_pos[jq] : gload(cpos + jq);
      // staged: the velocities from LDS, or from the cell slots that the
      // FP32 copies carry
      const double4 vi = !STAGED ? gload(cvel + iq) : (VLDS ? s_vel[iq] : gload(cvel + __float_as_int(s_rel[iq].w)));
      const double4 vj = !STAGED ? gload(cvel + jq) : (VLDS ? s_vel[jq] : gload(cvel + __float_as_int(s_rel[jq].w)));
      double dx, dy, dz;
      const double r2 = dpd_sep(pi, pj, L, invL, dx, dy, dz);
      if (r2 < 1.0 && r2 != 0.0) {
        const double r = sqrt(r2), ir = 1.0 / r;
        const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
        const double wr = 1.0 - r;
        const double vdot = fma(vi.x - vj.x, ex, fma(vi.y - vj.y, ey, (vi.z - vj.z) * ez));
        const double th = dpd_theta(P.seed, step, (int)pi.w, (int)pj.w);
        const double aij = P.nspec > 1 ? P.atab[4 * (int)vi.w + (int)vj.w] : P.a;
        // a_ij w - gamma w^2 (e.v) + sigma w theta / sqrt(dt)
        const double mag = fma(aij, wr, fma(-(P.gamma * wr * wr), vdot, P.sigma * wr * th * isdt));
        atomicAdd(&sh.acc[ia][0], (unsigned long long)to_fixed_fast(mag * ex, kRealFxScale));
        atomicAdd(&sh.acc[ia][1], (unsigned long long)to_fixed_fast(mag * ey, kRealFxScale));
        atomicAdd(&sh.acc[ia][2], (unsigned long long)to_fixed_fast(mag * ez, kRealFxScale));
      }
    }
    wave_sync();
  };
  // evaluate 64 queued pairs and move the rest (fewer than 64) to the front
  auto flush64 = [&](int qn) {
    evaluate(kWave);
    int j = 0, i = 0, a = 0;
    const bool mv = lane + kWave < qn;
    if (mv) {
      j = qj[lane + kWave];
      i = qi[lane + kWave];
      a = qa[lane + kWave];
    }
    wave_sync();
    if (mv) {
      qj[lane] = j;
      qi[lane] = i;
      qa[lane] = (unsigned char)a;
    }
  };

  int qn = 0;  // wavefront-uniform queue length, < 64 between steps
  for (;;) {
    int zi = 0;
    if (lane == 0) zi = atomicAdd(&sh.next, 1);
    zi = zs + __shfl(zi, 0, kWave);
    if (zi >= ze) break;
    const int ko = zi * 9 + 4;                  // the own column's cell of slice zi
    const int a_lo = sh.off[ko], n_a = sh.off[ko + 1] - a_lo;
    const int k0 = tiny ? 0 : (zi - 1) * 9, k1 = tiny ? nz * 9 : (zi + 2) * 9;
    const int lo = sh.off[k0], T = sh.off[k1] - lo;
    const int abase = sh.ownoff[zi] - own0;
    for (int a0 = 0; a0 < n_a; a0 += kWave) {
      const int g = (n_a - a0) < kWave ? (n_a - a0) : kWave;
      const int m = kWave / g;
      const bool act = lane < g * m;
      const int a = a0 + lane % g;
      int t = lane / g;
      const int ia = abase + a;
      const int iref = STAGED ? a_lo + a - base : sh.gcell[ko] * cap + a;
      float4 ri = make_float4(0.f, 0.f, 0.f, 0.f);
      double4 pi = make_double4(0.0, 0.0, 0.0, 0.0);
      if (STAGED) ri = s_rel[iref];
      else pi = gload(cpos + iref);
      for (;; t += U * m) {
        if (__ballot(act && t < T) == 0ull) break;
        int jref[U];
        float4 rj[U];
        double4 pj[U];
        // every lane loads (an in-range index when its step is past the
        // end), so that the loads of all steps are in flight together
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tu = t + u * m;
          const bool ok = act && tu < T;
          if (STAGED) {
            jref[u] = ok ? lo + tu - base : -1;
            rj[u] = s_rel[ok ? lo + tu - base : iref];
          } else {
            jref[u] = ok ? slot_of(lo + tu, k0, k1) : -1;
            pj[u] = gload(cpos + (ok ? jref[u] : iref));
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          bool take;
          if (STAGED) {
            const float dx = ri.x - rj[u].x, dy = ri.y - rj[u].y, dz = ri.z - rj[u].z;
            take = jref[u] >= 0 && jref[u] != iref && (tiny || dx * dx + dy * dy + dz * dz < 1.0f + kPairMargin);
          } else {
            double dx, dy, dz;
            const double r2 = dpd_sep(pi, pj[u], L, invL, dx, dy, dz);
            take = jref[u] >= 0 && jref[u] != iref && r2 < 1.0 && r2 != 0.0;
          }
          const unsigned long long bm = __ballot(take);
          if (take) {
            const int at = qn + (int)__popcll(bm & __lanemask_lt());
            qj[at] = jref[u];
            qi[at] = iref;
            qa[at] = (unsigned char)ia;
          }
          qn = __builtin_amdgcn_readfirstlane(qn + (int)__popcll(bm));
          if (qn >= kWave) {
            flush64(qn);
            qn -= kWave;
          }
        }
      }
    }
  }
  if (qn > 0) evaluate(qn);
}

template <int U, bool VLDS>
__device__ __forceinline__ void
dpd_pair_body(const DpdParams &P, uint64_t step, gptr<const double> __restrict__ pos,
              gptr<const int> __restrict__ dcnt, gptr<const double4> __restrict__ cpos,
              gptr<const double4> __restrict__ cvel, gptr<const int> __restrict__ bond_start,
              gptr<const int> __restrict__ bond_to, gptr<double> __restrict__ fdpd, int pb, int nb) {
  extern __shared__ __align__(16) unsigned char pair_smem[];
  __shared__ PairShared sh;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int lb = (pb % kXcds) * (nb / kXcds) + pb / kXcds;  // XCD-contiguous logical block
  const int n = P.ncell, cap = P.cap;
  const int col = lb / P.nseg, seg = lb % P.nseg;
  if (col >= n * n) return;  // whole block leaves together
  const int cx = col / n, cy = col % n;
  const bool tiny = n < 3;
  const int z0 = seg * P.seg_cells;
  const int zn = (n - z0) < P.seg_cells ? (n - z0) : P.seg_cells;  // own cells of the segment
  const int nz = tiny ? n : zn + 2;                                  // staged z-slices
  const int ncells = 9 * nz;
  const double L = P.L, edge = L / n, invL = 1.0 / L;
  // counts of the staged cells (invalid aliasing columns of tiny grids count 0)
  for (int k = threadIdx.x; k < ncells; k += kPairThreads) {
    const int zsl = k / 9, c9 = k % 9;
    const int ox = c9 / 3 - 1, oy = c9 % 3 - 1;
    int c = 0, cnt = 0;
    if (dpd_offset_valid(ox, n) && dpd_offset_valid(oy, n)) {
      const int z = tiny ? zsl : mod_pos(z0 - 1 + zsl, n);
      c = (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + z;
      cnt = dcnt[c];
      cnt = cnt < cap ? cnt : cap;
    }
    sh.cnt[k] = cnt;
    sh.gcell[k] = c;
  }
  __syncthreads();
  // exclusive prefix sum over at most 256 cells: one per thread, wavefront scans
  {
    const int k = threadIdx.x;
    const int v = k < ncells ? sh.cnt[k] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) sh.wsum[w] = x;
    __syncthreads();
    int b = 0;
    for (int q = 0; q < w; ++q) b += sh.wsum[q];
    if (k < ncells) sh.off[k] = b + x - v;
    if (k == ncells - 1) sh.off[ncells] = b + x;
    if (k <= nz) {
      int s = 0;
      for (int z = 0; z < k; ++z) s += sh.cnt[z * 9 + 4];
      sh.ownoff[k] = s;
    }
    __syncthreads();
  }
  // the stage: positions (with the particle index), with VLDS the predicted
  // velocities (with the species), and the FP32 image-shifted positions with
  // the particle's cell slot in the fourth word
  const int stage_cap = P.pair_stage;
  double4 *s_pos = reinterpret_cast<double4 *>(pair_smem);
  double4 *s_vel = VLDS ? s_pos + stage_cap : nullptr;
  float4 *s_rel = reinterpret_cast<float4 *>(s_pos + (VLDS ? 2 : 1) * stage_cap);
  // periodic image shifts and origin of the segment
  const double ox0 = cx * edge, oy0 = cy * edge, oz0 = (z0 - 1) * edge;
  const int zlo = tiny ? 0 : 1, zhi = zlo + (tiny ? n : zn);
  for (int zs = zlo; zs < zhi;) {
    // the chunk [zs, ze): the most own z-cells whose staged set and own
    // particles fit (every thread finds the same from LDS)
    const int kz0 = tiny ? 0 : zs - 1;
    int ze = zs;
    while (ze < zhi) {
      const int kz1 = tiny ? nz : ze + 2;
      if (sh.off[kz1 * 9] - sh.off[kz0 * 9] > stage_cap || sh.ownoff[ze + 1] - sh.ownoff[zs] > kPairOwn) break;
      ++ze;
    }
    bool staged = true;
    if (ze == zs) {  // one z-cell (at most cap <= kPairOwn own particles), read from global memory
      ze = zs + 1;
      staged = false;
    }
    const int kz1 = tiny ? nz : ze + 1;
    const int base = sh.off[kz0 * 9], S = sh.off[kz1 * 9] - base;
    const int nown = sh.ownoff[ze] - sh.ownoff[zs];
    if (staged) {
      // staged cell of each staged particle, then the copy: kPairPer
      // particles per thread with all their loads in flight together (an
      // index past the end repeats the last particle, which is written twice)
      for (int k = kz0 * 9 + threadIdx.x; k < kz1 * 9; k += kPairThreads) {
        const int o = sh.off[k] - base, c = sh.cnt[k];
        for (int q = 0; q < c; ++q) sh.cellof[o + q] = (unsigned char)(k - kz0 * 9);
      }
      __syncthreads();
      if (S > 0) {
        for (int p0 = 0; p0 < S; p0 += kPairPer * kPairThreads) {
          int pp[kPairPer], kk[kPairPer], gs[kPairPer];
          double4 e[kPairPer], v[kPairPer];
#pragma unroll
          for (int r = 0; r < kPairPer; ++r) {
            const int p = p0 + threadIdx.x + r * kPairThreads;
            pp[r] = p < S ? p : S - 1;
            kk[r] = kz0 * 9 + sh.cellof[pp[r]];
          }
#pragma unroll
          for (int r = 0; r < kPairPer; ++r) {
            const size_t g = (size_t)sh.gcell[kk[r]] * cap + (pp[r] + base - sh.off[kk[r]]);
            e[r] = gload(cpos + g);
            if (VLDS) v[r] = gload(cvel + g);
            gs[r] = (int)g;
          }
#pragma unroll
          for (int r = 0; r < kPairPer; ++r) {
            const int zsl = kk[r] / 9, c9 = kk[r] % 9;
            const int X = cx + c9 / 3 - 1, Y = cy + c9 % 3 - 1, Z = z0 - 1 + zsl;
            const double sx = (X < 0 ? -L : (X >= n ? L : 0.0)) - ox0;
            const double sy = (Y < 0 ? -L : (Y >= n ? L : 0.0)) - oy0;
            const double sz = (Z < 0 ? -L : (Z >= n ? L : 0.0)) - oz0;
            s_pos[pp[r]] = e[r];
            if (VLDS) s_vel[pp[r]] = v[r];
            s_rel[pp[r]] = make_float4((float)(e[r].x + sx), (float)(e[r].y + sy), (float)(e[r].z + sz),
                                       __int_as_float(gs[r]));
          }
        }
      }
    }
    for (int k = threadIdx.x; k < nown; k += kPairThreads) {
      sh.acc[k][0] = 0ull;
      sh.acc[k][1] = 0ull;
      sh.acc[k][2] = 0ull;
    }
    if (threadIdx.x == 0) sh.next = 0;
    __syncthreads();
    if (staged)
      dpd_pair_cells<U, true, VLDS>(P, step, cpos, cvel, sh, s_pos, s_vel, s_rel, base, zs, ze, nz, tiny);
    else
      dpd_pair_cells<U, false, VLDS>(P, step, cpos, cvel, sh, s_pos, s_vel, s_rel, base, zs, ze, nz, tiny);
    __syncthreads();
    // bonds, F_i = -K (r - r0) rhat_ij, and the force of each own particle
    for (int t = threadIdx.x; t < nown; t += kPairThreads) {
      int zi = zs;
      while (sh.ownoff[zi + 1] - sh.ownoff[zs] <= t) ++zi;
      const int a = t - (sh.ownoff[zi] - sh.ownoff[zs]);
      const int ko = zi * 9 + 4;
      const double4 e = staged ? s_pos[sh.off[ko] + a - base] : gload(cpos + (sh.gcell[ko] * cap + a));
      const int i = (int)e.w;
      long long fx = (long long)sh.acc[t][0], fy = (long long)sh.acc[t][1], fz = (long long)sh.acc[t][2];
      const int b1 = bond_start[i + 1];
      for (int b = bond_start[i]; b < b1; ++b) {
        const int j = bond_to[b];
        const double4 pj = make_double4(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], 0.0);
        double dx, dy, dz;
        const double r = sqrt(dpd_sep(e, pj, L, invL, dx, dy, dz));
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
    __syncthreads();  // the next chunk restages
    zs = ze;
  }
}

// step_dev: the step index is read from device memory (steps replayed from a
// graph), else it is `step`.
__global__ void __launch_bounds__(kPairThreads)
k_dpd_pair(DpdParams P, uint64_t step, const unsigned long long *step_dev, const double *__restrict__ pos,
           const int *__restrict__ dcnt, const double4 *__restrict__ cpos, const double4 *__restrict__ cvel,
           const int *__restrict__ bond_start, const int *__restrict__ bond_to, double *__restrict__ fdpd) {
  dpd_pair_body<kPairU, true>(P, step_dev ? (uint64_t)*step_dev : step, to_g(pos), to_g(dcnt), to_g(cpos),
                        to_g(cvel), to_g(bond_start), to_g(bond_to), to_g(fdpd), blockIdx.x, gridDim.x);
}

void pair_segments(int n, int target, int *seg_cells, int *nseg) {
  target = target < 1 ? 1 : (target > kPairSegMax ? kPairSegMax : target);
  *nseg = (n + target - 1) / target;
  *seg_cells = (n + *nseg - 1) / *nseg;
}

int pair_blocks(const DpdParams &P) {
  int64_t blocks = (int64_t)P.ncell * P.ncell * P.nseg;
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  return (int)blocks;
}

size_t pair_lds_bytes(const DpdParams &P, bool vlds) {
  return (size_t)P.pair_stage * ((vlds ? 2 : 1) * sizeof(double4) + sizeof(float4));
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

// The combine kernel of step k (forces, closing half kick) and the pre kernel
// of step k + 1 (predictor, half kick, drift, binning) in one launch: thread i
// finishes particle i's step and starts its next one.  No energy partials
// (steps inside a run skip them).  The real-space and mesh bin counts and the
// DPD cell counts come in two sets: the combine part clears step k's sets (b,
// fa.dcnt) while the pre part bins into step k + 1's (ch, dcnt).
// One wavefront per block: the kernel is a chain of dependent loads, stores
// and slot atomics per particle, and 4x more blocks spread it over 4x more
// CUs' memory pipelines (about 1 us less per step at N = 24000 than blocks of
// 256 threads).
constexpr int kCombinePreThreads = 64;

__global__ void __launch_bounds__(kCombinePreThreads)
k_combine_pre(int64_t N, const int *__restrict__ slot, const double4 *__restrict__ xq,
              const unsigned long long *__restrict__ freal, const double4 *__restrict__ part, int P2S,
              double fscale, int nblk, double *blk_eg, const unsigned long long *__restrict__ ereal,
              long long *blk_er, int *ccnt, int ncell3, int *xcnt, int M, FinishArgs fa, double *forces,
              DpdParams P, double *pos, int *dcnt, double4 *cpos, double4 *cvel, int *status,
              DpdCharges ch) {
  // the next step's own loads (position, compaction slot, charge) go out with
  // the combine's; the new force and half-kicked velocity stay in registers
  // (the velocity is stored once, after the next step's kick).  No barrier:
  // a thread's two halves touch only its own particle, and the combine
  // clears one set of bin counts while the pre part fills the other.
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r[3] = {0.0, 0.0, 0.0}, qi = 0.0, f[3], v[3];
  int j = -1;
  if (i < N) {
    j = dpd_pre_slot(ch, i, &qi);
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = pos[3 * i + a];
  }
  combine_body(N, to_g(slot), to_g(xq), to_g(freal), to_g(part), P2S, fscale, nblk, blk_eg, to_g(ereal), blk_er,
               ccnt, ncell3, xcnt, M * kXSub, fa, forces, blockIdx.x, f, v);
  dpd_pre_scalars(ch, i);
  if (i < N) dpd_pre_particle(i, 0, P, r, v, f, j, qi, pos, fa.vel, dcnt, cpos, cvel, status, ch);
}

hipError_t launch_combine_pre(const ComputeConfig &cfg, const ComputeBuffers &b, double *forces,
                              const FinishArgs &fa, const DpdParams &P, double *pos, int *dcnt, double4 *cpos,
                              double4 *cvel, int *status, const DpdCharges &ch, hipStream_t st, KernelTimer *tm) {
  // the per-block energy partials are sized for blocks of kPrepThreads; the
  // fused pre step takes the combine's half-kicked velocities (mode 0 only)
  if (fa.energies || fa.mode != 0) return hipErrorInvalidValue;
  const double fscale = combine_fscale(cfg);
  const int nb = (int)((cfg.N + kCombinePreThreads - 1) / kCombinePreThreads);
  if (tm) tm->before(9, st);
  hipLaunchKernelGGL(k_combine_pre, dim3(nb), dim3(kCombinePreThreads), 0, st, cfg.N, (const int *)b.slot,
                     (const double4 *)b.xq, (const unsigned long long *)b.freal, (const double4 *)b.part,
                     2 * cfg.mesh.win.p * cfg.mesh.nslot, fscale, nb, b.blk_eg,
                     (const unsigned long long *)b.ereal, b.blk_er, b.ccnt,
                     cfg.cells.ncell * cfg.cells.ncell * cfg.cells.ncell, b.xcnt, cfg.mesh.M, fa, forces, P, pos,
                     dcnt, cpos, cvel, status, ch);
  if (tm) tm->after(9, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched DPD kernels: one launch covers every member of a batch.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
kb_dpd_pre(const BatchMember *__restrict__ mem, const int2 *__restrict__ map, int mode) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  dpd_pre_body(m.N, mode, m.P, m.pos, m.vel, m.force, m.dcnt, m.cpos, m.cvel, m.status, m.ch, w.y);
}

template <int U>
__global__ void __launch_bounds__(kPairThreads)
kb_dpd_pair(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  dpd_pair_body<U, false>(m.P, *m.step, to_g(m.pos), to_g(m.dcnt), to_g(m.cpos), to_g(m.cvel),
                             to_g(m.bond_start), to_g(m.bond_to), to_g(m.fdpd), w.y, m.pair_blocks);
}

// Batched fused step boundary: the members' combine of step k (clearing
// their set of bin counts) and pre of step k + 1 (binning into the other);
// thread i finishes particle i's step and starts its next one.
__global__ void __launch_bounds__(kPrepThreads)
kb_combine_pre(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  FinishArgs fa;
  fa.mode = 0;
  fa.kappa = m.P.kappa;
  fa.dt = m.P.dt;
  fa.fdpd = m.fdpd;
  fa.vel = m.vel;
  fa.dcnt = m.dcnt;
  fa.ndcell3 = m.P.ncell * m.P.ncell * m.P.ncell;
  fa.energies = 0;
  fa.step_inc = m.step;
  const int nc = m.cfg.cells.ncell;
  // as in k_combine_pre: the next step's loads early, force and velocity in
  // registers, the velocity stored once
  const int64_t i = (int64_t)w.y * blockDim.x + threadIdx.x;
  double r[3] = {0.0, 0.0, 0.0}, qi = 0.0, f[3], v[3];
  int j = -1;
  if (i < m.N) {
    j = dpd_pre_slot(m.ch_next, i, &qi);
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = m.pos[3 * i + a];
  }
  combine_body(m.N, to_g(m.buf.slot), to_g(m.buf.xq), to_g(m.buf.freal), to_g(m.buf.part),
               2 * m.cfg.mesh.win.p * m.cfg.mesh.nslot, m.fscale, m.nblk, m.buf.blk_eg, to_g(m.buf.ereal),
               m.buf.blk_er, m.buf.ccnt, nc * nc * nc, m.buf.xcnt, m.cfg.mesh.M * kXSub, fa, m.force, w.y, f, v);
  dpd_pre_scalars(m.ch_next, i);
  if (i < m.N)
    dpd_pre_particle(i, 0, m.P, r, v, f, j, qi, m.pos, m.vel, m.dcnt_next, m.cpos, m.cvel, m.status, m.ch_next);
}

__global__ void k_set_u64(unsigned long long *dst, unsigned long long value) {
  if (threadIdx.x == 0) dst[0] = value;
}

__global__ void k_add_u64(unsigned long long *dst) {
  if (threadIdx.x == 0) dst[0] += 1ull;
}

// one system stages kPairStage particles with their velocities; every
// member of a batch stages kBatchPairStage without them
constexpr size_t kPairLdsBytes = (size_t)kPairStage * (2 * sizeof(double4) + sizeof(float4));
constexpr size_t kBatchPairLdsBytes = (size_t)kBatchPairStage * (sizeof(double4) + sizeof(float4));

hipError_t configure_pair_kernels(size_t lds_bytes) {
  const int v = (int)(lds_bytes > kPairLdsBytes ? lds_bytes : kPairLdsBytes);
  hipError_t e = hipFuncSetAttribute((const void *)k_dpd_pair, hipFuncAttributeMaxDynamicSharedMemorySize, v);
  const void *k[] = {(const void *)kb_dpd_pair<4>, (const void *)kb_dpd_pair<8>};
  for (const void *f : k)
    if (e == hipSuccess)
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchPairLdsBytes);
  return e;
}

hipError_t launch_batch_pre(const BatchMember *mem, const int2 *map, int nmap, int mode, hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_dpd_pre, dim3(nmap), dim3(256), 0, st, mem, map, mode);
  return hipGetLastError();
}

hipError_t launch_batch_combine_pre(const BatchMember *mem, const int2 *map, int nmap, hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_combine_pre, dim3(nmap), dim3(kPrepThreads), 0, st, mem, map);
  return hipGetLastError();
}

hipError_t launch_batch_pair(const BatchMember *mem, const int2 *map, int nmap, int steps, hipStream_t st) {
  if (steps != 4 && steps != 8) return hipErrorInvalidValue;
  if (nmap > 0) {
    if (steps == 4)
      hipLaunchKernelGGL(kb_dpd_pair<4>, dim3(nmap), dim3(kPairThreads), kBatchPairLdsBytes, st, mem, map);
    else
      hipLaunchKernelGGL(kb_dpd_pair<8>, dim3(nmap), dim3(kPairThreads), kBatchPairLdsBytes, st, mem, map);
  }
  return hipGetLastError();
}

hipError_t launch_add_u64(unsigned long long *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, st, dst);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long *dst, unsigned long long value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, dst, value);
  return hipGetLastError();
}

hipError_t launch_dpd_pre(int64_t N, int mode, const DpdParams &P, double *pos, double *vel,
                          const double *force, int *dcnt, double4 *cpos, double4 *cvel, int *status,
                          const DpdCharges &ch, hipStream_t st, KernelTimer *tm) {
  const int nb = (int)((N + 255) / 256);
  if (tm) tm->before(0, st);
  hipLaunchKernelGGL(k_dpd_pre, dim3(nb), dim3(256), 0, st, N, mode, P, pos, vel, force, dcnt, cpos, cvel,
                     status, ch);
  if (tm) tm->after(0, st);
  return hipGetLastError();
}

hipError_t launch_dpd_pair(int64_t N, const DpdParams &P, uint64_t step, const double *pos, const int *dcnt,
                           const double4 *cpos, const double4 *cvel, const int *bond_start, const int *bond_to,
                           double *fdpd, hipStream_t st, KernelTimer *tm, const unsigned long long *step_dev) {
  (void)N;
  const int nb = pair_blocks(P);
  if (tm) tm->before(1, st);
  hipLaunchKernelGGL(k_dpd_pair, dim3(nb), dim3(kPairThreads), pair_lds_bytes(P, true), st, P, step, step_dev, pos,
                     dcnt, cpos, cvel, bond_start, bond_to, fdpd);
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
