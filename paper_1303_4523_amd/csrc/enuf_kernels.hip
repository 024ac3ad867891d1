// enuf_kernels.hip -- HIP kernels (gfx950) of one ENUF energy + force evaluation.
//
// Pipeline of enuf_compute (all on one stream):
//   k_prep_count    count charged particles per block; clear cell counts
//   k_prep_compact  wrap positions, compact the charges in index order, bin
//                   them into the real-space cell grid and by mesh x-cell,
//                   reduce sum q, |q|, q^2
//   k_real          real-space pair term (eq. 31 + Slater correction eq. 27)
//   k_recip_fwd     per x-plane: window spread (transposed NFFT, eq. 14) into
//                   an LDS plane, z real-to-complex FFT, y FFT, keep |k| < Kc
//   k_recip_x       per ky row: x FFT, influence multiply and FP64 energy
//                   (eq. 18/20), inverse x FFT
//   k_recip_bwd     per x-plane: inverse y FFT, complex-to-real z FFT, gather
//                   of potential and window gradient at the charges (eq. 22-25)
//   k_combine       per particle: add the 2p plane partials and the real-space
//                   force, scatter to the output; final energies
// Accumulations that cross threads are either fixed-order reductions or exact
// int64 fixed-point sums, so results are bitwise reproducible.
#include "enuf_device.h"
#include "enuf_dpd.h"
#include "enuf_combine.h"

namespace enuf {

template <typename T> struct CplxOf;
template <> struct CplxOf<double> { using type = double2; };
template <> struct CplxOf<float> { using type = float2; };

__device__ inline double wrap_coord(double x, double L) {
  double y = x - L * floor(x / L);
  if (!(y < L) || y < 0.0) y = 0.0;
  return y;
}

__device__ inline void set_status(DevScalars *sc, int code) { atomicCAS(&sc->status, 0, code); }
__device__ inline void set_status(gptr<DevScalars> sc, int code) {
  int expected = 0;
  __hip_atomic_compare_exchange_strong(&sc->status, &expected, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Preparation
// ---------------------------------------------------------------------------
// Per block: the number of charged particles and the sums of q, |q| and q^2,
// a charge counting as 0 when its position or value is not finite (as the
// compaction stores it; such input is reported as ENUF_ENONFINITE here, before
// the neutrality of the sums is checked).
__global__ void __launch_bounds__(kPrepThreads)
k_prep_count(int64_t N, const double *__restrict__ pos, const double *__restrict__ q, int *blk_cnt,
             double *blk_sums, int *ccnt, int ncell3, int *xcnt, int M, DevScalars *sc) {
  __shared__ double s_dbl[kPrepThreads / kWave];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int flag = (i < N) && (q[i] != 0.0);
  double qi = 0.0;
  if (i < N) {
    qi = q[i];
    if (!(isfinite(pos[3 * i]) && isfinite(pos[3 * i + 1]) && isfinite(pos[3 * i + 2]) && isfinite(qi))) {
      qi = 0.0;
      set_status(sc, kENonFinite);
    }
  }
  const int c = __syncthreads_count(flag);
  const double sq = block_sum(qi, s_dbl);
  const double sa = block_sum(fabs(qi), s_dbl);
  const double s2 = block_sum(qi * qi, s_dbl);
  if (threadIdx.x == 0) {
    blk_cnt[blockIdx.x] = c;
    blk_sums[3 * blockIdx.x] = sq;
    blk_sums[3 * blockIdx.x + 1] = sa;
    blk_sums[3 * blockIdx.x + 2] = s2;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < ncell3; k += stride) ccnt[k] = 0;
  for (int64_t k = i; k < M; k += stride) xcnt[k] = 0;
}

// Sums of the charges, their count and the fixed-point scale of the mesh
// accumulator from the per-block partials of the count kernel (one block).
__device__ inline void prep_scalars(int nblk, const int *__restrict__ blk_cnt, const double *__restrict__ blk_sums,
                                    DevScalars *sc) {
  __shared__ int s_int[kPrepThreads / kWave];
  __shared__ double s_dbl[kPrepThreads / kWave];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  int nq = 0;
  for (int k = tid; k < nblk; k += blockDim.x) {
    a += blk_sums[3 * k];
    b += blk_sums[3 * k + 1];
    c += blk_sums[3 * k + 2];
    nq += blk_cnt[k];
  }
  a = block_sum(a, s_dbl);
  b = block_sum(b, s_dbl);
  c = block_sum(c, s_dbl);
  nq = block_sum_int(nq, s_int);
  if (tid == 0) {
    sc->nq = nq;
    sc->sum_q = a;
    sc->sum_absq = b;
    sc->sum_q2 = c;
    // Mesh values are bounded by sum |q| (the window is <= 1): choose the
    // largest power of two keeping sum|q| * scale below 2^61.
    int e;
    frexp(b + 1.0, &e);
    sc->scale = ldexp(1.0, 61 - e);
    sc->inv_scale = ldexp(1.0, e - 61);
    if (fabs(a) > 1e-10 * b) set_status(sc, kENonNeutral);
  }
}

__global__ void __launch_bounds__(kPrepThreads)
k_prep_compact(int64_t N, const double *__restrict__ pos, const double *__restrict__ q,
               double L, CellParams cp, const int *__restrict__ blk_cnt, int nblk,
               const double *__restrict__ blk_sums, double4 *xq, int *idx, int *slot, int *ccnt, double4 *cgrid,
               float4 *cpre, int *xcnt, int *xslot, int M, double m_over_l, int xcap, DevScalars *sc) {
  __shared__ int s_int[kPrepThreads / kWave];
  __shared__ int s_wcnt[kPrepThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
  if (blockIdx.x == 0) prep_scalars(nblk, blk_cnt, blk_sums, sc);

  int part = 0;
  for (int b = tid; b < (int)blockIdx.x; b += blockDim.x) part += blk_cnt[b];
  const int off = block_sum_int(part, s_int);

  double x = 0.0, y = 0.0, z = 0.0, qi = 0.0;
  int charged = 0, bad = 0;
  if (i < N) {
    qi = q[i];
    charged = (qi != 0.0);
    x = pos[3 * i];
    y = pos[3 * i + 1];
    z = pos[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(qi))) {
      bad = 1;
      x = y = z = 0.0;
      qi = 0.0;
    }
    x = wrap_coord(x, L);
    y = wrap_coord(y, L);
    z = wrap_coord(z, L);
  }
  const unsigned long long m = __ballot(charged);
  const int rank = __popcll(m & __lanemask_lt());
  if (lane == 0) s_wcnt[w] = __popcll(m);
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += s_wcnt[k];
  if (i < N) {
    if (charged) {
      const int j = off + woff + rank;
      xq[j] = make_double4(x, y, z, qi);
      idx[j] = (int)i;
      slot[i] = j;
      int cx = (int)(x * cp.inv_cell), cy = (int)(y * cp.inv_cell), cz = (int)(z * cp.inv_cell);
      cx = cx < cp.ncell ? cx : cp.ncell - 1;
      cy = cy < cp.ncell ? cy : cp.ncell - 1;
      cz = cz < cp.ncell ? cz : cp.ncell - 1;
      const int cell = (cx * cp.ncell + cy) * cp.ncell + cz;
      const int s = atomicAdd(&ccnt[cell], 1);
      if (s < cp.cap) {
        cgrid[(size_t)cell * cp.cap + s] = make_double4(x, y, z, qi);
        cpre[(size_t)cell * cp.cap + s] = make_float4((float)x, (float)y, (float)z, __int_as_float(j));
      } else {
        set_status(sc, kEOverflow);
      }
      double t;
      const int xc = mesh_cell(x, m_over_l, M, &t);
      const int xb = xc * kXSub + (j & (kXSub - 1));
      const int xs = atomicAdd(&xcnt[xb], 1);
      if (xs < xcap)
        xslot[(size_t)xb * xcap + xs] = j;
      else
        set_status(sc, kEOverflow);
    } else {
      slot[i] = -1;
    }
    if (bad) set_status(sc, kENonFinite);
  }
}

// ---------------------------------------------------------------------------
// Real space: eq. 31 with the additive Slater correction of eq. 27.
// u(r) = [erfc(a r) - (1 + x) e^{-2x}]/r, x = r/lambda; force factor
// f = -u'(r)/r so that F_i = q_i q_j f (r_i - r_j).  For x < 1/2 the
// closed forms cancel; there u = e^{-2x} b1/lambda - (2a/sqrt(pi)) e^{-a^2r^2} g0
// and f = e^{-2x} b2/lambda^3 - (2a^3/sqrt(pi)) e^{-a^2r^2} g1 with the
// all-positive series b1 = 1 + sum_{n>=2} 2^n x^{n-1}/n!,
// b2 = sum_{n>=3} 2^n x^{n-3}/n!, g0 = sum_{n>=0} 2^n z^{2n}/(2n+1)!!,
// g1 = sum_{n>=1} 2^n z^{2n-2}/(2n+1)!! (z = a r; the erf series is
// Abramowitz & Stegun 7.1.6).
// ---------------------------------------------------------------------------
__device__ inline bool real_pair(double r, double a, double lam, double *u, double *us, double *f) {
  // no contraction left to the compiler: every instantiation of the
  // real-space kernels rounds these terms alike (a system's forces are
  // bitwise the same alone and in a batch)
#pragma clang fp contract(off)
  const double k2 = 1.1283791670955125739;  // 2/sqrt(pi)
  if (lam > 0.0 && r < 0.5 * lam) {
    const double x = r / lam, y = 2.0 * x, z = a * r, z2 = z * z;
    double b2 = 4.0 / 3.0, term = 4.0 / 3.0, b1 = 1.0 + 2.0 * x + b2 * x * x;
    // the series stay rolled: this branch is rare (r < lambda / 2), and
    // unrolled it set the register count of the whole real-space kernel
#pragma unroll 1
    for (int n = 4; n < 30; ++n) {
      term *= y / n;
      b2 += term;
      b1 += term * x * x;
    }
    double t0 = 1.0, g0 = 1.0;
#pragma unroll 1
    for (int n = 1; n < 20; ++n) {
      t0 *= 2.0 * z2 / (2.0 * n + 1.0);
      g0 += t0;
    }
    double t1 = 2.0 / 3.0, g1 = 0.0;
#pragma unroll 1
    for (int n = 1; n < 20; ++n) {
      g1 += t1;
      t1 *= 2.0 * z2 / (2.0 * n + 3.0);
    }
    const double ex = exp(-y), ez = exp(-z2);
    *u = ex * b1 / lam - k2 * a * ez * g0;
    *us = (r > 0.0) ? -(1.0 + x) * ex / r : 0.0;
    *f = (r > 0.0) ? (ex * b2 / (lam * lam * lam) - k2 * a * a * a * ez * g1) : 0.0;
    return true;
  }
  if (r == 0.0) return false;
  const double ar = a * r, ec = erfc(ar), r2 = r * r;
  double uu = ec / r;
  double ff = (ec / r + k2 * a * exp(-ar * ar)) / r2;
  double ss = 0.0;
  if (lam > 0.0) {
    const double x = r / lam, ex = exp(-2.0 * x);
    ss = -(1.0 + x) * ex / r;
    ff -= (1.0 + 2.0 * x + 2.0 * x * x) * ex / (r2 * r);
  }
  *u = uu + ss;
  *us = ss;
  *f = ff;
  return true;
}

__device__ inline bool cell_offset_valid(int o, int n) {
  return n >= 3 || (n == 2 && o >= 0) || (n == 1 && o == 0);
}

// One wavefront per charge j.  Scan: lanes 0..53 take one of the 27
// neighbour cells and every other slot in it, test each candidate in FP32
// (the slot's FP32 position copy, with a margin that covers its rounding) and
// append those that pass to a wavefront queue in LDS (cell slot, compact
// index).  Evaluation: the whole wavefront takes the queued candidates 64 at
// a time, so the exact FP64 test (minimum image, r < r_cut) and the erfc /
// Slater terms run with full lanes however the pairs are spread over the
// cells; the pairs and displacements are exactly those of an all-FP64 scan.
// The wavefront sums the forces of all pairs of j (each pair is evaluated
// from both of its charges, so no thread writes another charge's force) and
// the energy of the pairs with k > j, as exact int64 fixed point; the
// energies go to j's own slot (no shared accumulator).
constexpr int kRealThreads = 256;

// (charge j is read again here rather than kept in registers through the scan)
__device__ __forceinline__ void real_flush(int qn, const int *qs, const int *qk, gptr<const double4> cgrid,
                                           gptr<const double4> xq, int j, double L, double invL, double rc2,
                                           double alpha, double lam, long long &fx, long long &fy,
                                           long long &fz, long long &ee, long long &es, int &err) {
  const int lane = threadIdx.x & (kWave - 1);
  const double4 ci = gload(xq + j);
  for (int e = lane; e < qn; e += kWave) {
    // minimum image and r^2 with their fused multiply-adds written out (no
    // contraction left to the compiler, as in real_pair)
#pragma clang fp contract(off)
    const int k = qk[e];
    const double4 cj = gload(cgrid + qs[e]);
    double dx = ci.x - cj.x, dy = ci.y - cj.y, dz = ci.z - cj.z;
    dx = fma(-L, rint(dx * invL), dx);
    dy = fma(-L, rint(dy * invL), dy);
    dz = fma(-L, rint(dz * invL), dz);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (!(r2 < rc2)) continue;  // inside the FP32 margin only
    double u, us, f;
    if (!real_pair(sqrt(r2), alpha, lam, &u, &us, &f)) {
      err = kECoincident;
      continue;
    }
    const double qq = ci.w * cj.w;
    const double g = qq * f;
    if (fabs(g) * sqrt(r2) * kRealFxScale > kFxLimit) err = kEOverflow;
    fx += to_fixed(g * dx, kRealFxScale);
    fy += to_fixed(g * dy, kRealFxScale);
    fz += to_fixed(g * dz, kRealFxScale);
    if (k > j) {
      ee += to_fixed(qq * u, kRealFxScale);
      es += to_fixed(qq * us, kRealFxScale);
    }
  }
}

// Squared radius of the FP32 pre-test: r_cut plus 8 FP32 ulps of the box
// length (the rounding of the positions, of L and of the differences stays
// below 4 ulps of L per component), squared and rounded up.
__device__ __forceinline__ float real_pretest_r2(double rc2, double L) {
  int e;
  frexp(L, &e);  // L < 2^e
  const double rc = sqrt(rc2) + 8.0 * ldexp(1.0, e - 24);
  return (float)(rc * rc * (1.0 + 1.0e-6));
}

// U: candidates per lane and pass (slots s, s + 2, ..., s + 2 (U - 1) of the
// lane's cell), all U loads issued before any is tested.  The queue takes
// U x 64 appends per pass and is flushed at > 64 entries.
template <int U>
__device__ __forceinline__ void
real_body(gptr<const double4> __restrict__ xq, gptr<const int> __restrict__ ccnt,
          gptr<const double4> __restrict__ cgrid, gptr<const float4> __restrict__ cpre, const CellParams &cp,
          double L, double alpha, double rc2, double lam, gptr<DevScalars> sc, gptr<unsigned long long> freal,
          gptr<unsigned long long> ereal, int bid, int nbid) {
  constexpr int kQueue = (U + 1) * kWave;  // queued candidates per wavefront
  __shared__ int s_qs[kRealThreads / kWave][kQueue];  // cell slot
  __shared__ int s_qk[kRealThreads / kWave][kQueue];  // compact index
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  int *qs = s_qs[w], *qk = s_qk[w];
  const int nq = sc->nq;
  const double invL = 1.0 / L;
  const float Lf = (float)L, invLf = 1.0f / Lf, rc2f = real_pretest_r2(rc2, L);
  for (int j = bid * wpb + w; j < nq; j += nbid * wpb) {
    float cxf, cyf, czf;
    int cx, cy, cz;
    {
      const double4 ci = gload(xq + j);
      cxf = (float)ci.x;
      cyf = (float)ci.y;
      czf = (float)ci.z;
      cx = (int)(ci.x * cp.inv_cell);
      cy = (int)(ci.y * cp.inv_cell);
      cz = (int)(ci.z * cp.inv_cell);
    }
    cx = cx < cp.ncell ? cx : cp.ncell - 1;
    cy = cy < cp.ncell ? cy : cp.ncell - 1;
    cz = cz < cp.ncell ? cz : cp.ncell - 1;
    long long fx = 0, fy = 0, fz = 0, ee = 0, es = 0;
    int err = 0;
    int c = -1, cnt = 0, s = lane / 27;
    if (lane < 54) {
      const int o = lane % 27;
      const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
      const int n = cp.ncell;
      if (cell_offset_valid(ox, n) && cell_offset_valid(oy, n) && cell_offset_valid(oz, n)) {
        c = (mod_pos(cx + ox, n) * n + mod_pos(cy + oy, n)) * n + mod_pos(cz + oz, n);
        cnt = ccnt[c];
        cnt = cnt < cp.cap ? cnt : cp.cap;
      }
    }
    const int cbase = (c < 0 ? 0 : c) * cp.cap;
    int qn = 0;  // wavefront-uniform queue length
    // FP32 pre-test of one candidate per lane; those that pass are queued
    auto test = [&](bool live, int sl, const float4 &cj) {
      bool take = false;
      const int k = __float_as_int(cj.w);
      if (live) {
        float dx = cxf - cj.x, dy = cyf - cj.y, dz = czf - cj.z;
        dx -= Lf * rintf(dx * invLf);
        dy -= Lf * rintf(dy * invLf);
        dz -= Lf * rintf(dz * invLf);
        take = (k != j) && (dx * dx + dy * dy + dz * dz < rc2f);
      }
      const unsigned long long m = __ballot(take);
      if (take) {
        const int at = qn + (int)__popcll(m & __lanemask_lt());
        qs[at] = sl;
        qk[at] = k;
      }
      qn += (int)__popcll(m);
    };
    auto flush = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      real_flush(qn, qs, qk, cgrid, xq, j, L, invL, rc2, alpha, lam, fx, fy, fz, ee, es, err);
      __builtin_amdgcn_wave_barrier();
      qn = 0;
    };
    // the sums are fixed point, so the queue order does not change the result
    while (true) {
      bool live[U];
#pragma unroll
      for (int u = 0; u < U; ++u) live[u] = s + 2 * u < cnt;
      if (__ballot(live[0]) == 0ull) break;
      float4 cc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cc[u] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (live[u]) cc[u] = gload(cpre + cbase + s + 2 * u);
#pragma unroll
      for (int u = 0; u < U; ++u) test(live[u], cbase + s + 2 * u, cc[u]);
      s += 2 * U;
      if (qn > kQueue - U * kWave) flush();
    }
    flush();
    if (err) set_status(sc, err);
    fx = wave_sum_ll(fx);
    fy = wave_sum_ll(fy);
    fz = wave_sum_ll(fz);
    ee = wave_sum_ll(ee);
    es = wave_sum_ll(es);
    if (lane == 0) {
      freal[3 * (size_t)j] = (unsigned long long)fx;
      freal[3 * (size_t)j + 1] = (unsigned long long)fy;
      freal[3 * (size_t)j + 2] = (unsigned long long)fz;
      ereal[2 * (size_t)j] = (unsigned long long)ee;
      ereal[2 * (size_t)j + 1] = (unsigned long long)es;
    }
  }
}

// one system: two candidates per lane and pass at the kernel's natural
// 168 VGPRs (3 waves per SIMD)
__global__ void __launch_bounds__(kRealThreads, 3)
k_real(const double4 *__restrict__ xq, const int *__restrict__ ccnt, const double4 *__restrict__ cgrid,
       const float4 *__restrict__ cpre, CellParams cp, double L, double alpha, double rc2, double lam,
       DevScalars *sc, unsigned long long *freal, unsigned long long *ereal) {
  real_body<2>(to_g(xq), to_g(ccnt), to_g(cgrid), to_g(cpre), cp, L, alpha, rc2, lam, to_g(sc), to_g(freal),
               to_g(ereal), blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Charges relevant to plane x0 are those of the 2p mesh x-cells
// x0 - p .. x0 + p - 1; the charges of cell x0 - p + b have the plane at
// stencil offset sx = 2p - 1 - b.  Work items are (charge, stencil row sy) in
// groups of P2pad lanes (2p rounded up to a power of two, so that a group
// never straddles a wavefront); lane sy evaluates the window of offset sy on
// each axis and the group shares them with shuffles.
// ---------------------------------------------------------------------------
// v mod M for -M <= v < 2M (a stencil index next to the mesh): no division.
__device__ __forceinline__ int wrap_once(int v, int M) { return v < 0 ? v + M : (v >= M ? v - M : v); }

__device__ inline int pow2_at_least(int v) {
  int r = 1;
  while (r < v) r <<= 1;
  return r;
}

struct PlaneCharges {
  int *cnt;  // [2p + 1] prefix sums over the 2p x-cells (LDS)
  int *cell; // [2p] x-cell of bin b (LDS)
};

// Fill the LDS prefix sums of the plane's 2p x-cells, kXSub sub-bins each
// (2p kXSub <= blockDim.x entries, one per thread); returns the charge count.
__device__ inline int plane_bins(int x0, int M, int p, gptr<const int> __restrict__ xcnt, int xcap, int *pre,
                                 int *cell) {
  __shared__ int s_ws[kPassThreads / kWave];
  const int NB = 2 * p * kXSub;
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  int n = 0;
  if (t < NB) {
    const int c = mod_pos(x0 - p + t / kXSub, M) * kXSub + t % kXSub;
    n = xcnt[c];
    n = n < xcap ? n : xcap;
    cell[t] = c;
  }
  int x = n;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) s_ws[w] = x;
  __syncthreads();
  int base = 0;
  for (int q = 0; q < w; ++q) base += s_ws[q];
  if (t < NB) pre[t + 1] = base + x;
  if (t == 0) pre[0] = 0;
  __syncthreads();
  return pre[NB];
}

// Offsets of charge e of the plane: its x-cell offset b (0 .. 2p-1) in the
// stencil, and its compact index.
__device__ inline int plane_charge(int e, int P2, const int *pre, const int *cell, gptr<const int> __restrict__ xslot,
                                   int xcap, int *b_out) {
  int lo = 0, hi = P2 * kXSub;  // pre[lo] <= e < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= e) lo = mid; else hi = mid;
  }
  *b_out = lo / kXSub;
  return xslot[(size_t)cell[lo] * xcap + (e - pre[lo])];
}

// Stage in LDS those of the plane's charges e0 .. e0 + cnt - 1 that belong to
// this work-group's share of the plane (compact index j with j mod parts ==
// part): position and charge, compact index and x-bin.  Returns how many.
// The share depends on the charges only, not on the order in which the
// binning stored them, so the partial spectra are reproducible; the staged
// order does not matter (the spread sums exactly, the gather is per charge).
// The loads of all staged charges are in flight together, so the spread and
// gather loops that follow read only LDS.
__device__ inline int stage_plane_charges(int e0, int cnt, int P2, const int *pre, const int *cell,
                                          gptr<const int> __restrict__ xslot, int xcap,
                                          gptr<const double4> __restrict__ xq, int part, int parts, double4 *s_c,
                                          int *s_jb, int *s_n) {
  if (threadIdx.x == 0) *s_n = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    int b;
    const int j = plane_charge(e0 + e, P2, pre, cell, xslot, xcap, &b);
    if (j % parts == part) {
      const int k = atomicAdd(s_n, 1);
      s_c[k] = gload(xq + j);
      s_jb[2 * k] = j;
      s_jb[2 * k + 1] = b;
    }
  }
  __syncthreads();
  return *s_n;
}

// The same staging split in two, for a plane whose charges all fit one stage
// and one per thread: plane_charge_slot issues the load of thread t's compact
// index (charge t of the plane) early; stage_plane_commit appends the charge
// (its record loaded by the caller in between) when it belongs to this
// work-group's share.  *s_n must have been cleared before a barrier.
__device__ inline int plane_charge_slot(int total, int P2, const int *pre, const int *cell,
                                        gptr<const int> __restrict__ xslot, int xcap, int *b_out) {
  if ((int)threadIdx.x >= total) return -1;
  return plane_charge(threadIdx.x, P2, pre, cell, xslot, xcap, b_out);
}
__device__ inline int stage_plane_commit(bool take, int j, int b, const double4 &c, double4 *s_c, int *s_jb,
                                         int *s_n) {
  if (take) {
    const int k = atomicAdd(s_n, 1);
    s_c[k] = c;
    s_jb[2 * k] = j;
    s_jb[2 * k + 1] = b;
  }
  __syncthreads();
  return *s_n;
}

// Mesh cell and fractional offset of one coordinate.
__device__ inline int cell_frac(double x, double m_over_l, int M, double *frac) {
  double t;
  const int c = mesh_cell(x, m_over_l, M, &t);
  *frac = t - (double)c;
  return c;
}

// ---------------------------------------------------------------------------
// Mesh pass 1: spread + z R2C FFT + y FFT for one x-plane.
// The plane is processed in chunks of mp.rows mesh rows (all of it when it
// fits): each chunk is spread into an int64 LDS accumulator, converted to T in
// place, z-transformed and its Kc retained modes moved into the spectrum lines
// Zre/Zim [Kc][Mz], which then take the y FFT.
// LDS: accumulator [rows][Mp] int64, spectrum lines, twiddles, window series.
// ---------------------------------------------------------------------------
__device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

template <typename T>
__device__ __forceinline__ void
recip_fwd_body(gptr<const double4> __restrict__ xq, gptr<const int> __restrict__ xcnt,
               gptr<const int> __restrict__ xslot, gptr<const T> __restrict__ wcoef,
               gptr<const DevScalars> __restrict__ sc, const MeshParams &mp,
               gptr<const typename CplxOf<T>::type> __restrict__ tw, gptr<longlong2> gfx, int x0, int part) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M = mp.M, Mp = mp.Mp, Mz = mp.Mz, Kc = mp.Kc, p = mp.win.p, P2 = 2 * p, D = mp.cheb_deg;
  const int R = mp.rows;
  const int P2pad = pow2_at_least(P2), lg_pad = __builtin_ctz(P2pad);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1);
  const float inv_kc = 1.0f / (float)Kc;

  long long *acc = reinterpret_cast<long long *>(smem);
  T *plane = reinterpret_cast<T *>(smem);
  size_t off = align16((size_t)R * Mp * sizeof(long long));
  T *Zre = reinterpret_cast<T *>(smem + off);
  T *Zim = Zre + (size_t)Kc * Mz;
  off += 2 * (size_t)Kc * Mz * sizeof(T);
  T *twr = reinterpret_cast<T *>(smem + off);
  T *twi = twr + M;
  off += 2 * (size_t)M * sizeof(T);
  // series at an odd stride Ds, so that the 2p offsets read by a wavefront fall in distinct banks
  const int Ds = (D + 1) | 1;
  T *cv = reinterpret_cast<T *>(smem + off);  // [P2][Ds] value series
  off += (size_t)P2 * Ds * sizeof(T);
  int *pre = reinterpret_cast<int *>(smem + off);
  int *bcell = pre + P2 * kXSub + 1;
  off = (off + (size_t)(2 * P2 * kXSub + 1) * sizeof(int) + 31) & ~(size_t)31;
  double4 *s_c = reinterpret_cast<double4 *>(smem + off);  // [stage] staged charges
  int *s_jb = reinterpret_cast<int *>(s_c + mp.stage);      // [stage][2] compact index, x-bin
  int *s_n = s_jb + 2 * mp.stage;                            // staged count

  for (int m = tid; m < M; m += nt) {
    const typename CplxOf<T>::type t = gload(tw + m);
    twr[m] = t.x;
    twi[m] = t.y;
  }
  for (int k = tid; k < P2 * (D + 1); k += nt) cv[(k / (D + 1)) * Ds + k % (D + 1)] = wcoef[k];
  const double scale = sc->scale, inv_scale = sc->inv_scale;
  const int total = plane_bins(x0, M, p, xcnt, mp.xcap, pre, bcell);  // synchronises

  const int gbase = lane & ~(P2pad - 1);
  for (int r0 = 0; r0 < M; r0 += R) {
    const int nr = (M - r0) < R ? (M - r0) : R;
    for (int k = tid; k < nr * Mp; k += nt) acc[k] = 0;
    __syncthreads();
    for (int e0 = 0; e0 < total; e0 += mp.stage) {
    const int cnt = stage_plane_charges(e0, (total - e0) < mp.stage ? (total - e0) : mp.stage, P2, pre, bcell,
                                        xslot, mp.xcap, xq, part, mp.parts, s_c, s_jb, s_n);
    // whole wavefronts iterate together so that the group shuffles see every lane
    const int items = ((cnt * P2pad + kWave - 1) / kWave) * kWave;
    for (int it = tid; it < items; it += nt) {
      const int e = it >> lg_pad, sy = it & (P2pad - 1);
      const bool has = e < cnt;
      bool act = has && sy < P2, in = false;
      T wz = (T)0, wrow = (T)0;
      int row = 0, bz = 0;
      if (has) {
        const int b = s_jb[2 * e + 1];
        const double4 c = s_c[e];
        double fx, fy, fz;
        cell_frac(c.x, mp.m_over_l, M, &fx);
        const int cy = cell_frac(c.y, mp.m_over_l, M, &fy);
        const int cz = cell_frac(c.z, mp.m_over_l, M, &fz);
        if (act) {
          const int sx = P2 - 1 - b;
          const T *const ser[3] = {cv + sy * Ds, cv + sx * Ds, cv + sy * Ds};
          const T arg[3] = {(T)(2.0 * fz - 1.0), (T)(2.0 * fx - 1.0), (T)(2.0 * fy - 1.0)};
          T w3[3];
          clenshaw_n<T, 3>(ser, arg, D, w3);
          wz = w3[0];
          row = wrap_once(cy - p + 1 + sy, M) - r0;
          in = (unsigned)row < (unsigned)nr;
          if (in)
            wrow = (T)c.w * w3[1] * w3[2];
          else
            row = 0;
          bz = cz - p + 1;
        }
      }
      long long *arow = acc + (size_t)row * Mp;
      int col = bz < 0 ? bz + M : bz;
      // eight stencil points at a time, so that their shuffles are in flight together
      for (int sz0 = 0; sz0 < P2; sz0 += 8) {
        T w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = __shfl(wz, gbase + sz0 + u, kWave);
        if (in) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (sz0 + u < P2) {
              const double v = (double)(wrow * w[u]);
              atomicAdd(reinterpret_cast<unsigned long long *>(&arow[col]), (unsigned long long)to_fixed(v, scale));
              col = (col + 1 == M) ? 0 : col + 1;
            }
          }
        }
      }
    }
    __syncthreads();  // before the next batch is staged, and before the conversion
    }

    // fixed point -> T rows (in place; FP32 rows move down in groups)
    if (sizeof(T) == 8) {
      for (int k = tid; k < nr * Mp; k += nt) {
        const long long v = acc[k];
        plane[k] = (T)((double)v * inv_scale);
      }
      __syncthreads();
    } else {
      int G = (4 * nt) / Mp;
      G = G < 1 ? 1 : G;
      for (int g0 = 0; g0 < nr; g0 += G) {
        const int n = ((nr - g0) < G ? (nr - g0) : G) * Mp;
        long long v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = tid + u * nt;
          if (k < n) v[u] = acc[(size_t)g0 * Mp + k];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = tid + u * nt;
          if (k < n) plane[(size_t)g0 * Mp + k] = (T)((double)v[u] * inv_scale);
        }
        __syncthreads();
      }
    }

    // z: rows 2c (real part) and 2c+1 (imaginary part) form complex line c
    lds_fft<T>(plane, plane + Mp, 2 * Mp, nr / 2, mp.fft, twr, twi, false);
    for (int id = tid; id < (nr / 2) * Kc; id += nt) {
      int k;
      const int c = fdivmod(id, Kc, inv_kc, &k), mk = k == 0 ? 0 : M - k;
      const T zr = plane[2 * c * Mp + k], zi = plane[(2 * c + 1) * Mp + k];
      const T mr = plane[2 * c * Mp + mk], mi = plane[(2 * c + 1) * Mp + mk];
      const int y = r0 + 2 * c;
      Zre[k * Mz + y] = (T)0.5 * (zr + mr);
      Zim[k * Mz + y] = (T)0.5 * (zi - mi);
      Zre[k * Mz + y + 1] = (T)0.5 * (zi + mi);
      Zim[k * Mz + y + 1] = (T)0.5 * (mr - zr);
    }
    __syncthreads();
  }
  // y: one complex line per kz
  lds_fft<T>(Zre, Zim, Mz, Kc, mp.fft, twr, twi, false);
  // the partial spectrum in fixed point: the parts of a plane then add exactly,
  // so the sum does not depend on how the charges were shared out
  const int nky = mp.nky;
  const double gs = scale * mp.gscale_f;
  gptr<longlong2> dst = gfx + ((size_t)part * M + x0) * nky * Kc;
  for (int id = tid; id < nky * Kc; id += nt) {
    int kz;
    const int kyi = fdivmod(id, Kc, inv_kc, &kz);
    const int m = mod_pos(kyi - (Kc - 1), M);
    gstore(dst + id, make_longlong2(to_fixed((double)Zre[kz * Mz + m], gs), to_fixed((double)Zim[kz * Mz + m], gs)));
  }
}

template <typename T>
__global__ void __launch_bounds__(kPassThreads)
k_recip_fwd(const double4 *__restrict__ xq, const int *__restrict__ xcnt, const int *__restrict__ xslot,
            const T *__restrict__ wcoef, const DevScalars *__restrict__ sc, MeshParams mp,
            const typename CplxOf<T>::type *__restrict__ tw, longlong2 *gfx) {
  recip_fwd_body<T>(to_g(xq), to_g(xcnt), to_g(xslot), to_g(wcoef), to_g(sc), mp, to_g(tw), to_g(gfx),
                    blockIdx.x % mp.M, blockIdx.x / mp.M);
}

// ---------------------------------------------------------------------------
// Mesh pass 2: x FFT, influence multiply + energy, inverse x FFT for one ky.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void
recip_x_body(const MeshParams &mp, gptr<const double> __restrict__ atab,
             gptr<const typename CplxOf<T>::type> __restrict__ tw, gptr<const DevScalars> __restrict__ sc,
             gptr<const longlong2> __restrict__ gfx, gptr<typename CplxOf<T>::type> gzy,
             gptr<typename CplxOf<T>::type> gzx, gptr<double> epart, int blk) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M = mp.M, Mz = mp.Mz, Kc = mp.Kc, nky = mp.nky;
  const int tid = threadIdx.x, nt = blockDim.x;
  // ky row and this work-group's range of kz lines
  const int kyi = blk % nky, xs = blk / nky;
  const int kz_lo = (int)((long long)Kc * xs / mp.xsplit), kz_hi = (int)((long long)Kc * (xs + 1) / mp.xsplit);
  const int ky = kyi - (Kc - 1);
  const int nset = mp.ik ? 2 : 1;  // ik: also i kx h, for the x component of the field
  T *Xre = reinterpret_cast<T *>(smem);  // [nset Kc][Mz]: lines of h, then of i kx h
  T *Xim = Xre + (size_t)nset * Kc * Mz;
  T *twr = Xim + (size_t)nset * Kc * Mz;
  T *twi = twr + M;
  const size_t red_off = ((2 * (size_t)nset * Kc * Mz + 2 * (size_t)M) * sizeof(T) + 15) & ~(size_t)15;
  double *at = reinterpret_cast<double *>(smem + red_off);  // [nky] influence table

  int nkz = 0;  // lines kz < nkz hold modes of the sphere
  while (nkz < Kc && nkz * nkz + ky * ky < Kc * Kc) ++nkz;
  const int l1 = nkz < kz_hi ? nkz : kz_hi;
  const int nl = l1 > kz_lo ? l1 - kz_lo : 0;  // transformed lines of this work-group
  const int nw = kz_hi - kz_lo;                 // stored lines (zero beyond nkz)
  const float inv_nl = 1.0f / (float)(nl > 0 ? nl : 1),
              inv_nw = 1.0f / (float)(nw > 0 ? nw : 1);

  for (int m = tid; m < M; m += nt) {
    const typename CplxOf<T>::type t = gload(tw + m);
    twr[m] = t.x;
    twi[m] = t.y;
  }
  for (int k = tid; k < nky; k += nt) at[k] = atab[k];
  // sum of the plane parts' fixed-point spectra (exact), then back to T
  const double ig = sc->inv_scale / mp.gscale_f;
  const size_t pstride = (size_t)M * nky * Kc;
  for (int id = tid; id < M * nl; id += nt) {
    int kz;
    const int x = fdivmod(id, nl, inv_nl, &kz);
    kz += kz_lo;
    const size_t at0 = ((size_t)x * nky + kyi) * Kc + kz;
    long long vr = 0, vi = 0;
    for (int pt = 0; pt < mp.parts; ++pt) {
      const longlong2 v = gload(gfx + pt * pstride + at0);
      vr += v.x;
      vi += v.y;
    }
    Xre[kz * Mz + x] = (T)((double)vr * ig);
    Xim[kz * Mz + x] = (T)((double)vi * ig);
  }
  __syncthreads();
  lds_fft<T>(Xre + (size_t)kz_lo * Mz, Xim + (size_t)kz_lo * Mz, Mz, nl, mp.fft, twr, twi, false);

  const double ay = at[kyi];
  // A wavefront per kz line: the energy of the line is the sum of its runs of
  // 64 modes (each a wavefront sum) in order, stored per line, so the total
  // does not depend on the work-group size or on how lines are grouped into
  // work-groups.  Stored lines past the sphere hold zero.
  const int lane = tid & (kWave - 1), wv = tid / kWave, nwv = nt / kWave;
  for (int l = wv; l < nw; l += nwv) {
    const int kz = kz_lo + l;
    double el = 0.0;
    for (int m0 = 0; l < nl && m0 < M; m0 += kWave) {
      const int m = m0 + lane;
      double e = 0.0;
      if (m < M) {
      const int kx = m < M / 2 ? m : m - M;
      const int k2 = kx * kx + ky * ky + kz * kz;
      T hr = (T)0, hi = (T)0;
      if (kx > -Kc && kx < Kc && k2 < Kc * Kc && k2 > 0) {
        const double c = at[kx + Kc - 1] * ay * at[kz + Kc - 1] / (double)k2;
        const double gr = (double)Xre[kz * Mz + m], gi = (double)Xim[kz * Mz + m];
        e = (kz > 0 ? 2.0 : 1.0) * c * (gr * gr + gi * gi);
        hr = (T)(c * gr);
        hi = (T)(c * gi);
      }
      Xre[kz * Mz + m] = hr;
      Xim[kz * Mz + m] = hi;
      if (nset == 2) {  // i kx (hr + i hi)
        Xre[(Kc + kz) * Mz + m] = -(T)kx * hi;
        Xim[(Kc + kz) * Mz + m] = (T)kx * hr;
      }
      }
      el += wave_sum(e);
    }
    if (lane == 0) epart[(size_t)kyi * Kc + kz] = el;
  }
  __syncthreads();
  for (int set = 0; set < nset; ++set) {
    T *re = Xre + (size_t)set * Kc * Mz, *im = Xim + (size_t)set * Kc * Mz;
    lds_fft<T>(re + (size_t)kz_lo * Mz, im + (size_t)kz_lo * Mz, Mz, nl, mp.fft, twr, twi, true);
    gptr<typename CplxOf<T>::type> dst = set == 0 ? gzy : gzx;
    for (int id = tid; id < M * nw; id += nt) {
      int kz;
      const int x = fdivmod(id, nw, inv_nw, &kz);
      kz += kz_lo;
      typename CplxOf<T>::type v;
      v.x = kz < nkz ? re[kz * Mz + x] : (T)0;
      v.y = kz < nkz ? im[kz * Mz + x] : (T)0;
      gstore(dst + ((size_t)x * nky + kyi) * Kc + kz, v);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kPassThreads)
k_recip_x(MeshParams mp, const double *__restrict__ atab,
          const typename CplxOf<T>::type *__restrict__ tw, const DevScalars *__restrict__ sc,
          const longlong2 *__restrict__ gfx, typename CplxOf<T>::type *gzy, typename CplxOf<T>::type *gzx,
          double *epart) {
  recip_x_body<T>(mp, to_g(atab), to_g(tw), to_g(sc), to_g(gfx), to_g(gzy), to_g(gzx), to_g(epart), blockIdx.x);
}

// ---------------------------------------------------------------------------
// Mesh pass 3: inverse y FFT, complex-to-real z FFT and gather for one plane.
// Each lane of a work-item group sums its mesh row against the z window and
// its derivative (shared across the group); the group reduces with shuffles.
// ---------------------------------------------------------------------------
template <typename T, bool IK>
__device__ __forceinline__ void
recip_bwd_body(gptr<const double4> __restrict__ xq, gptr<const int> __restrict__ xcnt,
               gptr<const int> __restrict__ xslot, gptr<const T> __restrict__ wcoef,
               gptr<const DevScalars> __restrict__ sc, const MeshParams &mp,
               gptr<const typename CplxOf<T>::type> __restrict__ tw,
               gptr<const typename CplxOf<T>::type> __restrict__ gzy,
               gptr<const typename CplxOf<T>::type> __restrict__ gzx, gptr<double4> part, int x0, int wpart) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M = mp.M, Mp = mp.Mp, Mz = mp.Mz, Kc = mp.Kc, nky = mp.nky, p = mp.win.p, P2 = 2 * p;
  const int D = mp.cheb_deg, R = mp.rows, nslot = mp.nslot;
  const int P2pad = pow2_at_least(P2), lg_pad = __builtin_ctz(P2pad);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1);
  const float inv_kc = 1.0f / (float)Kc, inv_m = 1.0f / (float)M;

  T *plane = reinterpret_cast<T *>(smem);  // [rows][Mp]
  size_t off = align16((size_t)R * Mp * sizeof(T));
  T *Zre = reinterpret_cast<T *>(smem + off);
  T *Zim = Zre + (size_t)Kc * Mz;
  off += 2 * (size_t)Kc * Mz * sizeof(T);
  T *twr = reinterpret_cast<T *>(smem + off);
  T *twi = twr + M;
  off += 2 * (size_t)M * sizeof(T);
  // series at an odd stride Ds, so that the 2p offsets read by a wavefront fall in distinct banks
  const int Ds = (D + 1) | 1;
  T *cv = reinterpret_cast<T *>(smem + off);  // [P2][Ds] value series
  T *cd = cv + (size_t)P2 * Ds;               // [P2][Ds] derivative series
  off += (size_t)P2 * 2 * Ds * sizeof(T);
  int *pre = reinterpret_cast<int *>(smem + off);
  int *bcell = pre + P2 * kXSub + 1;
  off = (off + (size_t)(2 * P2 * kXSub + 1) * sizeof(int) + 31) & ~(size_t)31;
  double4 *s_c = reinterpret_cast<double4 *>(smem + off);  // [stage] staged charges
  int *s_jb = reinterpret_cast<int *>(s_c + mp.stage);      // [stage][2] compact index, x-bin
  int *s_n = s_jb + 2 * mp.stage;                            // staged count

  for (int m = tid; m < M; m += nt) {
    const typename CplxOf<T>::type t = gload(tw + m);
    twr[m] = t.x;
    twi[m] = t.y;
  }
  for (int k = tid; k < 2 * P2 * (D + 1); k += nt) cv[(k / (D + 1)) * Ds + k % (D + 1)] = wcoef[k];
  if (tid == 0) *s_n = 0;
  const int total = plane_bins(x0, M, p, xcnt, mp.xcap, pre, bcell);  // synchronises
  // When the plane's charges fit one stage (one per thread), their loads are
  // issued now and complete under the transforms below.
  const bool early = total <= mp.stage && total <= nt;
  int ej = -1, eb = 0;
  double4 ec = make_double4(0.0, 0.0, 0.0, 0.0);
  if (early) ej = plane_charge_slot(total, P2, pre, bcell, xslot, mp.xcap, &eb);
  bool staged = false;
  int nstaged = 0;
  const int gbase = lane & ~(P2pad - 1);
  // Gradient forces: one field h, gathered with the window and its gradient.
  // ik forces (eq. 24-25): the three fields i k_t h, gathered with the window.
  constexpr int ncomp = IK ? 3 : 1;
#pragma unroll 1
  for (int comp = 0; comp < ncomp; ++comp) {
    for (int k = tid; k < 2 * Kc * Mz; k += nt) Zre[k] = (T)0;
    __syncthreads();
    gptr<const typename CplxOf<T>::type> src = (IK && comp == 0) ? gzx : gzy;
    for (int id = tid; id < nky * Kc; id += nt) {
      int kz;
      const int kyi = fdivmod(id, Kc, inv_kc, &kz);
      const int m = mod_pos(kyi - (Kc - 1), M);
      typename CplxOf<T>::type v = gload(src + ((size_t)x0 * nky + kyi) * Kc + kz);
      if (IK && comp > 0) {  // times i ky or i kz
        const T k = (T)(comp == 1 ? kyi - (Kc - 1) : kz);
        const T re = -k * v.y, im = k * v.x;
        v.x = re;
        v.y = im;
      }
      Zre[kz * Mz + m] = v.x;
      Zim[kz * Mz + m] = v.y;
    }
    if (early && comp == 0 && ej >= 0 && ej % mp.bparts == wpart) ec = gload(xq + ej);
    __syncthreads();
    lds_fft<T>(Zre, Zim, Mz, Kc, mp.fft, twr, twi, true);

    for (int r0 = 0; r0 < M; r0 += R) {
      const int nr = (M - r0) < R ? (M - r0) : R;
      // Hermitian z spectra of rows r0 + 2c and r0 + 2c + 1 packed as H1 + i H2
      for (int id = tid; id < (nr / 2) * M; id += nt) {
        int k;
        const int c = fdivmod(id, M, inv_m, &k), y = r0 + 2 * c;
        T re = (T)0, im = (T)0;
        if (k < Kc) {
          const T h1r = Zre[k * Mz + y], h1i = Zim[k * Mz + y];
          const T h2r = Zre[k * Mz + y + 1], h2i = Zim[k * Mz + y + 1];
          if (k == 0) {
            re = h1r;
            im = h2r;
          } else {
            re = h1r - h2i;
            im = h1i + h2r;
          }
        } else if (k > M - Kc) {
          const int kk = M - k;
          const T h1r = Zre[kk * Mz + y], h1i = Zim[kk * Mz + y];
          const T h2r = Zre[kk * Mz + y + 1], h2i = Zim[kk * Mz + y + 1];
          re = h1r + h2i;
          im = h2r - h1i;
        }
        plane[2 * c * Mp + k] = re;
        plane[(2 * c + 1) * Mp + k] = im;
      }
      __syncthreads();
      lds_fft<T>(plane, plane + Mp, 2 * Mp, nr / 2, mp.fft, twr, twi, true);

      const int chunk = r0 / R;
      for (int e0 = 0; e0 < total; e0 += mp.stage) {
      if (early && !staged) {
        nstaged = stage_plane_commit(ej >= 0 && ej % mp.bparts == wpart, ej, eb, ec, s_c, s_jb, s_n);
        staged = true;
      }
      const int cnt = early ? nstaged
                            : stage_plane_charges(e0, (total - e0) < mp.stage ? (total - e0) : mp.stage, P2, pre,
                                                  bcell, xslot, mp.xcap, xq, wpart, mp.bparts, s_c, s_jb, s_n);
      const int items = ((cnt * P2pad + kWave - 1) / kWave) * kWave;
      for (int it = tid; it < items; it += nt) {
        const int e = it >> lg_pad, sy = it & (P2pad - 1);
        const bool has = e < cnt, act = has && sy < P2;
        bool in = false;
        int j = 0, sx = 0, row = 0, bz = 0, cy = 0;
        T wz = (T)0, dwz = (T)0, wy = (T)0, dwy = (T)0, wx = (T)0, dwx = (T)0;
        if (has) {
          j = s_jb[2 * e];
          sx = P2 - 1 - s_jb[2 * e + 1];
          const double4 c = s_c[e];
          double fx, fy, fz;
          cell_frac(c.x, mp.m_over_l, M, &fx);
          cy = cell_frac(c.y, mp.m_over_l, M, &fy);
          const int cz = cell_frac(c.z, mp.m_over_l, M, &fz);
          if (act) {
            const T ux = (T)(2.0 * fx - 1.0), uy = (T)(2.0 * fy - 1.0), uz = (T)(2.0 * fz - 1.0);
            if (IK) {
              const T *const ser[3] = {cv + sy * Ds, cv + sx * Ds, cv + sy * Ds};
              const T arg[3] = {uz, ux, uy};
              T o[3];
              clenshaw_n<T, 3>(ser, arg, D, o);
              wz = o[0];
              wx = o[1];
              wy = o[2];
            } else {
              const T *const ser[6] = {cv + sy * Ds, cd + sy * Ds, cv + sx * Ds,
                                       cd + sx * Ds, cv + sy * Ds, cd + sy * Ds};
              const T arg[6] = {uz, uz, ux, ux, uy, uy};
              T o[6];
              clenshaw_n<T, 6>(ser, arg, D, o);
              wz = o[0];
              dwz = o[1];
              wx = o[2];
              dwx = o[3];
              wy = o[4];
              dwy = o[5];
            }
            row = wrap_once(cy - p + 1 + sy, M) - r0;
            in = (unsigned)row < (unsigned)nr;
            if (!in) {
              row = 0;
              wy = (T)0;
              dwy = (T)0;
            }
            bz = cz - p + 1;
          }
        }
        const T *hrow = plane + (size_t)row * Mp;
        int col = bz < 0 ? bz + M : bz;
        T a = (T)0, bsum = (T)0;
        // eight stencil points at a time: shuffles and row loads in flight together
        for (int sz0 = 0; sz0 < P2; sz0 += 8) {
          T w[8], d[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            w[u] = __shfl(wz, gbase + sz0 + u, kWave);
            d[u] = IK ? (T)0 : __shfl(dwz, gbase + sz0 + u, kWave);
          }
          if (in) {
            T h[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int c = col + u;
              h[u] = sz0 + u < P2 ? hrow[c >= M ? c - M : c] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (sz0 + u < P2) {
                a += h[u] * w[u];
                bsum += h[u] * d[u];
              }
            }
            col += 8;
            col = col >= M ? col - M : col;
          }
        }
        T A = wy * a, By = dwy * a, Bz = wy * bsum;
        for (int o = P2pad / 2; o >= 1; o >>= 1) {
          A += __shfl_xor(A, o, kWave);
          By += __shfl_xor(By, o, kWave);
          Bz += __shfl_xor(Bz, o, kWave);
        }
        if (has && sy == 0) {
          // the chunk of the charge's first stencil row writes slot 0 (and
          // clears slot 1 when all its rows are in that chunk); the chunk of
          // its last row writes slot 1
          int slot = 0;
          bool write = true, clear1 = false;
          if (nslot > 1) {
            const int first = mod_pos(cy - p + 1, M) / R, last = mod_pos(cy + p, M) / R;
            write = chunk == first || chunk == last;
            slot = chunk == first ? 0 : 1;
            clear1 = chunk == first && first == last;
          }
          if (write) {
            const gptr<double4> dst = part + ((size_t)j * P2 + sx) * nslot;
            if (!IK) {
              gstore(dst + slot, make_double4((double)(dwx * A), (double)(wx * By), (double)(wx * Bz),
                                              (double)(wx * A)));
              if (clear1) gstore(dst + 1, make_double4(0.0, 0.0, 0.0, 0.0));
            } else {
              // component comp of the field; the potential entry stays zero
              const gptr<double> d = (gptr<double>)(dst + slot);
              d[comp] = (double)(wx * A);
              if (comp == 0) d[3] = 0.0;
              if (clear1) {
                const gptr<double> d1 = (gptr<double>)(dst + 1);
                d1[comp] = 0.0;
                if (comp == 0) d1[3] = 0.0;
              }
            }
          }
        }
      }
      if (!early) __syncthreads();  // the next batch restages the charges
      }
      __syncthreads();  // the next chunk overwrites the plane
    }
  }
}

template <typename T, bool IK>
__global__ void __launch_bounds__(kPassThreads)
k_recip_bwd(const double4 *__restrict__ xq, const int *__restrict__ xcnt, const int *__restrict__ xslot,
            const T *__restrict__ wcoef, const DevScalars *__restrict__ sc, MeshParams mp,
            const typename CplxOf<T>::type *__restrict__ tw,
            const typename CplxOf<T>::type *__restrict__ gzy, const typename CplxOf<T>::type *__restrict__ gzx,
            double4 *part) {
  recip_bwd_body<T, IK>(to_g(xq), to_g(xcnt), to_g(xslot), to_g(wcoef), to_g(sc), mp, to_g(tw), to_g(gzy),
                        to_g(gzx), to_g(part), blockIdx.x % mp.M, blockIdx.x / mp.M);
}

// ---------------------------------------------------------------------------
// Combine: forces per particle and per-block energy partials.
// ---------------------------------------------------------------------------
// Final energies of one evaluation from the per-block partials of the combine
// kernel and the k-space sums per (ky, kz) line (one block; a separate launch, so the
// partials of every combine block are visible without a device-wide fence).
__device__ __forceinline__ void finish_body(int nblk, const double *__restrict__ blk_eg,
                                            const long long *__restrict__ blk_er,
                                            const double *__restrict__ epart, int nlines,
                                            const DevScalars *__restrict__ sc, double alpha, double inv2piL,
                                            double *energy, double *energy5, unsigned long long *step) {
  __shared__ double s_dbl[kPrepThreads / kWave];
  __shared__ long long s_ll[kPrepThreads / kWave];
  const int tid = threadIdx.x;
  double g = 0.0, k = 0.0;
  long long tr = 0, ts = 0;
  for (int b = tid; b < nblk; b += blockDim.x) {
    g += blk_eg[b];
    tr += blk_er[2 * b];
    ts += blk_er[2 * b + 1];
  }
  for (int b = tid; b < nlines; b += blockDim.x) k += epart[b];
  g = block_sum(g, s_dbl);
  k = block_sum(k, s_dbl);
  tr = block_sum_ll(tr, s_ll);
  ts = block_sum_ll(ts, s_ll);
  if (tid == 0) {
    const double e_real = (double)tr * kRealFxInv;
    const double e_sl = (double)ts * kRealFxInv;
    const double e_rec = k * inv2piL;
    const double e_self = -alpha * 0.56418958354775628695 * sc->sum_q2;  // 1/sqrt(pi)
    if (energy) energy[0] = e_real + e_rec + e_self;
    if (energy5) {
      energy5[0] = e_real;
      energy5[1] = e_sl;
      energy5[2] = e_rec;
      energy5[3] = e_self;
      energy5[4] = g * inv2piL;
    }
    if (step) step[0] += 1ull;
  }
}

__global__ void __launch_bounds__(kPrepThreads)
k_finish(int nblk, const double *__restrict__ blk_eg, const long long *__restrict__ blk_er,
         const double *__restrict__ epart, int nlines, const DevScalars *__restrict__ sc, double alpha,
         double inv2piL, double *energy, double *energy5) {
  finish_body(nblk, blk_eg, blk_er, epart, nlines, sc, alpha, inv2piL, energy, energy5, nullptr);
}

__global__ void __launch_bounds__(kPrepThreads)
k_combine(int64_t N, const int *__restrict__ slot, const double4 *__restrict__ xq,
          const unsigned long long *freal, const double4 *__restrict__ part, int P2S, double fscale, int nblk,
          double *blk_eg, const unsigned long long *__restrict__ ereal, long long *blk_er, int *ccnt, int ncell3,
          int *xcnt, int M, FinishArgs fa, double *forces) {
  combine_body(N, to_g(slot), to_g(xq), to_g(freal), to_g(part), P2S, fscale, nblk, blk_eg, to_g(ereal), blk_er,
               ccnt, ncell3, xcnt, M, fa, forces, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Batched kernels: one launch covers every member of a batch; block b works
// on block map[b].y of member map[b].x with that member's geometry and buffers.
// ---------------------------------------------------------------------------
// batches (dense members, many passes per charge): four candidates per lane
// and pass, held to 3 waves per SIMD (4.2 % less batch step time than two
// candidates; one system alone ran 0.6 us slower with four)
__global__ void __launch_bounds__(kRealThreads, 3)
kb_real(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  real_body<4>(to_g(m.buf.xq), to_g(m.buf.ccnt), to_g(m.buf.cgrid), to_g(m.buf.cpre), m.cfg.cells, m.cfg.L,
               m.cfg.alpha, m.cfg.r_cut * m.cfg.r_cut, m.cfg.lambda, to_g(m.buf.sc), to_g(m.buf.freal),
               to_g(m.buf.ereal), w.y, m.real_blocks);
}

template <typename T> struct MemberTables;
template <> struct MemberTables<double> {
  static __device__ const double *wcoef(const ComputeBuffers &b) { return b.wcoef64; }
  static __device__ const double2 *tw(const ComputeBuffers &b) { return b.tw64; }
};
template <> struct MemberTables<float> {
  static __device__ const float *wcoef(const ComputeBuffers &b) { return b.wcoef32; }
  static __device__ const float2 *tw(const ComputeBuffers &b) { return b.tw32; }
};

template <typename T>
__global__ void __launch_bounds__(kPassThreads)
kb_recip_fwd(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  recip_fwd_body<T>(to_g(m.buf.xq), to_g(m.buf.xcnt), to_g(m.buf.xslot), to_g(MemberTables<T>::wcoef(m.buf)),
                    to_g(m.buf.sc), m.cfg.mesh, to_g(MemberTables<T>::tw(m.buf)),
                    to_g(reinterpret_cast<longlong2 *>(m.buf.gzy)), w.y % m.cfg.mesh.M, w.y / m.cfg.mesh.M);
}

template <typename T>
__global__ void __launch_bounds__(kPassThreads)
kb_recip_x(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  using C = typename CplxOf<T>::type;
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  recip_x_body<T>(m.cfg.mesh, to_g(m.buf.atab), to_g(MemberTables<T>::tw(m.buf)), to_g(m.buf.sc),
                  to_g(reinterpret_cast<const longlong2 *>(m.buf.gzy)),
                  to_g(reinterpret_cast<C *>((char *)m.buf.gzy + spectrum_h_offset(m.cfg.mesh))),
                  to_g(reinterpret_cast<C *>(m.buf.gzx)), to_g(m.buf.epart), w.y);
}

template <typename T, bool IK>
__global__ void __launch_bounds__(kPassThreads)
kb_recip_bwd(const BatchMember *__restrict__ mem, const int2 *__restrict__ map) {
  using C = typename CplxOf<T>::type;
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  recip_bwd_body<T, IK>(to_g(m.buf.xq), to_g(m.buf.xcnt), to_g(m.buf.xslot), to_g(MemberTables<T>::wcoef(m.buf)),
                    to_g(m.buf.sc), m.cfg.mesh, to_g(MemberTables<T>::tw(m.buf)),
                    to_g(reinterpret_cast<const C *>((const char *)m.buf.gzy + spectrum_h_offset(m.cfg.mesh))),
                    to_g(reinterpret_cast<const C *>(m.buf.gzx)), to_g(m.buf.part), w.y % m.cfg.mesh.M,
                    w.y / m.cfg.mesh.M);
}

__global__ void __launch_bounds__(kPrepThreads)
kb_combine(const BatchMember *__restrict__ mem, const int2 *__restrict__ map, int mode) {
  const int2 w = map[blockIdx.x];
  const BatchMember &m = mem[w.x];
  FinishArgs fa;
  fa.mode = mode;
  fa.kappa = m.P.kappa;
  fa.dt = m.P.dt;
  fa.fdpd = m.fdpd;
  fa.vel = m.vel;
  fa.dcnt = m.dcnt;
  fa.ndcell3 = m.P.ncell * m.P.ncell * m.P.ncell;
  const int nc = m.cfg.cells.ncell;
  combine_body(m.N, to_g(m.buf.slot), to_g(m.buf.xq), to_g(m.buf.freal), to_g(m.buf.part),
               2 * m.cfg.mesh.win.p * m.cfg.mesh.nslot, m.fscale, m.nblk, m.buf.blk_eg, to_g(m.buf.ereal),
               m.buf.blk_er, m.buf.ccnt, nc * nc * nc, m.buf.xcnt, m.cfg.mesh.M * kXSub, fa, m.force, w.y);
}

__global__ void __launch_bounds__(kPrepThreads)
kb_finish(const BatchMember *__restrict__ mem, int mode) {
  const BatchMember &m = mem[blockIdx.x];
  finish_body(m.nblk, m.buf.blk_eg, m.buf.blk_er, m.buf.epart, m.cfg.mesh.nky * m.cfg.mesh.Kc, m.buf.sc,
              m.cfg.alpha, m.inv2piL,
              nullptr, m.e5, mode == 0 ? m.step : nullptr);
}

hipError_t launch_batch_real(const BatchMember *mem, const int2 *map, int nmap, hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_real, dim3(nmap), dim3(kRealThreads), 0, st, mem, map);
  return hipGetLastError();
}

template <typename T>
static void launch_batch_mesh(const BatchMember *mem, int ik, const int2 *fwd, int nfwd, const int2 *x, int nx,
                              const int2 *bwd, int nbwd, size_t lds_fwd, size_t lds_x, size_t lds_bwd, int tp,
                              int tx, hipStream_t st, KernelTimer *tm) {
  if (tm) tm->before(5, st);
  if (nfwd > 0) hipLaunchKernelGGL(kb_recip_fwd<T>, dim3(nfwd), dim3(tp), lds_fwd, st, mem, fwd);
  if (tm) tm->after(5, st);
  if (tm) tm->before(6, st);
  if (nx > 0) hipLaunchKernelGGL(kb_recip_x<T>, dim3(nx), dim3(tx), lds_x, st, mem, x);
  if (tm) tm->after(6, st);
  if (tm) tm->before(7, st);
  if (nbwd > 0) {
    if (ik)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(kb_recip_bwd<T, true>), dim3(nbwd), dim3(tp), lds_bwd, st, mem, bwd);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(kb_recip_bwd<T, false>), dim3(nbwd), dim3(tp), lds_bwd, st, mem, bwd);
  }
  if (tm) tm->after(7, st);
}

hipError_t launch_batch_recip(const BatchMember *mem, int precision, int ik, const int2 *fwd, int nfwd,
                              const int2 *x, int nx, const int2 *bwd, int nbwd, size_t lds_fwd, size_t lds_x,
                              size_t lds_bwd, int pass_threads, int x_threads, hipStream_t st, KernelTimer *tm) {
  if (pass_threads < 1 || pass_threads > kPassThreads || x_threads < 1 || x_threads > kPassThreads)
    return hipErrorInvalidValue;
  if (precision == 0)
    launch_batch_mesh<double>(mem, ik, fwd, nfwd, x, nx, bwd, nbwd, lds_fwd, lds_x, lds_bwd, pass_threads,
                              x_threads, st, tm);
  else
    launch_batch_mesh<float>(mem, ik, fwd, nfwd, x, nx, bwd, nbwd, lds_fwd, lds_x, lds_bwd, pass_threads,
                             x_threads, st, tm);
  return hipGetLastError();
}

hipError_t launch_batch_combine(const BatchMember *mem, int nmem, const int2 *map, int nmap, int mode,
                                hipStream_t st) {
  if (nmap > 0) hipLaunchKernelGGL(kb_combine, dim3(nmap), dim3(kPrepThreads), 0, st, mem, map, mode);
  if (nmem > 0) hipLaunchKernelGGL(kb_finish, dim3(nmem), dim3(kPrepThreads), 0, st, mem, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
void mesh_lds_bytes(const MeshParams &m, int precision, size_t *fwd, size_t *x, size_t *bwd) {
  const size_t ts = precision == 0 ? sizeof(double) : sizeof(float);
  const int P2 = 2 * m.win.p;
  const size_t misc = (size_t)P2 * 2 * ((m.cheb_deg + 1) | 1) * ts + (2 * (size_t)P2 * kXSub + P2 + 2) * sizeof(int) + 32 +
                      (size_t)m.stage * (sizeof(double4) + 2 * sizeof(int)) + 48;
  const size_t a16 = 15;
  const size_t acc = ((size_t)m.rows * m.Mp * sizeof(long long) + a16) & ~a16;
  const size_t rows_t = ((size_t)m.rows * m.Mp * ts + a16) & ~a16;
  const size_t zp = 2 * (size_t)m.Kc * m.Mz * ts;
  const size_t tw = 2 * (size_t)m.M * ts;
  *fwd = acc + zp + tw + misc;
  *x = ((zp * (m.ik ? 2 : 1) + tw + 15) & ~(size_t)15) + (size_t)m.nky * sizeof(double) + 16;
  *bwd = rows_t + zp + tw + misc;
}

bool mesh_choose_rows(MeshParams &m, int precision, size_t max_lds) {
  for (int nchunk = 1; nchunk <= m.M / 2; ++nchunk) {
    int rows = (m.M + nchunk - 1) / nchunk;
    rows += rows & 1;
    if (nchunk > 1 && rows < 2 * m.win.p) return false;
    MeshParams t = m;
    t.rows = rows;
    t.nchunk = (m.M + rows - 1) / rows;
    t.nslot = t.nchunk > 1 ? 2 : 1;
    if (t.nchunk > 1 && m.M - (t.nchunk - 1) * rows < 2 * m.win.p) continue;  // keep every chunk >= 2p rows
    // the largest charge stage that fits beside these rows
    for (int stage = kStage; stage >= 32; stage /= 2) {
      t.stage = stage;
      size_t f, x, b;
      mesh_lds_bytes(t, precision, &f, &x, &b);
      if (x > max_lds) return false;
      if (f <= max_lds && b <= max_lds) {
        m.rows = t.rows;
        m.nchunk = t.nchunk;
        m.nslot = t.nslot;
        m.stage = t.stage;
        return true;
      }
    }
  }
  return false;
}

hipError_t configure_kernels(size_t max_lds) {
  const int v = (int)max_lds;
  hipError_t e;
  e = hipFuncSetAttribute((const void *)k_recip_fwd<double>, hipFuncAttributeMaxDynamicSharedMemorySize, v);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_recip_fwd<float>, hipFuncAttributeMaxDynamicSharedMemorySize, v);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_recip_x<double>, hipFuncAttributeMaxDynamicSharedMemorySize, v);

  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_recip_x<float>, hipFuncAttributeMaxDynamicSharedMemorySize, v);
  if (e != hipSuccess) return e;
  const void *more[] = {(const void *)k_recip_bwd<double, false>,  (const void *)k_recip_bwd<float, false>,
                        (const void *)k_recip_bwd<double, true>,   (const void *)k_recip_bwd<float, true>,
                        (const void *)kb_recip_fwd<double>,        (const void *)kb_recip_fwd<float>,
                        (const void *)kb_recip_x<double>,          (const void *)kb_recip_x<float>,
                        (const void *)kb_recip_bwd<double, false>, (const void *)kb_recip_bwd<float, false>,
                        (const void *)kb_recip_bwd<double, true>,  (const void *)kb_recip_bwd<float, true>};
  const void *const *batched = more;
  for (size_t k = 0; k < sizeof(more) / sizeof(more[0]); ++k) {
    e = hipFuncSetAttribute(batched[k], hipFuncAttributeMaxDynamicSharedMemorySize, v);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
static void launch_mesh(const ComputeConfig &cfg, const ComputeBuffers &b, hipStream_t st, KernelTimer *tm,
                        int x_threads) {
  using C = typename CplxOf<T>::type;
  const C *tw = reinterpret_cast<const C *>(sizeof(T) == 8 ? (const void *)b.tw64 : (const void *)b.tw32);
  const T *wc = reinterpret_cast<const T *>(sizeof(T) == 8 ? (const void *)b.wcoef64 : (const void *)b.wcoef32);
  const MeshParams &mp = cfg.mesh;
  longlong2 *gfx = reinterpret_cast<longlong2 *>(b.gzy);  // partial spectra of the plane parts
  C *gh = reinterpret_cast<C *>((char *)b.gzy + spectrum_h_offset(mp));  // field spectrum
  const int nplane = mp.M * mp.parts;
  if (tm) tm->before(5, st);
  hipLaunchKernelGGL(k_recip_fwd<T>, dim3(nplane), dim3(kPassThreads), cfg.lds_fwd, st, (const double4 *)b.xq,
                     (const int *)b.xcnt, (const int *)b.xslot, wc, (const DevScalars *)b.sc, mp, tw, gfx);
  if (tm) tm->after(5, st);
  if (tm) tm->before(6, st);
  hipLaunchKernelGGL(k_recip_x<T>, dim3(mp.nky * mp.xsplit), dim3(x_threads), cfg.lds_x, st, mp, b.atab, tw,
                     (const DevScalars *)b.sc, (const longlong2 *)gfx, gh, reinterpret_cast<C *>(b.gzx), b.epart);
  if (tm) tm->after(6, st);
  if (tm) tm->before(7, st);
  if (mp.ik)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recip_bwd<T, true>), dim3(mp.M * mp.bparts), dim3(kPassThreads), cfg.lds_bwd, st,
                       (const double4 *)b.xq, (const int *)b.xcnt, (const int *)b.xslot, wc,
                       (const DevScalars *)b.sc, mp, tw, (const C *)gh, (const C *)b.gzx, b.part);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recip_bwd<T, false>), dim3(mp.M * mp.bparts), dim3(kPassThreads), cfg.lds_bwd, st,
                       (const double4 *)b.xq, (const int *)b.xcnt, (const int *)b.xslot, wc,
                       (const DevScalars *)b.sc, mp, tw, (const C *)gh, (const C *)b.gzx, b.part);
  if (tm) tm->after(7, st);
}

hipError_t launch_prep(const ComputeConfig &cfg, const ComputeBuffers &b, const double *pos,
                       const double *q, hipStream_t st, KernelTimer *tm) {
  const int nblk = cfg.nblk;
  const int ncell3 = cfg.cells.ncell * cfg.cells.ncell * cfg.cells.ncell;
  if (tm) tm->before(2, st);
  hipLaunchKernelGGL(k_prep_count, dim3(nblk), dim3(kPrepThreads), 0, st, cfg.N, pos, q, b.blk_cnt, b.blk_sums,
                     b.ccnt, ncell3, b.xcnt, cfg.mesh.M * kXSub, b.sc);
  if (tm) tm->after(2, st);
  if (tm) tm->before(3, st);
  hipLaunchKernelGGL(k_prep_compact, dim3(nblk), dim3(kPrepThreads), 0, st, cfg.N, pos, q, cfg.L, cfg.cells,
                     (const int *)b.blk_cnt, nblk, (const double *)b.blk_sums, b.xq, b.idx, b.slot, b.ccnt,
                     b.cgrid, b.cpre, b.xcnt, b.xslot, cfg.mesh.M, cfg.mesh.m_over_l, cfg.mesh.xcap, b.sc);
  if (tm) tm->after(3, st);
  return hipGetLastError();
}

hipError_t launch_real(const ComputeConfig &cfg, const ComputeBuffers &b, int64_t nq_max, hipStream_t st,
                       KernelTimer *tm) {
  int64_t g = (nq_max + 3) / 4;
  const int grid_real = (int)(g < 1 ? 1 : (g < 2048 ? g : 2048));
  if (tm) tm->before(4, st);
  hipLaunchKernelGGL(k_real, dim3(grid_real), dim3(kRealThreads), 0, st, (const double4 *)b.xq,
                     (const int *)b.ccnt, (const double4 *)b.cgrid, (const float4 *)b.cpre, cfg.cells, cfg.L,
                     cfg.alpha, cfg.r_cut * cfg.r_cut, cfg.lambda, b.sc, b.freal, b.ereal);
  if (tm) tm->after(4, st);
  return hipGetLastError();
}

hipError_t launch_recip(const ComputeConfig &cfg, const ComputeBuffers &b, int64_t nq_max, hipStream_t st,
                        KernelTimer *tm, int x_threads) {
  (void)nq_max;
  // one thread per butterfly of an x line at least (the x pass sums its
  // energy per (ky, kz) line, so the work-group size does not change it)
  int tx = x_threads < kWave ? kWave : (x_threads > kPassThreads ? kPassThreads : x_threads);
  while (tx < fft_max_butterflies(cfg.mesh.fft) && tx < kPassThreads) tx *= 2;
  if (tx > kPassThreads) tx = kPassThreads;
  if (cfg.precision == 0)
    launch_mesh<double>(cfg, b, st, tm, tx);
  else
    launch_mesh<float>(cfg, b, st, tm, tx);
  return hipGetLastError();
}

hipError_t launch_combine(const ComputeConfig &cfg, const ComputeBuffers &b, double *forces,
                          double *energy_total, double *energy5, const FinishArgs &fa, hipStream_t st,
                          KernelTimer *tm) {
  const int nblk = cfg.nblk;
  const int ncell3 = cfg.cells.ncell * cfg.cells.ncell * cfg.cells.ncell;
  const double L = cfg.L;
  const double fscale = combine_fscale(cfg);
  const double inv2piL = 1.0 / (2.0 * M_PI * L);
  const int kid = fa.mode < 0 ? 8 : 9;
  if (tm) tm->before(kid, st);
  hipLaunchKernelGGL(k_combine, dim3(nblk), dim3(kPrepThreads), 0, st, cfg.N, (const int *)b.slot,
                     (const double4 *)b.xq, (const unsigned long long *)b.freal, (const double4 *)b.part,
                     2 * cfg.mesh.win.p * cfg.mesh.nslot, fscale, nblk, b.blk_eg,
                     (const unsigned long long *)b.ereal, b.blk_er, b.ccnt, ncell3, b.xcnt, cfg.mesh.M * kXSub, fa,
                     forces);
  if (fa.energies)
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kPrepThreads), 0, st, nblk, (const double *)b.blk_eg,
                       (const long long *)b.blk_er, (const double *)b.epart, cfg.mesh.nky * cfg.mesh.Kc,
                       (const DevScalars *)b.sc, cfg.alpha, inv2piL, energy_total, energy5);
  if (tm) tm->after(kid, st);
  return hipGetLastError();
}

hipError_t launch_compute(const ComputeConfig &cfg, const ComputeBuffers &b, const double *pos,
                          const double *q, double *forces, double *energy_total, double *energy5,
                          hipStream_t st, KernelTimer *tm) {
  hipError_t e = launch_prep(cfg, b, pos, q, st, tm);
  if (e == hipSuccess) e = launch_real(cfg, b, cfg.N, st, tm);
  if (e == hipSuccess) e = launch_recip(cfg, b, cfg.N, st, tm);
  if (e == hipSuccess) e = launch_combine(cfg, b, forces, energy_total, energy5, FinishArgs(), st, tm);
  return e;
}

}  // namespace enuf
