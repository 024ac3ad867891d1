// enuf_observables.hip -- structure observables sampled on the device during
// a trajectory: the pair-distance histogram by particle class behind the
// radial distribution functions (Sec. 5) and the radius of gyration of
// chains (Sec. 6).  Enqueued on the caller's stream between steps, so that a
// run samples its trajectory without copying it to the host.
#include <hip/hip_runtime.h>

#include <cmath>

#include "enuf_internal.h"

namespace enuf {
namespace {

constexpr int kHistTile = 256;         // selected particles per tile (one per thread)

// Minimum-image component v - L rint(v / L) with no fused multiply-add, so
// that the squared distance (and so the bin) is the one a plain IEEE FP64
// evaluation of the same expression gives.
__device__ __forceinline__ double min_image_nofma(double v, double L) {
#pragma clang fp contract(off)
  return v - L * rint(v / L);
}

__device__ __forceinline__ double dist2_nofma(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double r2 = dx * dx + dy * dy;
  return r2 + dz * dz;
}

__device__ __forceinline__ double edge2(int k, double w) {
#pragma clang fp contract(off)
  const double e = (double)k * w;
  return e * e;
}

// One block per (i tile, j tile) with j tile >= i tile: the j tile's
// positions and classes are staged in LDS, each thread takes one i and walks
// the tile (j > i within the diagonal tile), and counts go to a block-private
// LDS histogram that is added to the global one at the end.  The bin is
// decided on r^2 against the squared bin edges (k w)^2, so it is independent
// of how the square root of the first guess rounds.  Entries whose index or
// class is out of range are skipped.
__global__ void __launch_bounds__(kHistTile)
k_pair_histogram(const double *__restrict__ pos, int64_t n, int64_t nsel, const int64_t *__restrict__ sel,
                 const int *__restrict__ cls, int ncls, double L, double w, int nbins,
                 unsigned long long *__restrict__ hist) {
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj < ti) return;  // whole block leaves before any barrier
  extern __shared__ unsigned int s_hist[];
  __shared__ double s_x[kHistTile], s_y[kHistTile], s_z[kHistTile];
  __shared__ int s_c[kHistTile];
  const int nh = ncls * ncls * nbins;
  for (int k = threadIdx.x; k < nh; k += blockDim.x) s_hist[k] = 0u;
  {
    const int64_t b = (int64_t)tj * kHistTile + threadIdx.x;
    int c = -1;
    double x = 0.0, y = 0.0, z = 0.0;
    if (b < nsel) {
      const int64_t j = sel[b];
      const int cj = cls[b];
      if (j >= 0 && j < n && cj >= 0 && cj < ncls) {
        c = cj;
        x = pos[3 * j];
        y = pos[3 * j + 1];
        z = pos[3 * j + 2];
      }
    }
    s_x[threadIdx.x] = x;
    s_y[threadIdx.x] = y;
    s_z[threadIdx.x] = z;
    s_c[threadIdx.x] = c;
  }
  __syncthreads();
  const int64_t a = (int64_t)ti * kHistTile + threadIdx.x;
  int ci = -1;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (a < nsel) {
    const int64_t i = sel[a];
    const int c = cls[a];
    if (i >= 0 && i < n && c >= 0 && c < ncls) {
      ci = c;
      xi = pos[3 * i];
      yi = pos[3 * i + 1];
      zi = pos[3 * i + 2];
    }
  }
  if (ci >= 0) {
    const double emax = edge2(nbins, w);
    const int j0 = (ti == tj) ? (int)threadIdx.x + 1 : 0;
    for (int jj = j0; jj < kHistTile; ++jj) {
      const int cj = s_c[jj];
      if (cj < 0) continue;
      const double dx = min_image_nofma(s_x[jj] - xi, L);
      const double dy = min_image_nofma(s_y[jj] - yi, L);
      const double dz = min_image_nofma(s_z[jj] - zi, L);
      const double r2 = dist2_nofma(dx, dy, dz);
      if (!(r2 < emax)) continue;
      int k = (int)(sqrt(r2) / w);
      k = k < nbins - 1 ? k : nbins - 1;
      while (k > 0 && edge2(k, w) > r2) --k;
      while (k < nbins - 1 && edge2(k + 1, w) <= r2) ++k;
      const int lo = ci < cj ? ci : cj, hi = ci < cj ? cj : ci;
      atomicAdd(&s_hist[(lo * ncls + hi) * nbins + k], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nh; k += blockDim.x) {
    const unsigned int v = s_hist[k];
    if (v) atomicAdd(&hist[k], (unsigned long long)v);
  }
}

// One thread per chain: unwrap along the bonds by the minimum image of each
// bond vector, then the mean square distance from the chain's centre.  A
// chain with a bead index out of range gets NaN.
__global__ void __launch_bounds__(64)
k_chain_rg2(const double *__restrict__ pos, int64_t n, int nchains, int len, const int64_t *__restrict__ beads,
            double L, double *__restrict__ out) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchains) return;
  const int64_t *bd = beads + (size_t)c * len;
  for (int k = 0; k < len; ++k)
    if (bd[k] < 0 || bd[k] >= n) {
      out[c] = __builtin_nan("");
      return;
    }
  // first pass: centre of the unwrapped chain
  double ux = pos[3 * bd[0]], uy = pos[3 * bd[0] + 1], uz = pos[3 * bd[0] + 2];
  double sx = ux, sy = uy, sz = uz;
  for (int k = 1; k < len; ++k) {
    const int64_t p = bd[k], q = bd[k - 1];
    ux += min_image_nofma(pos[3 * p] - pos[3 * q], L);
    uy += min_image_nofma(pos[3 * p + 1] - pos[3 * q + 1], L);
    uz += min_image_nofma(pos[3 * p + 2] - pos[3 * q + 2], L);
    sx += ux;
    sy += uy;
    sz += uz;
  }
  const double cx = sx / len, cy = sy / len, cz = sz / len;
  // second pass: the same unwrapped positions, squared distances from the centre
  ux = pos[3 * bd[0]];
  uy = pos[3 * bd[0] + 1];
  uz = pos[3 * bd[0] + 2];
  double s = 0.0;
  for (int k = 0; k < len; ++k) {
    if (k > 0) {
      const int64_t p = bd[k], q = bd[k - 1];
      ux += min_image_nofma(pos[3 * p] - pos[3 * q], L);
      uy += min_image_nofma(pos[3 * p + 1] - pos[3 * q + 1], L);
      uz += min_image_nofma(pos[3 * p + 2] - pos[3 * q + 2], L);
    }
    const double vx = ux - cx, vy = uy - cy, vz = uz - cz;
    s += vx * vx;
    s += vy * vy;
    s += vz * vz;
  }
  out[c] = s / len;
}

}  // namespace

hipError_t launch_pair_histogram(const double *pos, int64_t n, int64_t nsel, const int64_t *sel, const int *cls,
                                 int ncls, double box, double r_max, int nbins, unsigned long long *hist,
                                 hipStream_t st) {
  if (nsel < 2) return hipSuccess;
  const int64_t nt = (nsel + kHistTile - 1) / kHistTile;
  const size_t lds = (size_t)ncls * ncls * nbins * sizeof(unsigned int);
  hipLaunchKernelGGL(k_pair_histogram, dim3((unsigned)nt, (unsigned)nt), dim3(kHistTile), lds, st, pos, n, nsel,
                     sel, cls, ncls, box, r_max / nbins, nbins, hist);
  return hipGetLastError();
}

hipError_t launch_chain_rg2(const double *pos, int64_t n, int nchains, int len, const int64_t *beads, double box,
                            double *out, hipStream_t st) {
  if (nchains < 1) return hipSuccess;
  hipLaunchKernelGGL(k_chain_rg2, dim3((nchains + 63) / 64), dim3(64), 0, st, pos, n, nchains, len, beads, box,
                     out);
  return hipGetLastError();
}

}  // namespace enuf
