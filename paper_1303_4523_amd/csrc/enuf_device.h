// enuf_device.h -- device helpers of the ENUF kernels (gfx950): window
// functions, wavefront reductions and the LDS-resident Stockham FFT.
#pragma once

#include "enuf_internal.h"

namespace enuf {

// ---------------------------------------------------------------------------
// Small math helpers
// ---------------------------------------------------------------------------
__device__ inline double dev_exp(double x) { return exp(x); }
__device__ inline float dev_exp(float x) { return expf(x); }
__device__ inline double dev_sqrt(double x) { return sqrt(x); }
__device__ inline float dev_sqrt(float x) { return sqrtf(x); }

__device__ inline int mod_pos(int a, int m) {
  int r = a % m;
  return r < 0 ? r + m : r;
}

// Mesh coordinate t = x * M / L of a wrapped coordinate and its cell floor(t),
// clamped to [0, M-1] (x < L can still round to t == M).  Every kernel derives
// stencil positions through this one function so that they agree exactly.
__device__ inline int mesh_cell(double x, double m_over_l, int M, double *t) {
  double tt = x * m_over_l;
  int c = (int)floor(tt);
  c = c < 0 ? 0 : (c > M - 1 ? M - 1 : c);
  *t = tt;
  return c;
}

// ---------------------------------------------------------------------------
// NFFT window phi(u), |u| <= p, normalised to phi(0) = 1, and its derivative.
//
// Kaiser-Bessel (NFFT literature):  phi(u) = p sinh(b s) / (s sinh(b p)),
// s = sqrt(p^2 - u^2).  With e1 = exp(b (s - p)), e2 = exp(-2 b s):
//   phi  = p e1 (1 - e2) c1 / s,        c1 = 1/(1 - exp(-2 b p)),
//   phi' = -p u e1 c1 [b s (1 + e2) - (1 - e2)] / s^3.
// For b s < 1/2 both closed forms lose digits, so the even power series of
// sinh(z)/z and (z cosh z - sinh z)/z^3 (z = b s) are summed instead.
// Gaussian:  phi(u) = exp(-u^2 / b_G),  phi' = -2 u / b_G phi.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void window_eval(const WindowParams &w, T u, T *val, T *der) {
  if (w.kind == 1) {
    const T ib = (T)w.inv_bg;
    T g = dev_exp(-u * u * ib);
    *val = g;
    *der = (T)(-2) * u * ib * g;
    return;
  }
  const T p = (T)w.p, b = (T)w.b;
  T s2 = p * p - u * u;
  s2 = s2 > (T)0 ? s2 : (T)0;
  const T s = dev_sqrt(s2);
  const T z = b * s;
  if (z >= (T)0.5) {
    const T e1 = dev_exp(b * (s - p));
    const T e2 = dev_exp((T)(-2) * z);
    const T c1 = (T)w.c1;
    *val = p * e1 * ((T)1 - e2) * c1 / s;
    *der = -p * u * e1 * c1 * (z * ((T)1 + e2) - ((T)1 - e2)) / (s2 * s);
  } else {
    // sinh(z)/z = sum z^{2m}/(2m+1)!            (term ratio z^2 / (2m (2m+1)))
    // (z cosh z - sinh z)/z^3 = sum z^{2m} / ((2m+3) (2m+1)!)   (ratio z^2 / (2m (2m+3)))
    const T z2 = z * z;
    T a = (T)1, h = (T)(1.0 / 3.0), ta = (T)1, th = (T)(1.0 / 3.0);
#pragma unroll
    for (int m = 1; m <= 6; ++m) {
      ta *= z2 / (T)((2 * m) * (2 * m + 1));
      a += ta;
      th *= z2 / (T)((2 * m) * (2 * m + 3));
      h += th;
    }
    const T isb = (T)w.inv_sinh_bp;
    *val = p * b * a * isb;
    *der = -p * u * b * b * b * h * isb;
  }
}

// ---------------------------------------------------------------------------
// Wavefront reductions (butterfly over 64 lanes; every lane ends with the sum;
// the order of additions is fixed, so results are reproducible).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline long long to_fixed(double v, double scale) {
  return __double2ll_rn(v * scale);
}

// ---------------------------------------------------------------------------
// Stockham autosort FFT over complex lines held in LDS (split re/im storage).
// Line l, element e lives at re[l * ls + e], im[l * ls + e].  Each pass of
// radix R reads element j + r n/R, applies the twiddle exp(-2 pi i k r/(Ns R))
// with k = j mod Ns, performs an R-point DFT and writes to
// (j / Ns) Ns R + k + r Ns, which leaves the result in natural order after
// the last pass.  Passes are done in place: each thread first loads all of
// its butterflies into registers, the block synchronises, then stores.
// Lines are processed in groups small enough for MaxBfly butterflies per
// thread.  inverse: the unnormalised inverse via conj(FFT(conj(x))).
// All threads of the block must call this function.
// ---------------------------------------------------------------------------
// Butterflies per thread per sweep: bounded so that the register arrays of a
// radix-5 pass stay small.
template <typename T> struct MaxBfly { static constexpr int value = 2; };

template <typename T, int R>
__device__ inline void dft_radix(T *xr, T *xi) {
  if constexpr (R == 2) {
    T ar = xr[0], ai = xi[0];
    xr[0] = ar + xr[1]; xi[0] = ai + xi[1];
    xr[1] = ar - xr[1]; xi[1] = ai - xi[1];
  } else if constexpr (R == 4) {
    T t0r = xr[0] + xr[2], t0i = xi[0] + xi[2];
    T t1r = xr[0] - xr[2], t1i = xi[0] - xi[2];
    T t2r = xr[1] + xr[3], t2i = xi[1] + xi[3];
    // (x1 - x3) * (-i)
    T t3r = xi[1] - xi[3], t3i = xr[3] - xr[1];
    xr[0] = t0r + t2r; xi[0] = t0i + t2i;
    xr[2] = t0r - t2r; xi[2] = t0i - t2i;
    xr[1] = t1r + t3r; xi[1] = t1i + t3i;
    xr[3] = t1r - t3r; xi[3] = t1i - t3i;
  } else if constexpr (R == 3) {
    const T c = (T)(-0.5), s = (T)(-0.86602540378443864676);  // e^{-2 pi i/3}
    T tr = xr[1] + xr[2], ti = xi[1] + xi[2];
    T dr = xr[1] - xr[2], di = xi[1] - xi[2];
    T mr = xr[0] + c * tr, mi = xi[0] + c * ti;
    xr[0] = xr[0] + tr; xi[0] = xi[0] + ti;
    // y1 = m + i s d, y2 = m - i s d  (s < 0 carries the sign of the exponent)
    xr[1] = mr - s * di; xi[1] = mi + s * dr;
    xr[2] = mr + s * di; xi[2] = mi - s * dr;
  } else {  // R == 5
    const T c1 = (T)0.30901699437494742410, c2 = (T)(-0.80901699437494742410);
    const T s1 = (T)(-0.95105651629515357212), s2 = (T)(-0.58778525229247312917);
    T ar = xr[1] + xr[4], ai = xi[1] + xi[4], br = xr[1] - xr[4], bi = xi[1] - xi[4];
    T cr = xr[2] + xr[3], ci = xi[2] + xi[3], dr = xr[2] - xr[3], di = xi[2] - xi[3];
    T x0r = xr[0], x0i = xi[0];
    T m1r = x0r + c1 * ar + c2 * cr, m1i = x0i + c1 * ai + c2 * ci;
    T m2r = x0r + c2 * ar + c1 * cr, m2i = x0i + c2 * ai + c1 * ci;
    // i (s1 b + s2 d) and i (s2 b - s1 d)
    T n1r = -(s1 * bi + s2 * di), n1i = s1 * br + s2 * dr;
    T n2r = -(s2 * bi - s1 * di), n2i = s2 * br - s1 * dr;
    xr[0] = x0r + ar + cr; xi[0] = x0i + ai + ci;
    xr[1] = m1r + n1r; xi[1] = m1i + n1i;
    xr[4] = m1r - n1r; xi[4] = m1i - n1i;
    xr[2] = m2r + n2r; xi[2] = m2i + n2i;
    xr[3] = m2r - n2r; xi[3] = m2i - n2i;
  }
}

// One radix-R pass over `nlines` lines of length n, span Ns before the pass.
template <typename T, int R>
__device__ void stockham_pass(T *re, T *im, int ls, int nlines, int n, int Ns, const T *twr,
                              const T *twi, bool conj_in, bool conj_out) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int nb = n / R;
  const int tstep = n / (Ns * R);
  constexpr int kMaxBfly = MaxBfly<T>::value;
  int lg = (kMaxBfly * nt) / nb;  // whole lines per sweep
  if (lg < 1) lg = 1;
  for (int l0 = 0; l0 < nlines; l0 += lg) {
    const int lines = (nlines - l0) < lg ? (nlines - l0) : lg;
    const int total = lines * nb;
    T vr[kMaxBfly][R], vi[kMaxBfly][R];
#pragma unroll
    for (int q = 0; q < kMaxBfly; ++q) {
      const int id = tid + q * nt;
      if (id < total) {
        const int base = (l0 + id / nb) * ls + id % nb;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          vr[q][r] = re[base + r * nb];
          const T v = im[base + r * nb];
          vi[q][r] = conj_in ? -v : v;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxBfly; ++q) {
      const int id = tid + q * nt;
      if (id < total) {
        const int line = l0 + id / nb, j = id % nb;
        const int k = j % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int ti = k * r * tstep;
          const T wr = twr[ti], wi = twi[ti];
          const T xr = vr[q][r], xi = vi[q][r];
          vr[q][r] = xr * wr - xi * wi;
          vi[q][r] = xr * wi + xi * wr;
        }
        dft_radix<T, R>(vr[q], vi[q]);
        const int ob = line * ls + (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          re[ob + r * Ns] = vr[q][r];
          im[ob + r * Ns] = conj_out ? -vi[q][r] : vi[q][r];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
__device__ void lds_fft(T *re, T *im, int ls, int nlines, const FftPlan &pl,
                        const T *twr, const T *twi, bool inverse) {
  int Ns = 1;
  for (int ps = 0; ps < pl.npass; ++ps) {
    const int R = pl.radix[ps];
    const bool ci = inverse && ps == 0, co = inverse && ps == pl.npass - 1;
    switch (R) {
      case 2: stockham_pass<T, 2>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      case 3: stockham_pass<T, 3>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      case 4: stockham_pass<T, 4>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      default: stockham_pass<T, 5>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
    }
    Ns *= R;
  }
}

}  // namespace enuf
