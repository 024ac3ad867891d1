// enuf_device.h -- device helpers of the ENUF kernels (gfx950): window
// series evaluation, wavefront reductions and the LDS-resident Stockham FFT.
#pragma once

#include "enuf_internal.h"

namespace enuf {

// ---------------------------------------------------------------------------
// Small math helpers
// ---------------------------------------------------------------------------
// Pointers to global memory.  The batched kernels read buffer addresses from
// a member table in device memory, and a pointer loaded from memory is
// generic (flat) unless its address space is stated.  Flat loads are counted
// against LDS traffic too, which would serialise them behind the LDS atomics
// and queue writes of these kernels, so the kernel bodies take global pointers.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_g(T *p) {
  return (gptr<T>)p;
}

// Loads and stores of HIP vector types (double2/4, float2) through global
// pointers go through their native vector representation.
template <typename V>
__device__ __forceinline__ V gload(gptr<const V> p) {
  V r;
  get_native_vector(r) = *(gptr<const typename V::Native_vec_>)p;
  return r;
}
template <typename V>
__device__ __forceinline__ V gload(gptr<V> p) {
  return gload<V>((gptr<const V>)p);
}
template <typename V>
__device__ __forceinline__ void gstore(gptr<V> p, const V &v) {
  *(gptr<typename V::Native_vec_>)p = get_native_vector(v);
}

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

// q = a / b and *rem = a % b for 0 <= a < 2^22 and 1 <= b < 2^11, from a
// single-precision reciprocal inv_b = 1/b: the estimate a * inv_b is within
// 0.5 of a/b, so its floor is off by at most one and is corrected (a few
// instructions instead of an integer division).
__device__ __forceinline__ int fdivmod(int a, int b, float inv_b, int *rem) {
  int q = (int)((float)a * inv_b);
  int r = a - q * b;
  if (r < 0) {
    --q;
    r += b;
  } else if (r >= b) {
    ++q;
    r -= b;
  }
  *rem = r;
  return q;
}

// ---------------------------------------------------------------------------
// Chebyshev series sum_{k<=n} c_k T_k(x) by Clenshaw's recurrence.  The mesh
// kernels evaluate the window from per-offset series of this form (the
// piecewise-polynomial kernel evaluation of Barnett, Magland & af Klinteberg,
// SIAM J. Sci. Comput. 2019), fitted on the host to the window above.
// ---------------------------------------------------------------------------
// NS Chebyshev series of one degree n evaluated together: series i has
// coefficients c[i][0..n] and argument x[i].  One loop advances every
// recurrence, so their coefficient loads and multiply-adds interleave (a loop
// per series would wait on each load in turn).
template <typename T, int NS>
__device__ __forceinline__ void clenshaw_n(const T *const (&c)[NS], const T (&x)[NS], int n, T (&out)[NS]) {
  T b1[NS], b2[NS], x2[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    b1[i] = (T)0;
    b2[i] = (T)0;
    x2[i] = x[i] + x[i];
  }
#pragma unroll 4
  for (int k = n; k >= 1; --k) {
    T ck[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) ck[i] = c[i][k];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const T t = ck[i] + x2[i] * b1[i] - b2[i];
      b2[i] = b1[i];
      b1[i] = t;
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i] = c[i][0] + x[i] * b1[i] - b2[i];
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

// The same rounding (to nearest, ties to even) of v * scale in three
// instructions for |v * scale| < 2^51 - 1: adding 1.5 * 2^52 moves the value
// into the binade [2^52, 2^53), whose spacing is 1, so the addition itself
// rounds to an integer and the bit pattern is that integer plus the constant's.
// Larger magnitudes are clamped to +-(2^51 - 1) (the clamp also keeps the
// product from being fused with the addition, which would round once instead
// of twice).
__device__ inline long long to_fixed_fast(double v, double scale) {
  constexpr double kMagic = 6755399441055744.0;   // 1.5 * 2^52
  constexpr double kLim = 2251799813685247.0;     // 2^51 - 1
  const double x = fmin(fmax(v * scale, -kLim), kLim);
  return __double_as_longlong(x + kMagic) - __double_as_longlong(kMagic);
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
// Butterflies per thread per sweep.  One: a radix-8 butterfly already holds
// 16 values, and the mesh kernels run at the edge of their register budget.
template <typename T, int R> struct MaxBfly { static constexpr int value = 1; };

template <typename T, int R>
__device__ __forceinline__ void dft_radix(T *xr, T *xi) {
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
  } else if constexpr (R == 8) {
    // two 4-point DFTs of the even and odd elements, then e^{-2 pi i k/8} on the odd ones
    T er[4] = {xr[0], xr[2], xr[4], xr[6]}, ei[4] = {xi[0], xi[2], xi[4], xi[6]};
    T orr[4] = {xr[1], xr[3], xr[5], xr[7]}, oi[4] = {xi[1], xi[3], xi[5], xi[7]};
    dft_radix<T, 4>(er, ei);
    dft_radix<T, 4>(orr, oi);
    const T h = (T)0.70710678118654752440;
    const T t1r = h * (orr[1] + oi[1]), t1i = h * (oi[1] - orr[1]);   // (1 - i)/sqrt2
    const T t2r = oi[2], t2i = -orr[2];                                // -i
    const T t3r = h * (oi[3] - orr[3]), t3i = -h * (orr[3] + oi[3]);   // -(1 + i)/sqrt2
    xr[0] = er[0] + orr[0]; xi[0] = ei[0] + oi[0];
    xr[4] = er[0] - orr[0]; xi[4] = ei[0] - oi[0];
    xr[1] = er[1] + t1r; xi[1] = ei[1] + t1i;
    xr[5] = er[1] - t1r; xi[5] = ei[1] - t1i;
    xr[2] = er[2] + t2r; xi[2] = ei[2] + t2i;
    xr[6] = er[2] - t2r; xi[6] = ei[2] - t2i;
    xr[3] = er[3] + t3r; xi[3] = ei[3] + t3i;
    xr[7] = er[3] - t3r; xi[7] = ei[3] - t3i;
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
// Thread t takes butterfly j = t mod (n/R) of lines t div (n/R), + lpb, ...
// (lpb lines per sweep): its index arithmetic and its R - 1 twiddles are the
// same for every line, so they are computed once per pass, not per butterfly.
template <typename T, int R>
__device__ __forceinline__ void stockham_pass(T *re, T *im, int ls, int nlines, int n, int Ns, const T *twr,
                              const T *twi, bool conj_in, bool conj_out) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int nb = n / R;                 // butterflies per line (<= n / 2 < blockDim.x)
  const int tstep = n / (Ns * R);
  const int lpb = nt / nb;              // lines per sweep step
  const int lrow = tid / nb, j = tid - lrow * nb;
  const bool active = lrow < lpb;
  const int k = j % Ns;
  const int ob = (j / Ns) * Ns * R + k;  // output offset of the butterfly within its line
  T wr[R], wi[R];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const int ti = k * r * tstep;
    wr[r] = twr[ti];
    wi[r] = twi[ti];
  }
  constexpr int kMaxBfly = MaxBfly<T, R>::value;
  for (int l0 = 0; l0 < nlines; l0 += lpb * kMaxBfly) {
    T vr[kMaxBfly][R], vi[kMaxBfly][R];
#pragma unroll
    for (int q = 0; q < kMaxBfly; ++q) {
      const int line = l0 + lrow + q * lpb;
      if (active && line < nlines) {
        const int base = line * ls + j;
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
      const int line = l0 + lrow + q * lpb;
      if (active && line < nlines) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const T xr = vr[q][r], xi = vi[q][r];
          vr[q][r] = xr * wr[r] - xi * wi[r];
          vi[q][r] = xr * wi[r] + xi * wr[r];
        }
        dft_radix<T, R>(vr[q], vi[q]);
        const int o = line * ls + ob;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          re[o + r * Ns] = vr[q][r];
          im[o + r * Ns] = conj_out ? -vi[q][r] : vi[q][r];
        }
      }
    }
    __syncthreads();
  }
}

// Passes of a length-N transform with radices fixed at compile time: the
// index arithmetic of every pass folds to constants.
template <typename T, bool INV, int N, int NS, int R, int... Rest>
__device__ __forceinline__ void fft_passes(T *re, T *im, int ls, int nlines, const T *twr, const T *twi) {
  constexpr bool first = NS == 1, last = sizeof...(Rest) == 0;
  stockham_pass<T, R>(re, im, ls, nlines, N, NS, twr, twi, INV && first, INV && last);
  if constexpr (!last) fft_passes<T, INV, N, NS * R, Rest...>(re, im, ls, nlines, twr, twi);
}

template <typename T, int N, int... Rs>
__device__ __forceinline__ void fft_fixed(T *re, T *im, int ls, int nlines, const T *twr, const T *twi,
                                          bool inverse) {
  if (inverse)
    fft_passes<T, true, N, 1, Rs...>(re, im, ls, nlines, twr, twi);
  else
    fft_passes<T, false, N, 1, Rs...>(re, im, ls, nlines, twr, twi);
}

template <typename T>
__device__ __forceinline__ void lds_fft(T *re, T *im, int ls, int nlines, const FftPlan &pl,
                        const T *twr, const T *twi, bool inverse) {
  // power-of-two meshes take fixed radix-8 sequences; other lengths the plan's
  switch (pl.n) {
    case 32: fft_fixed<T, 32, 8, 4>(re, im, ls, nlines, twr, twi, inverse); return;
    case 64: fft_fixed<T, 64, 8, 8>(re, im, ls, nlines, twr, twi, inverse); return;
    case 128: fft_fixed<T, 128, 8, 4, 4>(re, im, ls, nlines, twr, twi, inverse); return;
    default: break;
  }
  int Ns = 1;
  for (int ps = 0; ps < pl.npass; ++ps) {
    const int R = pl.radix[ps];
    const bool ci = inverse && ps == 0, co = inverse && ps == pl.npass - 1;
    switch (R) {
      case 2: stockham_pass<T, 2>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      case 3: stockham_pass<T, 3>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      case 4: stockham_pass<T, 4>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      case 8: stockham_pass<T, 8>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
      default: stockham_pass<T, 5>(re, im, ls, nlines, pl.n, Ns, twr, twi, ci, co); break;
    }
    Ns *= R;
  }
}

}  // namespace enuf
