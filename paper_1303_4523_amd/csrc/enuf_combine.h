// enuf_combine.h -- device code shared by the ENUF and DPD kernel files: block
// reductions and the combine body (forces and energy partials of one
// evaluation).
#pragma once

#include "enuf_device.h"

namespace enuf {

// ---------------------------------------------------------------------------
// Block reductions with a fixed order of additions.
// scratch needs blockDim.x / 64 entries.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

__device__ __forceinline__ int block_sum_int(int v, int *scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

__device__ __forceinline__ long long block_sum_ll(long long v, long long *scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  v = wave_sum_ll(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  long long s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

__device__ __forceinline__ void
combine_body(int64_t N, gptr<const int> __restrict__ slot, gptr<const double4> __restrict__ xq,
             gptr<const unsigned long long> freal, gptr<const double4> __restrict__ part, int P2S,
             double fscale, int nblk, double *blk_eg, gptr<const unsigned long long> __restrict__ ereal,
             long long *blk_er, int *ccnt, int ncell3, int *xcnt, int M, const FinishArgs &fa, double *forces,
             int bid, double *f_out = nullptr, double *v_out = nullptr) {
  __shared__ double s_dbl[kPrepThreads / kWave];
  __shared__ long long s_ll[kPrepThreads / kWave];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)bid * blockDim.x + tid;
  {
    // the pair kernel of this step has read the step index; the next reads the advanced one
    if (fa.step_inc && bid == 0 && tid == 0) *fa.step_inc += 1ull;
    // cell counts are left cleared for the next evaluation (their consumers
    // ran before); the DPD counts are cleared here unless fa.dcnt is null
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t c = i; c < ncell3; c += stride) ccnt[c] = 0;
    for (int64_t c = i; c < M; c += stride) xcnt[c] = 0;
    if (fa.mode >= 0 && fa.dcnt)
      for (int64_t c = i; c < fa.ndcell3; c += stride) fa.dcnt[c] = 0;
  }
  double eg = 0.0;
  long long er = 0, esl = 0;
  if (i < N) {
    // the pair forces and velocities do not depend on the slot: loaded with it
    double fp[3] = {0.0, 0.0, 0.0}, vv[3] = {0.0, 0.0, 0.0};
    if (fa.mode >= 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        fp[a] = fa.fdpd[3 * i + a];
        if (fa.mode == 0) vv[a] = fa.vel[3 * i + a];
      }
    }
    const int j = slot[i];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (j >= 0) {
      // the fused multiply-adds of this body are written out (no contraction
      // left to the compiler): the combine is inlined into several kernels,
      // which must round alike
#pragma clang fp contract(off)
      er = (long long)ereal[2 * (size_t)j];
      esl = (long long)ereal[2 * (size_t)j + 1];
      double bx = 0.0, by = 0.0, bz = 0.0, a = 0.0;
#pragma unroll 8
      for (int s = 0; s < P2S; ++s) {
        const double4 v = gload(part + (size_t)j * P2S + s);
        bx += v.x;
        by += v.y;
        bz += v.z;
        a += v.w;
      }
      const double qj = gload(xq + j).w;
      const double qs = -(qj * fscale);
      fx = fma(qs, bx, (double)(long long)freal[3 * (size_t)j] * kRealFxInv);
      fy = fma(qs, by, (double)(long long)freal[3 * (size_t)j + 1] * kRealFxInv);
      fz = fma(qs, bz, (double)(long long)freal[3 * (size_t)j + 2] * kRealFxInv);
      eg = qj * a;
    }
    if (fa.mode < 0) {
      forces[3 * i] = fx;
      forces[3 * i + 1] = fy;
      forces[3 * i + 2] = fz;
    } else {
#pragma clang fp contract(off)
      const double fe[3] = {fx, fy, fz};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double f = fma(fa.kappa, fe[a], fp[a]);
        forces[3 * i + a] = f;
        const double v = fma(0.5 * fa.dt, f, vv[a]);
        // a fused next step (v_out) takes the force and the half-kicked
        // velocity from here and stores the velocity after its own kick, so
        // this store would be overwritten by the same thread
        if (v_out) {
          f_out[a] = f;
          v_out[a] = v;
        } else if (fa.mode == 0) {
          fa.vel[3 * i + a] = v;
        }
      }
    }
  }
  if (fa.energies) {  // block-uniform: the per-block energy partials only when they are reduced
    eg = block_sum(eg, s_dbl);
    er = block_sum_ll(er, s_ll);
    esl = block_sum_ll(esl, s_ll);
    if (tid == 0) {
      blk_eg[bid] = eg;
      blk_er[2 * bid] = er;
      blk_er[2 * bid + 1] = esl;
    }
  }
}

}  // namespace enuf
