// ecs_reduce.h -- block reductions and the device-side Bi-CGSTAB scalar
// recurrence shared by the kernels that fuse a dot product into their pass.
#pragma once

#include "ecs_krylov.h"

namespace ecs {

constexpr int kRedThreads = 256;  // 4 waves of 64

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of a complex value (blockDim.x == kRedThreads); result in thread 0
__device__ __forceinline__ cplx<double> block_sum(cplx<double> v, cplx<double> *lds /* >= 4 */) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  cplx<double> s = mk<double>(0, 0);
  if (threadIdx.x == 0)
    for (int q = 0; q < kRedThreads / 64; q++) s = s + lds[q];
  return s;
}

// This thread's share of a second-stage reduction: x[t] + x[t + B] + ... over
// the entries below n (t = threadIdx.x, B = kRedThreads), added in that order.
// The loads of a chunk are all issued before the first add: a plain strided
// loop waits for each load before issuing the next, one memory round trip
// per entry.
__device__ __forceinline__ cplx<double> strided_sum(const cplx<double> *x, int n) {
  constexpr int U = 16;
  cplx<double> s = mk<double>(0, 0);
  for (int b0 = threadIdx.x; b0 < n; b0 += U * kRedThreads) {
    cplx<double> v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int b = b0 + u * kRedThreads;
      v[u] = x[b < n ? b : b0];
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (b0 + u * kRedThreads < n) s = s + v[u];
  }
  return s;
}

// Bi-CGSTAB scalar recurrence on the reduced dot products d0, d1.
__device__ inline void bicg_update(BicgScalars *S, int mode, cplx<double> d0, cplx<double> d1) {
  const cplx<double> zero = mk<double>(0, 0);
  switch (mode) {
    case kBicgAlpha:  // alpha = rho / (r^, v)
      if (abs2(d0) == 0 || S->bad) { S->bad = 1; S->alpha = zero; break; }
      S->alpha = cdiv(S->rho, d0);
      break;
    case kBicgOmega:  // omega = (t, s) / (t, t)
      if (d1.re == 0 || S->bad) { S->bad = 1; S->omega = zero; break; }
      S->omega = (1.0 / d1.re) * d0;
      break;
    case kBicgInit:  // (re)start: rho = (r^, r) = ||r||^2, p = r on the first step
      S->breakdowns += S->bad;
      S->rnorm2 = d0.re;
      S->est = sqrt(d0.re) / S->bnorm;
      S->rho = mk<double>(d0.re, 0);
      S->alpha = mk<double>(1, 0);
      S->omega = mk<double>(1, 0);
      S->beta = zero;
      S->bad = !(S->est == S->est) || isinf(S->est) || d0.re == 0;
      break;
    case kBicgNormRho: {  // end of a step: ||r||^2 = d0, rho1 = (r^, r) = d1, beta for the next step
      S->rnorm2 = d0.re;
      S->est = sqrt(d0.re) / S->bnorm;
      if (!(S->est == S->est) || isinf(S->est)) S->bad = 1;
      if (abs2(d1) == 0 || abs2(S->rho) == 0 || abs2(S->omega) == 0 || S->bad) {
        S->bad = 1; S->beta = zero; S->alpha = zero; S->omega = zero;
        break;
      }
      S->beta = cdiv(d1, S->rho) * cdiv(S->alpha, S->omega);
      S->rho = d1;
      break;
    }
  }
}

}  // namespace ecs
