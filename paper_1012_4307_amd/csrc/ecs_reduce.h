// ecs_reduce.h -- block reductions and the device-side Bi-CGSTAB scalar
// recurrence shared by the kernels that fuse a dot product into their pass.
#pragma once

#include "ecs_krylov.h"

namespace ecs {

constexpr int kRedThreads = 256;  // 4 waves of 64

// The wave's sum in every lane: the butterfly v += v[lane ^ o], o = 32, 16,
// ..., 1, with each exchange done in registers rather than through the LDS
// crossbar -- lanes ^ 32 and ^ 16 by the permlane swaps (each returns both
// halves of the swapped pair: a lane takes the half that came from the other
// side), ^ 8 by a row rotation by 8 (exact within a 16-lane row), and ^ 4, 2,
// 1 by rotations by 4, 2, 1: after the ^ 8 step every value repeats with
// period 8 within its row (then 4, then 2), so a lane's rotation partner
// holds the same value as its xor partner.  Every addition has the same
// operands in the same order as the plain butterfly, so the sums are equal
// bit for bit.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_xor32(double v) {
  const bool low = (__lane_id() & 32) == 0;
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(low ? hi[1] : hi[0], low ? lo[1] : lo[0]);
}
__device__ __forceinline__ double lane_xor16(double v) {
  const bool even = (__lane_id() & 16) == 0;
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(even ? hi[1] : hi[0], even ? lo[1] : lo[0]);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += lane_xor32(v);
  v += lane_xor16(v);
  v += dpp_move<0x128>(v);  // row_ror:8
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x122>(v);  // row_ror:2
  v += dpp_move<0x121>(v);  // row_ror:1
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
