// Changeover-weighted force sum over a range of packed massive sources
// (Sect. 2.1.3, the direct-force routine): the inner loop shared by the kick
// kernels.  Sources are read with wave-uniform (scalar) loads.
#pragma once

#include <hip/hip_runtime.h>

#include "device_math.h"
#include "mx_internal.h"

namespace mxd {

// one interaction: K = 1 weight mu y^3, y the hardware rsqrt with the
// third-order correction y0 (1 + 3e/2 + 15e^2/8), e = 1 - s2 y0^2
// k15 = 1.5 and k1875 = 1.875 are passed in VGPRs (loop invariants) so that the
// correction is two three-operand FMAs without per-iteration constant moves.
__device__ __forceinline__ double fast_weight(double mu, double s2, double k15, double k1875) {
  double y0 = __builtin_amdgcn_rsq(s2);
  double y2 = y0 * y0;
  double e = fma(-s2, y2, 1.0);
  double c = fma(e, fma(e, k1875, k15), 1.0);
  return (mu * y0) * y2 * c;
}

__device__ __forceinline__ void vgpr_constants(double& k15, double& k1875) {
  k15 = 1.5;
  k1875 = 1.875;
  asm volatile("" : "+v"(k15), "+v"(k1875));
}

// For non-negative doubles the IEEE bit patterns order like the values.  The
// wave's largest target rc2 is reduced to its high word; upper_rc2 combines it
// with a source's rc2 into a wave-uniform bound (high word = larger high word,
// low word all ones) that is >= both values and within 2^-20 relative of the
// larger.  Pairs below the bound take the exact changeover test.
__device__ __forceinline__ uint32_t wave_max_hi(double rc2t) {
  uint32_t hi = (uint32_t)(__double_as_longlong(rc2t) >> 32);
  for (int off = 32; off > 0; off >>= 1) hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
  return __builtin_amdgcn_readfirstlane(hi);
}

__device__ __forceinline__ double upper_rc2(double rc2s, uint32_t wave_hi) {
  uint32_t hs = (uint32_t)(__double_as_longlong(rc2s) >> 32);
  uint32_t h = hs > wave_hi ? hs : wave_hi;
  return __longlong_as_double((long long)(((uint64_t)h << 32) | 0xffffffffull));
}

// Sources [s0, s1) in ascending order, two per iteration (independent chains
// for the scheduler), the next two records requested before the current ones
// are used.  The changeover branch is taken only when either pair is inside
// its changeover radius.
__device__ __forceinline__ void force_sum(const KickSource* __restrict__ src, int s0, int s1,
                                          double xt, double yt, double zt, double rc2t,
                                          double rct, double& ax, double& ay, double& az) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // high word of the largest target rc2 in the wave (wave-uniform, SALU)
  const uint32_t wave_hi = wave_max_hi(rc2t);
  double k15, k1875;
  vgpr_constants(k15, k1875);
  int s = s0;
  if (s + 1 < s1) {
    KickSource A = src[s], B = src[s + 1];
    for (; s + 1 < s1; s += 2) {
      const int na = s + 2 < s1 ? s + 2 : s;
      const int nb2 = s + 3 < s1 ? s + 3 : s;
      const KickSource NA = src[na], NB = src[nb2];
      double dxa = A.x - xt, dya = A.y - yt, dza = A.z - zt;
      double dxb = B.x - xt, dyb = B.y - yt, dzb = B.z - zt;
      double s2a = fma(dza, dza, fma(dya, dya, dxa * dxa));
      double s2b = fma(dzb, dzb, fma(dyb, dyb, dxb * dxb));
      double wa = fast_weight(A.mu, s2a, k15, k1875);
      double wb = fast_weight(B.mu, s2b, k15, k1875);
      // wave-uniform threshold >= max(rc2_source, rc2 of every target of the wave)
      if (__builtin_expect((s2a < upper_rc2(A.rc2, wave_hi)) | (s2b < upper_rc2(B.rc2, wave_hi)), 0)) {
        double rc2a = fmax(A.rc2, rc2t), rc2b = fmax(B.rc2, rc2t);
        if (s2a < rc2a) wa = A.mu * mxd::changeover_weight_slow(s2a, fmax(A.rc, rct), rc2a);
        if (s2b < rc2b) wb = B.mu * mxd::changeover_weight_slow(s2b, fmax(B.rc, rct), rc2b);
      }
      a0 = fma(wa, dxa, a0);
      a1 = fma(wa, dya, a1);
      a2 = fma(wa, dza, a2);
      a0 = fma(wb, dxb, a0);
      a1 = fma(wb, dyb, a1);
      a2 = fma(wb, dzb, a2);
      A = NA;
      B = NB;
    }
  }
  if (s < s1) {
    const KickSource A = src[s];
    double dx = A.x - xt, dy = A.y - yt, dz = A.z - zt;
    double s2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double rc2 = fmax(A.rc2, rc2t);
    double w = fast_weight(A.mu, s2, k15, k1875);
    if (s2 < rc2) w = A.mu * mxd::changeover_weight_slow(s2, fmax(A.rc, rct), rc2);
    a0 = fma(w, dx, a0);
    a1 = fma(w, dy, a1);
    a2 = fma(w, dz, a2);
  }
  ax = a0; ay = a1; az = a2;
}

}  // namespace mxd
