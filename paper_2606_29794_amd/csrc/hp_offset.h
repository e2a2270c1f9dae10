// hp_offset.h -- the spherical offset of Sec. 3.4 in the form the kernels
// evaluate it, shared by the forward and backward render kernels.
//
// The paper measures the great-circle distance d_gc from the Gaussian centre
// to the pixel centre (haversine) and splits it along the bearing beta taken
// at the centre: d = d_gc (sin beta, cos beta) in the (east, north) tangent
// frame.  With the unit tangent frame (e_omega, e_phi) at the centre u and
// a = p.e_omega, b = p.e_phi, c = p.u for the pixel direction p, the same
// vector is d = (d_gc / sin d_gc) (a, b) with sin d_gc = sqrt(a^2 + b^2) and
// d_gc = atan2(sqrt(a^2 + b^2), c).  So q = d^T Sigma_arc^-1 d = k2 * qt with
// qt = A a^2 + 2 B a b + C b^2 and k2 = (d_gc / sin d_gc)^2 >= 1.
#pragma once

#include <hip/hip_runtime.h>

// (asin s / s)^2 as a polynomial in s^2 for c > 0 and s^2 < 1/16:
// (asin x)^2 = (1/2) sum_n (2x)^(2n) / (n^2 C(2n, n)); truncation error < 3e-9.
#define HP_K2_S2MAX 0.0625f
__device__ __forceinline__ float hp_k2_series(float s2) {
  return 1.f + s2 * (0.33333333f + s2 * (0.17777778f + s2 * (0.11428571f + s2 * (0.081269841f + s2 * 0.061568062f))));
}
__device__ __forceinline__ float hp_k2_series_deriv(float s2) {  // d k2 / d s2
  return 0.33333333f + s2 * (2.f * 0.17777778f + s2 * (3.f * 0.11428571f + s2 * (4.f * 0.081269841f + s2 * 5.f * 0.061568062f)));
}

// k2 = (atan2(s, c) / s)^2 for any (s^2, c); returns +inf at the antipode.
__device__ __forceinline__ float hp_k2(float s2, float c) {
  if (c > 0.f && s2 < HP_K2_S2MAX) return hp_k2_series(s2);
  if (!(s2 > 0.f)) return c > 0.f ? 1.f : __int_as_float(0x7f800000);
  const float s = sqrtf(s2);
  const float d = atan2f(s, c);
  return d * d / s2;
}

// k2 and its partial derivatives with respect to s^2 (dk2_ds2) and c (dk2_dc),
// on any extension off the unit sphere: only derivatives along motions that
// keep a^2 + b^2 + c^2 = 1 are used.
__device__ __forceinline__ float hp_k2_grad(float s2, float c, float* dk2_ds2, float* dk2_dc) {
  if (c > 0.f && s2 < HP_K2_S2MAX) {
    *dk2_ds2 = hp_k2_series_deriv(s2);
    *dk2_dc = 0.f;
    return hp_k2_series(s2);
  }
  if (!(s2 > 0.f)) {
    *dk2_ds2 = 0.f;
    *dk2_dc = 0.f;
    return c > 0.f ? 1.f : __int_as_float(0x7f800000);
  }
  const float s = sqrtf(s2);
  const float d = atan2f(s, c);
  const float ir2 = __builtin_amdgcn_rcpf(s2 + c * c);
  const float is2 = __builtin_amdgcn_rcpf(s2);
  const float is = __builtin_amdgcn_rcpf(s);
  const float k2 = d * d * is2;
  // d/ds (d^2/s^2) = 2 d (c / r2) / s^2 - 2 d^2 / s^3; chain ds/ds2 = 1/(2s)
  const float dk2_ds = 2.f * d * c * ir2 * is2 - 2.f * k2 * is;
  *dk2_ds2 = 0.5f * dk2_ds * is;
  *dk2_dc = -2.f * d * s * ir2 * is2;
  return k2;
}
