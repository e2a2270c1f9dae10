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

// Per (pixel, Gaussian) quantities from the pixel direction p and the
// Gaussian's record (r0 = (u, opacity), r1 = (e_omega.x, e_omega.z, e_phi.x,
// e_phi.y), r2 = (e_phi.z, A, B, C)).  Written with explicit fused
// multiply-adds so that the forward and the backward kernels, which must
// take identical hit decisions, round every step identically.
struct HpOffset {
  float a, b;    // p . e_omega, p . e_phi
  float u1, u2;  // (A a + B b, B a + C b)
  float qt;      // A a^2 + 2 B a b + C b^2 = a u1 + b u2
};
__device__ __forceinline__ HpOffset hp_offset(const float p[3], float4 r1, float4 r2) {
  HpOffset o;
  o.a = fmaf(p[2], r1.y, p[0] * r1.x);
  o.b = fmaf(p[2], r2.x, fmaf(p[1], r1.w, p[0] * r1.z));
  o.u1 = fmaf(r2.y, o.a, r2.z * o.b);
  o.u2 = fmaf(r2.z, o.a, r2.w * o.b);
  o.qt = fmaf(o.a, o.u1, o.b * o.u2);
  return o;
}
// c = p . u and s^2 = a^2 + b^2
__device__ __forceinline__ float hp_offset_c(const float p[3], float4 r0) {
  return fmaf(p[2], r0.z, fmaf(p[1], r0.y, p[0] * r0.x));
}
__device__ __forceinline__ float hp_offset_s2(const HpOffset& o) { return fmaf(o.b, o.b, o.a * o.a); }

// exp(-x / 2) as one multiply and the hardware base-2 exponential.  -log2(e)/2
// is exact in float (log2 e rounded, halved), so the product is rounded once,
// exactly as in exp2(x * log2 e) with x already halved.
__device__ __forceinline__ float hp_exp_neg_half(float x) {
  return __builtin_amdgcn_exp2f(x * (-0.5f * 1.44269504088896341f));
}

// (asin s / s)^2 as a polynomial in s^2 for c > 0 and s^2 < 1/16:
// (asin x)^2 = (1/2) sum_n (2x)^(2n) / (n^2 C(2n, n)); truncation error < 3e-9.
#define HP_K2_S2MAX 0.0625f
__device__ __forceinline__ float hp_k2_series(float s2) {
  return 1.f + s2 * (0.33333333f + s2 * (0.17777778f + s2 * (0.11428571f + s2 * (0.081269841f + s2 * 0.061568062f))));
}
__device__ __forceinline__ float hp_k2_series_deriv(float s2) {  // d k2 / d s2
  return 0.33333333f + s2 * (2.f * 0.17777778f + s2 * (3.f * 0.11428571f + s2 * (4.f * 0.081269841f + s2 * 5.f * 0.061568062f)));
}

// atan2(s, c) for s > 0 (angles in (0, pi)): reduced to t = min / max of
// (s, |c|) in [0, 1], atan t = t P(t^2) with P a degree-8 polynomial fitted
// to atan(t) / t on [0, 1] for least maximum relative error by Lawson's
// algorithm (fit_atan.py; fit error 1.5e-8, 5.1e-8 with the coefficients
// rounded to float, under one ulp at 1), then reflected about pi/4 and pi/2.
__device__ __forceinline__ float hp_atan2_pos(float s, float c) {
  const float ac = fabsf(c);
  const bool steep = s > ac;
  const float t = (steep ? ac : s) * __builtin_amdgcn_rcpf(steep ? s : ac);
  const float t2 = t * t;
  float r = 0.0028500466f;
  r = r * t2 - 0.016069299f;
  r = r * t2 + 0.042692691f;
  r = r * t2 - 0.075044036f;
  r = r * t2 + 0.10640991f;
  r = r * t2 - 0.14203662f;
  r = r * t2 + 0.19992623f;
  r = r * t2 - 0.33333072f;
  r = (r * t2 + 1.f) * t;
  r = steep ? 1.57079633f - r : r;
  return c < 0.f ? 3.14159265f - r : r;
}

// k2 = (atan2(s, c) / s)^2 for any (s^2, c); returns +inf at the antipode.
// Outside the series range it is g^2 with g = atan2(s, c) / s, evaluated by
// exactly the same operations here and in hp_k2_grad, so that the forward and
// the backward pass take the same hit decisions.
__device__ __forceinline__ float hp_k2(float s2, float c) {
  if (c > 0.f && s2 < HP_K2_S2MAX) return hp_k2_series(s2);
  if (!(s2 > 0.f)) return c > 0.f ? 1.f : __int_as_float(0x7f800000);
  const float s = __builtin_amdgcn_sqrtf(s2);
  const float g = hp_atan2_pos(s, c) * __builtin_amdgcn_rcpf(s);
  return g * g;
}

// k2 and its partial derivatives with respect to s^2 (dk2_ds2) and c (dk2_dc).
// Only derivatives along motions that keep s^2 + c^2 = 1 are used (the pixel
// direction in the Gaussian's orthonormal frame), so the derivatives of
// atan2 are taken on the unit circle: d/ds = c, d/dc = -s.  Then with
// g = atan2(s, c) / s: dk2/ds = 2 g (c - g) / s and dk2/dc = -2 g.
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
  const float s = __builtin_amdgcn_sqrtf(s2);
  const float is = __builtin_amdgcn_rcpf(s);
  const float g = hp_atan2_pos(s, c) * is;
  *dk2_ds2 = g * (c - g) * (is * is);  // (dk2/ds) / (2 s)
  *dk2_dc = -2.f * g;
  return g * g;
}
