// hp_sh.h -- real spherical harmonics up to degree 3 in Cartesian form
// (orthonormal on the unit sphere, no Condon-Shortley phase), index
// k = l*l + l + m, evaluated at a unit direction (x, y, z).
#pragma once

#include <hip/hip_runtime.h>

// normalisation constants
#define HP_SH_C0 0.28209479177387814f   // 1 / (2 sqrt(pi))
#define HP_SH_C1 0.48860251190291992f   // sqrt(3 / (4 pi))
#define HP_SH_C2A 1.0925484305920792f   // sqrt(15 / pi) / 2
#define HP_SH_C2B 0.31539156525252005f  // sqrt(5 / pi) / 4
#define HP_SH_C2C 0.54627421529603959f  // sqrt(15 / pi) / 4
#define HP_SH_C3A 0.59004358992664352f  // sqrt(35 / (2 pi)) / 4
#define HP_SH_C3B 2.8906114426405538f   // sqrt(105 / pi) / 2
#define HP_SH_C3C 0.45704579946446572f  // sqrt(21 / (2 pi)) / 4
#define HP_SH_C3D 0.37317633259011540f  // sqrt(7 / pi) / 4
#define HP_SH_C3E 1.4453057213202769f   // sqrt(105 / pi) / 4

__device__ __forceinline__ void hp_sh_eval(int deg, float x, float y, float z, float* Y) {
  Y[0] = HP_SH_C0;
  if (deg < 1) return;
  Y[1] = HP_SH_C1 * y;
  Y[2] = HP_SH_C1 * z;
  Y[3] = HP_SH_C1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = HP_SH_C2A * x * y;
  Y[5] = HP_SH_C2A * y * z;
  Y[6] = HP_SH_C2B * (3.f * zz - 1.f);
  Y[7] = HP_SH_C2A * x * z;
  Y[8] = HP_SH_C2C * (xx - yy);
  if (deg < 3) return;
  Y[9] = HP_SH_C3A * y * (3.f * xx - yy);
  Y[10] = HP_SH_C3B * x * y * z;
  Y[11] = HP_SH_C3C * y * (5.f * zz - 1.f);
  Y[12] = HP_SH_C3D * z * (5.f * zz - 3.f);
  Y[13] = HP_SH_C3C * x * (5.f * zz - 1.f);
  Y[14] = HP_SH_C3E * z * (xx - yy);
  Y[15] = HP_SH_C3A * x * (xx - 3.f * yy);
}

// Gradient of sum_k w[k] Y_k with respect to the (unnormalised) Cartesian
// arguments, treating x, y, z as independent.
__device__ __forceinline__ void hp_sh_grad(int deg, float x, float y, float z, const float* w, float* gx, float* gy,
                                           float* gz) {
  float dx = 0.f, dy = 0.f, dz = 0.f;
  if (deg >= 1) {
    dy += HP_SH_C1 * w[1];
    dz += HP_SH_C1 * w[2];
    dx += HP_SH_C1 * w[3];
  }
  if (deg >= 2) {
    dx += HP_SH_C2A * (y * w[4] + z * w[7]) + 2.f * HP_SH_C2C * x * w[8];
    dy += HP_SH_C2A * (x * w[4] + z * w[5]) - 2.f * HP_SH_C2C * y * w[8];
    dz += HP_SH_C2A * (y * w[5] + x * w[7]) + 6.f * HP_SH_C2B * z * w[6];
  }
  if (deg >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    dx += HP_SH_C3A * 6.f * x * y * w[9] + HP_SH_C3B * y * z * w[10] + HP_SH_C3C * (5.f * zz - 1.f) * w[13] +
          2.f * HP_SH_C3E * x * z * w[14] + HP_SH_C3A * (3.f * xx - 3.f * yy) * w[15];
    dy += HP_SH_C3A * (3.f * xx - 3.f * yy) * w[9] + HP_SH_C3B * x * z * w[10] + HP_SH_C3C * (5.f * zz - 1.f) * w[11] -
          2.f * HP_SH_C3E * y * z * w[14] - HP_SH_C3A * 6.f * x * y * w[15];
    dz += HP_SH_C3B * x * y * w[10] + HP_SH_C3C * 10.f * y * z * w[11] + HP_SH_C3D * (15.f * zz - 3.f) * w[12] +
          HP_SH_C3C * 10.f * x * z * w[13] + HP_SH_C3E * (xx - yy) * w[14];
  }
  *gx = dx;
  *gy = dy;
  *gz = dz;
}
