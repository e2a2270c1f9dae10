// k_preprocess.hip -- stage 1 of Alg. 1: per-Gaussian projection onto the
// HEALPix sphere (Eq. lonlat_projection), radian covariance with the latitude
// scaling of Eq. arc_scaling, conic, bounding radius and SH colour.
#include "hp_common.h"
#include "hp_sh.h"

// Projection of one Gaussian (inputs already in registers) for one view.
__device__ __forceinline__ void project_one(int deg, float mx, float my, float mz, const float s_in[3],
                                            const float qin[4], float op, const float* shc /*[16][3]*/,
                                            const HpViewK& V, float r_min, float rs_sigma, float sh_off, float guard,
                                            float4 out[4], float* depth, float* radius) {
  const float tx = V.W[0] * mx + V.W[1] * my + V.W[2] * mz + V.b[0];
  const float ty = V.W[3] * mx + V.W[4] * my + V.W[5] * mz + V.b[1];
  const float tz = V.W[6] * mx + V.W[7] * my + V.W[8] * mz + V.b[2];
  const float rho = sqrtf(tx * tx + tz * tz);
  const float r = sqrtf(rho * rho + ty * ty);
  bool ok = (r >= r_min) && (rho > 1e-12f * r);
  float4 r0 = make_float4(0, 0, 0, 0), r1 = r0, r2 = r0, r3 = r0;
  float dep = __int_as_float(0x7f800000), rad = 0.f;
  if (ok) {
    const float ir = 1.f / r, irho = 1.f / rho;
    const float ux = tx * ir, uy = ty * ir, uz = tz * ir;
    const float cp = rho * ir, sp = uy;          // cos/sin of latitude phi
    const float co = tz * irho, so = tx * irho;  // cos/sin of longitude omega
    // tangent frame: e_omega = (co, 0, -so), e_phi = (-sp so, cp, -sp co)
    const float eo0 = co, eo2 = -so;
    const float ep0 = -sp * so, ep1 = cp, ep2 = -sp * co;
    // rotation from the normalised quaternion (w, x, y, z)
    float qw = qin[0], qx = qin[1], qy = qin[2], qz = qin[3];
    const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const float R00 = 1.f - 2.f * (qy * qy + qz * qz), R01 = 2.f * (qx * qy - qw * qz), R02 = 2.f * (qx * qz + qw * qy);
    const float R10 = 2.f * (qx * qy + qw * qz), R11 = 1.f - 2.f * (qx * qx + qz * qz), R12 = 2.f * (qy * qz - qw * qx);
    const float R20 = 2.f * (qx * qz - qw * qy), R21 = 2.f * (qy * qz + qw * qx), R22 = 1.f - 2.f * (qx * qx + qy * qy);
    // E W (2x3)
    float a0 = eo0 * V.W[0] + eo2 * V.W[6], a1 = eo0 * V.W[1] + eo2 * V.W[7], a2 = eo0 * V.W[2] + eo2 * V.W[8];
    float b0 = ep0 * V.W[0] + ep1 * V.W[3] + ep2 * V.W[6];
    float b1 = ep0 * V.W[1] + ep1 * V.W[4] + ep2 * V.W[7];
    float b2 = ep0 * V.W[2] + ep1 * V.W[5] + ep2 * V.W[8];
    // V = (E W R diag(s)) / r, so Sigma_arc = V V^T
    const float s0 = s_in[0] * ir, s1 = s_in[1] * ir, s2 = s_in[2] * ir;
    const float v00 = (a0 * R00 + a1 * R10 + a2 * R20) * s0;
    const float v01 = (a0 * R01 + a1 * R11 + a2 * R21) * s1;
    const float v02 = (a0 * R02 + a1 * R12 + a2 * R22) * s2;
    const float v10 = (b0 * R00 + b1 * R10 + b2 * R20) * s0;
    const float v11 = (b0 * R01 + b1 * R11 + b2 * R21) * s1;
    const float v12 = (b0 * R02 + b1 * R12 + b2 * R22) * s2;
    const float sa = v00 * v00 + v01 * v01 + v02 * v02;
    const float sb = v00 * v10 + v01 * v11 + v02 * v12;
    const float sc = v10 * v10 + v11 * v11 + v12 * v12;
    // det(V V^T) = |v0 x v1|^2 (Lagrange identity): no cancellation
    const float c0 = v01 * v12 - v02 * v11, c1 = v02 * v10 - v00 * v12, c2 = v00 * v11 - v01 * v10;
    const float det = c0 * c0 + c1 * c1 + c2 * c2;
    if (det > 0.f && isfinite(det)) {
      const float idet = 1.f / det;
      const float hm = 0.5f * (sa + sc), hd = 0.5f * (sa - sc);
      const float lmax = hm + sqrtf(hd * hd + sb * sb);
      rad = fminf((float)M_PI, rs_sigma * sqrtf(lmax));
      dep = r;
      // view-dependent colour
      const float vx = mx - V.c[0], vy = my - V.c[1], vz = mz - V.c[2];
      const float ivn = rsqrtf(vx * vx + vy * vy + vz * vz);
      float Y[16];
      hp_sh_eval(deg, vx * ivn, vy * ivn, vz * ivn, Y);
      const int K = (deg + 1) * (deg + 1);
      float col[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = sh_off;
        for (int k = 0; k < K; ++k) acc += shc[k * 3 + ch] * Y[k];
        col[ch] = fmaxf(acc, 0.f);
      }
      r0 = make_float4(ux, uy, uz, op);
      r1 = make_float4(eo0, eo2, ep0, ep1);
      r2 = make_float4(ep2, sc * idet, -sb * idet, sa * idet);
      // sin of half the tile-test angle r_s + guard, used by the binning
      r3 = make_float4(col[0], col[1], col[2], sinf(0.5f * fminf(rad + guard, (float)M_PI)));
    }
  }
  out[0] = r0;
  out[1] = r1;
  out[2] = r2;
  out[3] = r3;
  *depth = dep;
  *radius = rad;
}

#define HP_MAX_VIEWS 8
struct PreBatch {
  int n;
  HpViewK V[HP_MAX_VIEWS];
  float4* rec[HP_MAX_VIEWS];
  float* depth[HP_MAX_VIEWS];
  float* radius[HP_MAX_VIEWS];
  float4* disc[HP_MAX_VIEWS];
};

// One thread per Gaussian; SoA inputs give coalesced loads and are read once
// for all the views of the batch.  The 64-byte records of a block's 256
// Gaussians are contiguous in memory: they go through LDS so that every
// store instruction writes 4 KB of whole lines (a thread storing its own
// record would leave every store a quarter-line write).
// DEG: SH degree as a compile-time constant, so that the coefficient loads
// are unconditional and all in flight together
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(int64_t P, const float* __restrict__ mean,
                                                    const float* __restrict__ scale, const float* __restrict__ rot,
                                                    const float* __restrict__ opac, const float* __restrict__ sh,
                                                    PreBatch B, float r_min, float rs_sigma, float sh_off,
                                                    float guard) {
  __shared__ float4 s_rec[4 * 256];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 256;
  const int64_t i = i0 + tid;
  const bool ok = i < P;
  const int64_t ii = ok ? i : P - 1;  // past the end: a valid Gaussian, result dropped
  const float mx = mean[ii], my = mean[P + ii], mz = mean[2 * P + ii];
  const float s[3] = {scale[ii], scale[P + ii], scale[2 * P + ii]};
  const float q[4] = {rot[ii], rot[P + ii], rot[2 * P + ii], rot[3 * P + ii]};
  const float op = opac[ii];
  constexpr int K = (DEG + 1) * (DEG + 1);
  float shc[48];
#pragma unroll
  for (int k = 0; k < 48; ++k) shc[k] = k < 3 * K ? sh[(int64_t)k * P + ii] : 0.f;
  const int64_t nq = 4 * (P - i0 < 256 ? P - i0 : 256);  // float4 of this block's records
  for (int v = 0; v < B.n; ++v) {
    float4 r[4];
    float dep, rad;
    project_one(DEG, mx, my, mz, s, q, op, shc, B.V[v], r_min, rs_sigma, sh_off, guard, r, &dep, &rad);
    if (ok) {
      B.depth[v][i] = dep;
      B.radius[v][i] = rad;
      B.disc[v][i] = make_float4(r[0].x, r[0].y, r[0].z, r[3].w);
    }
    __syncthreads();  // the previous view's records have left LDS
#pragma unroll
    for (int k = 0; k < 4; ++k) s_rec[4 * tid + k] = r[k];
    __syncthreads();
    float4* dst = B.rec[v] + 4 * i0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k * 256 + tid < nq) dst[k * 256 + tid] = s_rec[k * 256 + tid];
  }
}

extern "C" size_t hp_projected_bytes(int64_t P) { return P < 0 ? 0 : hp_proj_size(P); }

extern "C" const float* hp_projected_depth(const void* projected, int64_t P) {
  return projected ? hp_proj_view((const char*)projected, P).depth : nullptr;
}
extern "C" const float* hp_projected_radius(const void* projected, int64_t P) {
  return projected ? hp_proj_view((const char*)projected, P).radius : nullptr;
}

extern "C" hp_status hp_preprocess(const hp_gaussians* g, const hp_view* view, const hp_params* prm, void* projected,
                                   size_t projected_bytes, void* stream) {
  HP_TRY(hp_check_gaussians(g));
  HP_TRY(hp_check_view(view, prm));
  if (!projected) return HP_ERR_INVALID_ARG;
  if (projected_bytes < hp_proj_size(g->P)) return HP_ERR_CAPACITY;
  if (g->P == 0) return HP_OK;
  return hp_preprocess_batch(g, 1, view, prm, &projected, projected_bytes, stream);
}

extern "C" hp_status hp_preprocess_batch(const hp_gaussians* g, int32_t n_views, const hp_view* views,
                                         const hp_params* prm, void* const* projected, size_t projected_bytes,
                                         void* stream) {
  HP_TRY(hp_check_gaussians(g));
  if (n_views < 1 || n_views > HP_MAX_VIEWS || !views || !projected) return HP_ERR_INVALID_ARG;
  PreBatch B;
  B.n = n_views;
  for (int v = 0; v < n_views; ++v) {
    HP_TRY(hp_check_view(&views[v], prm));
    if (!projected[v]) return HP_ERR_INVALID_ARG;
    HpProjView pv = hp_proj_view((char*)projected[v], g->P);
    B.V[v] = hp_viewk(&views[v]);
    B.rec[v] = pv.rec;
    B.depth[v] = pv.depth;
    B.radius[v] = pv.radius;
    B.disc[v] = pv.disc;
  }
  if (projected_bytes < hp_proj_size(g->P)) return HP_ERR_CAPACITY;
  if (g->P == 0) return HP_OK;
  const dim3 grid(hp_blocks(g->P, 256)), block(256);
  hipStream_t st = (hipStream_t)stream;
  switch (g->sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess<0>, grid, block, 0, st, g->P, g->mean, g->scale, g->rot, g->opacity, g->sh, B,
                               prm->r_min, prm->rs_sigma, prm->sh_offset, prm->bin_guard); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, grid, block, 0, st, g->P, g->mean, g->scale, g->rot, g->opacity, g->sh, B,
                               prm->r_min, prm->rs_sigma, prm->sh_offset, prm->bin_guard); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, grid, block, 0, st, g->P, g->mean, g->scale, g->rot, g->opacity, g->sh, B,
                               prm->r_min, prm->rs_sigma, prm->sh_offset, prm->bin_guard); break;
    default: hipLaunchKernelGGL(k_preprocess<3>, grid, block, 0, st, g->P, g->mean, g->scale, g->rot, g->opacity, g->sh, B,
                                prm->r_min, prm->rs_sigma, prm->sh_offset, prm->bin_guard); break;
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// ---------------------------------------------------------------------------
// Backward of stage 1 (Sec. 3.2, Eqs. backward_lat_scale and grad_via_J_S).
// Inputs per Gaussian: dL/d(colour, opacity, conic A B C, omega, phi) from the
// pixel pass.  Sigma_arc = V V^T with V = (1/r) E W R diag(s) and E the unit
// tangent frame, which equals S_phi J W R diag(s): the latitude term of Eq.
// backward_lat_scale and the J term of Eq. grad_via_J_S both arrive through
// the dependence of E and r on the camera-space centre t.
// ---------------------------------------------------------------------------
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_bwd(int64_t P, const float* __restrict__ mean,
                                                        const float* __restrict__ scale, const float* __restrict__ rot,
                                                        const float* __restrict__ sh, HpViewK V, float r_min,
                                                        float sh_off, const float* __restrict__ acc,
                                                        float* __restrict__ gmean, float* __restrict__ gscale,
                                                        float* __restrict__ grot, float* __restrict__ gopac,
                                                        float* __restrict__ gsh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  // [0..8] as the pixel pass writes them, [9] dL/d(1/r) of the depth channel
  float gy[10];
  bool any = false;
#pragma unroll
  for (int m = 0; m < 10; ++m) {
    gy[m] = acc[m * P + i];
    any = any || gy[m] != 0.f;
  }
  if (!any) return;
  const float mx = mean[i], my = mean[P + i], mz = mean[2 * P + i];
  const float tx = V.W[0] * mx + V.W[1] * my + V.W[2] * mz + V.b[0];
  const float ty = V.W[3] * mx + V.W[4] * my + V.W[5] * mz + V.b[1];
  const float tz = V.W[6] * mx + V.W[7] * my + V.W[8] * mz + V.b[2];
  const float rho = sqrtf(tx * tx + tz * tz);
  const float r = sqrtf(rho * rho + ty * ty);
  if (!((r >= r_min) && (rho > 1e-12f * r))) return;
  const float ir = 1.f / r, irho = 1.f / rho;
  const float cp = rho * ir, sp = ty * ir, co = tz * irho, so = tx * irho;
  const float ux = tx * ir, uy = ty * ir, uz = tz * ir;
  const float E[2][3] = {{co, 0.f, -so}, {-sp * so, cp, -sp * co}};
  // rotation
  const float q0 = rot[i], q1 = rot[P + i], q2 = rot[2 * P + i], q3 = rot[3 * P + i];
  const float qn = rsqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const float w = q0 * qn, x = q1 * qn, y = q2 * qn, z = q3 * qn;
  const float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                         {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                         {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  float EW[2][3], M[2][3], Vm[2][3];
  const float s[3] = {scale[i], scale[P + i], scale[2 * P + i]};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) EW[a][j] = E[a][0] * V.W[j] + E[a][1] * V.W[3 + j] + E[a][2] * V.W[6 + j];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      M[a][k] = EW[a][0] * R[0][k] + EW[a][1] * R[1][k] + EW[a][2] * R[2][k];
      Vm[a][k] = M[a][k] * s[k] * ir;
    }
  const float sa = Vm[0][0] * Vm[0][0] + Vm[0][1] * Vm[0][1] + Vm[0][2] * Vm[0][2];
  const float sb = Vm[0][0] * Vm[1][0] + Vm[0][1] * Vm[1][1] + Vm[0][2] * Vm[1][2];
  const float sc = Vm[1][0] * Vm[1][0] + Vm[1][1] * Vm[1][1] + Vm[1][2] * Vm[1][2];
  const float c0 = Vm[0][1] * Vm[1][2] - Vm[0][2] * Vm[1][1], c1 = Vm[0][2] * Vm[1][0] - Vm[0][0] * Vm[1][2],
              c2 = Vm[0][0] * Vm[1][1] - Vm[0][1] * Vm[1][0];
  const float det = c0 * c0 + c1 * c1 + c2 * c2;
  if (!(det > 0.f)) return;
  const float idet = 1.f / det;
  const float QA = sc * idet, QB = -sb * idet, QC = sa * idet;
  // conic -> Sigma_arc:  G_S = -Q G_Q Q with G_Q = [[gA, gB/2], [gB/2, gC]]
  const float gA = gy[4], gB = 0.5f * gy[5], gC = gy[6];
  const float t00 = QA * gA + QB * gB, t01 = QA * gB + QB * gC;
  const float t10 = QB * gA + QC * gB, t11 = QB * gB + QC * gC;
  const float G00 = -(t00 * QA + t01 * QB), G01 = -(t00 * QB + t01 * QC), G11 = -(t10 * QB + t11 * QC);
  // Sigma = V V^T  ->  dL/dV = 2 G V
  float gV[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gV[0][k] = 2.f * (G00 * Vm[0][k] + G01 * Vm[1][k]);
    gV[1][k] = 2.f * (G01 * Vm[0][k] + G11 * Vm[1][k]);
  }
  // V = M diag(s) / r
  float gr = 0.f, gM[2][3], dscale[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dscale[k] = (gV[0][k] * M[0][k] + gV[1][k] * M[1][k]) * ir;
    gM[0][k] = gV[0][k] * s[k] * ir;
    gM[1][k] = gV[1][k] * s[k] * ir;
    gr -= (gV[0][k] * Vm[0][k] + gV[1][k] * Vm[1][k]) * ir;
  }
  // M = EW R
  float gEW[2][3], gR[3][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) gEW[a][j] = gM[a][0] * R[j][0] + gM[a][1] * R[j][1] + gM[a][2] * R[j][2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) gR[j][k] = EW[0][j] * gM[0][k] + EW[1][j] * gM[1][k];
  // EW = E W
  float gE[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) gE[a][k] = gEW[a][0] * V.W[3 * k] + gEW[a][1] * V.W[3 * k + 1] + gEW[a][2] * V.W[3 * k + 2];
  // frame motion: de_w/dw = (-so, 0, -co), de_p/dw = -sin(phi) e_w, de_p/dp = -u
  // inverse depth: d(1/r)/dr = -1/r^2, so d(1/r)/dt = -t / r^3 (Sec. 3.2)
  gr -= gy[9] * ir * ir;
  float gw = gy[7] + gE[0][0] * (-so) + gE[0][2] * (-co) - sp * (gE[1][0] * co + gE[1][2] * (-so));
  float gp = gy[8] - (gE[1][0] * ux + gE[1][1] * uy + gE[1][2] * uz);
  // (omega, phi, r) -> t:  d omega/dt = e_w / (r cos phi), d phi/dt = e_p / r, dr/dt = u
  const float kw = gw * ir / cp, kp = gp * ir;
  const float gtx = kw * co + kp * E[1][0] + gr * ux;
  const float gty = kp * E[1][1] + gr * uy;
  const float gtz = kw * (-so) + kp * E[1][2] + gr * uz;
  // t = W mu + b
  float gmx = V.W[0] * gtx + V.W[3] * gty + V.W[6] * gtz;
  float gmy = V.W[1] * gtx + V.W[4] * gty + V.W[7] * gtz;
  float gmz = V.W[2] * gtx + V.W[5] * gty + V.W[8] * gtz;
  // rotation matrix -> normalised quaternion -> raw quaternion
  const float gw_q = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
  const float gx_q = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.f * x * gR[1][1] - w * gR[1][2] + z * gR[2][0] +
                            w * gR[2][1] - 2.f * x * gR[2][2]);
  const float gy_q = 2.f * (-2.f * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                            w * gR[2][0] + z * gR[2][1] - 2.f * y * gR[2][2]);
  const float gz_q = 2.f * (-2.f * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.f * z * gR[1][1] +
                            y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
  const float dotq = w * gw_q + x * gx_q + y * gy_q + z * gz_q;
  const float drot[4] = {(gw_q - w * dotq) * qn, (gx_q - x * dotq) * qn, (gy_q - y * dotq) * qn,
                         (gz_q - z * dotq) * qn};
  // colour: SH coefficients and the viewing direction
  const float vx = mx - V.c[0], vy = my - V.c[1], vz = mz - V.c[2];
  const float ivn = rsqrtf(vx * vx + vy * vy + vz * vz);
  const float dx = vx * ivn, dy = vy * ivn, dz = vz * ivn;
  float Y[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) Y[k] = 0.f;  // basis functions above the degree stay 0
  hp_sh_eval(DEG, dx, dy, dz, Y);
  constexpr int K = (DEG + 1) * (DEG + 1);
  // all coefficients first (independent loads, all in flight at once)
  float shc[48];
#pragma unroll
  for (int k = 0; k < 48; ++k) shc[k] = k < 3 * K ? sh[(int64_t)k * P + i] : 0.f;
  float gcol[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float colour = sh_off;
#pragma unroll
    for (int k = 0; k < 16; ++k) colour += shc[k * 3 + ch] * Y[k];
    gcol[ch] = colour < 0.f ? 0.f : gy[ch];  // a clamped channel passes no gradient
  }
  float wk[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) wk[k] = gcol[0] * shc[3 * k] + gcol[1] * shc[3 * k + 1] + gcol[2] * shc[3 * k + 2];

  if (DEG > 0) {
    float ddx, ddy, ddz;
    hp_sh_grad(DEG, dx, dy, dz, wk, &ddx, &ddy, &ddz);
    const float dd = ddx * dx + ddy * dy + ddz * dz;
    gmx += (ddx - dx * dd) * ivn;
    gmy += (ddy - dy * dd) * ivn;
    gmz += (ddz - dz * dd) * ivn;
  }
  // accumulate into the gradient buffers: every read first, then every write,
  // so that the read-modify-writes of this Gaussian overlap
  float om[3], osc[3], orot[4], oop, osh[3 * K];
#pragma unroll
  for (int k = 0; k < 3; ++k) { om[k] = gmean[k * P + i]; osc[k] = gscale[k * P + i]; }
#pragma unroll
  for (int k = 0; k < 4; ++k) orot[k] = grot[k * P + i];
  oop = gopac[i];
#pragma unroll
  for (int k = 0; k < 3 * K; ++k) osh[k] = gsh[(int64_t)k * P + i];
  gmean[i] = om[0] + gmx;
  gmean[P + i] = om[1] + gmy;
  gmean[2 * P + i] = om[2] + gmz;
#pragma unroll
  for (int k = 0; k < 3; ++k) gscale[k * P + i] = osc[k] + dscale[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) grot[k * P + i] = orot[k] + drot[k];
  gopac[i] = oop + gy[3];
#pragma unroll
  for (int k = 0; k < 3 * K; ++k) gsh[(int64_t)k * P + i] = osh[k] + gcol[k % 3] * Y[k / 3];
}

hp_status hp_preprocess_bwd_launch(const hp_gaussians* g, const hp_view* view, const hp_params* prm, const float* acc,
                                   hp_gaussians_grad* grad, hipStream_t s) {
  const dim3 grid(hp_blocks(g->P, 256)), block(256);
  const HpViewK vk = hp_viewk(view);
#define HP_PRE_BWD(D)                                                                                                \
  hipLaunchKernelGGL(k_preprocess_bwd<D>, grid, block, 0, s, g->P, g->mean, g->scale, g->rot, g->sh, vk, prm->r_min, \
                     prm->sh_offset, acc, grad->mean, grad->scale, grad->rot, grad->opacity, grad->sh)
  switch (g->sh_degree) {
    case 0: HP_PRE_BWD(0); break;
    case 1: HP_PRE_BWD(1); break;
    case 2: HP_PRE_BWD(2); break;
    default: HP_PRE_BWD(3); break;
  }
#undef HP_PRE_BWD
  HP_CHECK_LAUNCH();
  return HP_OK;
}
