// k_ssim.hip -- HEALPix-SSIM and the training loss of Sec. 4.1.
//
// One workgroup per active tile.  The tile's B x B pixels plus a 5-pixel halo
// are gathered into LDS through the face-extended chart (neighbouring faces
// with their axes turned to line up; the missing quadrant of a three-face
// vertex and inactive pixels carry weight 0).  On that regular patch the 11x11
// Gaussian window is separable, so the weighted sums of (1, x, y, x^2, y^2, xy)
// are two 11-tap passes; dividing by the summed weight renormalises where
// neighbours are missing.  The backward pass is the transposed convolution:
// the chart neighbourhood relation is symmetric with equal offset lengths, so
// the adjoint gathers the per-pixel SSIM partials over the same window.
#include "hp_common.h"

#define SS_R 5
#define SS_W 11
#define SS_MAXB 16
#define SS_MAXH (SS_MAXB + 2 * SS_R)  // 26

struct SsimArgs {
  int order, b, kt;
  const int32_t* active_tiles;
  const int32_t* tile_start;
  const int32_t* tile_count;
  const uint32_t* tile_bits;
  int64_t n_active;
  float C1, C2, lam;
  float g[SS_W];  // raw window weights exp(-a^2 / (2 sigma^2))
};

// compact slot of nested pixel q, or -1 when inactive / absent
__device__ __forceinline__ int64_t ss_slot(const SsimArgs& A, int64_t q) {
  if (q < 0) return -1;
  const int per_b = 2 * A.b;
  const int64_t t = q >> per_b;
  const int loc = (int)(q - (t << per_b));
  // a fully active tile holds its pixels in nested order: no rank to count
  if (A.tile_count[t] == (1 << per_b)) return (int64_t)A.tile_start[t] + loc;
  const uint32_t* bits = A.tile_bits + 8 * t;
  const uint32_t word = bits[loc >> 5];
  if (!((word >> (loc & 31)) & 1u)) return -1;
  int rank = __popc(word & ((1u << (loc & 31)) - 1u));
  for (int k = 0; k < (loc >> 5); ++k) rank += __popc(bits[k]);
  return (int64_t)A.tile_start[t] + rank;
}

// Patch cell of gather index i (a bijection of [0, H*H)): the first B*B
// indices are the tile's own pixels in NESTED order, which a fully active
// tile stores contiguously (coalesced loads), the rest the halo row by row.
__device__ __forceinline__ int ss_cell(int i, int B, int H) {
  if (i < B * B) {
    const int x = (int)hp_compact_bits((uint32_t)i), y = (int)hp_compact_bits((uint32_t)i >> 1);
    return (y + SS_R) * H + x + SS_R;
  }
  int h = i - B * B;
  if (h < SS_R * H) return h;  // rows above the tile
  h -= SS_R * H;
  if (h < 2 * SS_R * B) {  // left and right of the tile's rows
    const int row = SS_R + h / (2 * SS_R), c = h % (2 * SS_R);
    return row * H + (c < SS_R ? c : c + B);
  }
  h -= 2 * SS_R * B;
  return (SS_R + B) * H + h;  // rows below
}

__device__ __forceinline__ void ss_tile_origin(const SsimArgs& A, int ct, int* f, int* x0, int* y0) {
  const int t = A.active_tiles[ct];
  int tx, ty;
  hp_nest_xyf(A.kt, t, &tx, &ty, f);
  *x0 = tx << A.b;
  *y0 = ty << A.b;
}

// Forward: SSIM per active pixel and channel; per-block partial sums of SSIM
// and |img - ref|; optionally the per-pixel partials needed by the backward,
// G[m][n] = (d SSIM / d S_m) / Z for m in (sum x, sum x^2, sum xy) x channel.
__global__ __launch_bounds__(256) void k_ssim_fwd(SsimArgs A, const float* __restrict__ img,
                                                  const float* __restrict__ ref, float* __restrict__ smap,
                                                  float* __restrict__ G, float2* __restrict__ part) {
  // one LDS buffer serves first as the gathered patch [7][H*H] and then, once
  // every thread holds its horizontal-pass sums in registers, as the pass
  // output [16][B*H]: 26.6 KB instead of 45.5 KB, so twice the workgroups fit
  constexpr int kIn = SS_MAXH * SS_MAXH, kH = SS_MAXB * SS_MAXH;
  __shared__ float s_buf[16 * kH];
  __shared__ float s_red[2][4];
  const int ct = hp_xcd_tile(blockIdx.x, gridDim.x), tid = threadIdx.x;
  const int B = 1 << A.b, H = B + 2 * SS_R;
  int f, x0, y0;
  ss_tile_origin(A, ct, &f, &x0, &y0);
  for (int i = tid; i < H * H; i += 256) {
    const int cell = ss_cell(i, B, H);
    const int cx = cell % H, cy = cell / H;
    const int64_t slot = ss_slot(A, hp_chart_pixel(A.order, f, x0 + cx - SS_R, y0 + cy - SS_R));
    float m = 0.f, v[6] = {0, 0, 0, 0, 0, 0};
    if (slot >= 0) {
      m = 1.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        v[ch] = img[ch * A.n_active + slot];
        v[3 + ch] = ref[ch * A.n_active + slot];
      }
    }
    s_buf[cell] = m;
#pragma unroll
    for (int k = 0; k < 6; ++k) s_buf[(1 + k) * kIn + cell] = v[k];
  }
  __syncthreads();
  // the centre values of this thread's pixel, for the L1 term
  float xc[3] = {0.f, 0.f, 0.f}, yc[3] = {0.f, 0.f, 0.f};
  const int px = tid % B, py = tid / B;
  if (tid < B * B) {
    const int cc = (py + SS_R) * H + px + SS_R;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      xc[ch] = s_buf[(1 + ch) * kIn + cc];
      yc[ch] = s_buf[(4 + ch) * kIn + cc];
    }
  }
  // pass 1 along x: rows 0..H-1 of the patch, output columns 0..B-1; at most
  // two outputs per thread (B * H <= 416)
  float acc[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[j][k] = 0.f;
    const int pos = tid + 256 * j;
    if (pos < B * H) {
      const int ox = pos % B, row = pos / B;
      // partial unroll: a full one keeps every tap's loads live at once
#pragma unroll 3
      for (int a = 0; a < SS_W; ++a) {
        const int cell = row * H + ox + a;
        const float w = A.g[a] * s_buf[cell];
        acc[j][0] += w;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          const float x = s_buf[(1 + ch) * kIn + cell], y = s_buf[(4 + ch) * kIn + cell];
          acc[j][1 + ch] += w * x;
          acc[j][4 + ch] += w * y;
          acc[j][7 + ch] += w * x * x;
          acc[j][10 + ch] += w * y * y;
          acc[j][13 + ch] += w * x * y;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pos = tid + 256 * j;
    if (pos < B * H) {
#pragma unroll
      for (int k = 0; k < 16; ++k) s_buf[k * kH + pos] = acc[j][k];  // pos = row * B + ox
    }
  }
  __syncthreads();
  float ssum = 0.f, lsum = 0.f;
  if (tid < B * B) {
    float S[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) S[k] = 0.f;
#pragma unroll 3
    for (int bb = 0; bb < SS_W; ++bb) {
      const int idx = (py + bb) * B + px;
#pragma unroll
      for (int k = 0; k < 16; ++k) S[k] += A.g[bb] * s_buf[k * kH + idx];
    }
    const int64_t slot = ss_slot(A, hp_xyf_nest(A.order, x0 + px, y0 + py, f));
    if (slot >= 0) {
      const float iZ = 1.f / S[0];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float mx = S[1 + ch] * iZ, my = S[4 + ch] * iZ;
        const float vx = S[7 + ch] * iZ - mx * mx, vy = S[10 + ch] * iZ - my * my;
        const float cxy = S[13 + ch] * iZ - mx * my;
        const float An = 2.f * mx * my + A.C1, Bn = 2.f * cxy + A.C2;
        const float Ad = mx * mx + my * my + A.C1, Bd = vx + vy + A.C2;
        const float iden = 1.f / (Ad * Bd);
        const float s = An * Bn * iden;
        ssum += s;
        lsum += fabsf(xc[ch] - yc[ch]);
        if (smap) smap[ch * A.n_active + slot] = s;
        if (G) {
          // s(sx, sxx, sxy) with the y sums fixed; sx = mx etc. (normalised)
          const float ds_dmx = (2.f * my * Bn - An * 2.f * my) * iden - s * (2.f * mx / Ad - 2.f * mx / Bd);
          const float ds_dvxx = -s / Bd;
          const float ds_dcxy = 2.f * An * iden;
          G[(0 * 3 + ch) * A.n_active + slot] = ds_dmx * iZ;
          G[(1 * 3 + ch) * A.n_active + slot] = ds_dvxx * iZ;
          G[(2 * 3 + ch) * A.n_active + slot] = ds_dcxy * iZ;
        }
      }
    }
  }
  // block reduction of (ssum, lsum)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ssum += __shfl_xor(ssum, off, 64);
    lsum += __shfl_xor(lsum, off, 64);
  }
  if (hp_lane() == 0) { s_red[0][tid >> 6] = ssum; s_red[1][tid >> 6] = lsum; }
  __syncthreads();
  if (tid == 0)
    part[ct] = make_float2(s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3],
                           s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3]);
}

// single block: mean SSIM, mean L1, loss
__global__ __launch_bounds__(1024) void k_ssim_reduce(const float2* __restrict__ part, int n, int64_t n_active,
                                                      float lam, float* __restrict__ out) {
  __shared__ double s[2][16];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += 1024) { a += part[i].x; b += part[i].y; }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if (hp_lane() == 0) { s[0][threadIdx.x >> 6] = a; s[1][threadIdx.x >> 6] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int k = 0; k < 16; ++k) { sa += s[0][k]; sb += s[1][k]; }
    const double nn = 3.0 * (double)n_active;
    const double ssim = sa / nn, l1 = sb / nn;
    out[0] = (float)ssim;
    out[1] = (float)l1;
    out[2] = (float)((1.0 - lam) * l1 + lam * (1.0 - ssim));
  }
}

// Backward: dL/dimg_p = dL/dloss * [ (1 - lam) sign(img - ref) / (3n)
//   - lam / (3n) * sum_{q in W(p)} g(q - p) (G0_q + 2 x_p G1_q + y_p G2_q) ]
__global__ __launch_bounds__(256) void k_ssim_bwd(SsimArgs A, const float* __restrict__ img,
                                                  const float* __restrict__ ref, const float* __restrict__ G,
                                                  const float* __restrict__ dL_dloss, float* __restrict__ dimg) {
  // the gathered patch [9][H*H] and the horizontal-pass output [9][B*H]
  // share one buffer (pass-1 sums wait in registers across a barrier)
  constexpr int kIn = SS_MAXH * SS_MAXH, kH = SS_MAXB * SS_MAXH;
  __shared__ float s_buf[9 * kIn];
  const int ct = hp_xcd_tile(blockIdx.x, gridDim.x), tid = threadIdx.x;
  const int B = 1 << A.b, H = B + 2 * SS_R;
  int f, x0, y0;
  ss_tile_origin(A, ct, &f, &x0, &y0);
  for (int i = tid; i < H * H; i += 256) {
    const int cell = ss_cell(i, B, H);
    const int cx = cell % H, cy = cell / H;
    const int64_t slot = ss_slot(A, hp_chart_pixel(A.order, f, x0 + cx - SS_R, y0 + cy - SS_R));
#pragma unroll
    for (int k = 0; k < 9; ++k) s_buf[k * kIn + cell] = slot >= 0 ? G[k * A.n_active + slot] : 0.f;
  }
  __syncthreads();
  float acc[2][9];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[j][k] = 0.f;
    const int pos = tid + 256 * j;
    if (pos < B * H) {
      const int ox = pos % B, row = pos / B;
#pragma unroll
      for (int a = 0; a < SS_W; ++a) {
        const int cell = row * H + ox + a;
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[j][k] += A.g[a] * s_buf[k * kIn + cell];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pos = tid + 256 * j;
    if (pos < B * H) {
#pragma unroll
      for (int k = 0; k < 9; ++k) s_buf[k * kH + pos] = acc[j][k];
    }
  }
  __syncthreads();
  if (tid >= B * B) return;
  const int px = tid % B, py = tid / B;
  const int64_t slot = ss_slot(A, hp_xyf_nest(A.order, x0 + px, y0 + py, f));
  if (slot < 0) return;
  float S[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) S[k] = 0.f;
#pragma unroll
  for (int bb = 0; bb < SS_W; ++bb) {
    const int idx = (py + bb) * B + px;
#pragma unroll
    for (int k = 0; k < 9; ++k) S[k] += A.g[bb] * s_buf[k * kH + idx];
  }
  const float up = *dL_dloss;
  const float inv3n = 1.f / (3.f * (float)A.n_active);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const float x = img[ch * A.n_active + slot], y = ref[ch * A.n_active + slot];
    const float dssim = S[0 * 3 + ch] + 2.f * x * S[1 * 3 + ch] + y * S[2 * 3 + ch];
    const float sgn = (float)((x > y) - (x < y));
    dimg[ch * A.n_active + slot] = up * inv3n * ((1.f - A.lam) * sgn - A.lam * dssim);
  }
}

static size_t ssim_ws_size(int64_t n_active, int64_t ntile) {
  return hp_align256((size_t)9 * n_active * 4) + hp_align256((size_t)ntile * sizeof(float2));
}

extern "C" size_t hp_ssim_workspace_bytes(int32_t order, int32_t tile_log2, int64_t n_active) {
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4 || n_active < 0) return 0;
  return ssim_ws_size(n_active, hp_geom(order, tile_log2).ntile);
}

// shared argument checks and set-up of the three entry points
static hp_status ssim_setup(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                            const hp_params* prm, const hp_ssim_params* sp, const void* mask, const void* ws,
                            size_t ws_bytes, SsimArgs* A, float** Gm, float2** part) {
  HP_TRY(hp_check_params(prm));
  if (!sp || !mask || !ws) return HP_ERR_INVALID_ARG;
  if (order < 3 || order > HP_MAX_ORDER) return order < 0 || order > HP_MAX_ORDER ? HP_ERR_INVALID_ARG : HP_ERR_UNSUPPORTED;
  if (n_active <= 0 || n_tiles <= 0 || !img || !ref) return HP_ERR_INVALID_ARG;
  if (!(sp->sigma > 0) || !(sp->C1 > 0) || !(sp->C2 > 0) || !(sp->lambda >= 0 && sp->lambda <= 1))
    return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(order, prm->tile_log2);
  if (n_tiles > g.ntile || n_active > g.npix) return HP_ERR_INVALID_ARG;
  if (ws_bytes < ssim_ws_size(n_active, g.ntile)) return HP_ERR_CAPACITY;
  const HpMaskView mv = hp_mask_view((const char*)mask, g);
  A->order = order; A->b = g.b; A->kt = g.kt;
  A->active_tiles = mv.active_tiles; A->tile_start = mv.tile_start; A->tile_count = mv.tile_count;
  A->tile_bits = mv.tile_bits; A->n_active = n_active;
  A->C1 = sp->C1; A->C2 = sp->C2; A->lam = sp->lambda;
  for (int a = 0; a < SS_W; ++a) {
    const double d = a - SS_R;
    A->g[a] = (float)exp(-d * d / (2.0 * (double)sp->sigma * (double)sp->sigma));
  }
  *Gm = (float*)ws;
  *part = (float2*)((char*)ws + hp_align256((size_t)9 * n_active * 4));
  return HP_OK;
}

static hp_status ssim_fwd_launch(const SsimArgs& A, const float* img, const float* ref, int32_t n_tiles, float lam,
                                 float* out, float* ssim_map, float* Gm, float2* part, hipStream_t s) {
  hipLaunchKernelGGL(k_ssim_fwd, dim3((unsigned)n_tiles), dim3(256), 0, s, A, img, ref, ssim_map, Gm, part);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(1024), 0, s, (const float2*)part, (int)n_tiles, A.n_active, lam, out);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_ssim(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                             const hp_params* prm, const hp_ssim_params* sp, const void* mask, float* out,
                             float* ssim_map, const float* dL_dloss, float* dL_dimg, void* ws, size_t ws_bytes,
                             void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, ws, ws_bytes, &A, &Gm, &part));
  if (!out || (dL_dloss && !dL_dimg)) return HP_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  HP_TRY(ssim_fwd_launch(A, img, ref, n_tiles, sp->lambda, out, ssim_map, dL_dloss ? Gm : nullptr, part, s));
  if (dL_dloss) {
    hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)n_tiles), dim3(256), 0, s, A, img, ref, (const float*)Gm, dL_dloss,
                       dL_dimg);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

extern "C" hp_status hp_ssim_forward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles,
                                           int32_t order, const hp_params* prm, const hp_ssim_params* sp,
                                           const void* mask, float* out, float* ssim_map, void* ws, size_t ws_bytes,
                                           void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, ws, ws_bytes, &A, &Gm, &part));
  if (!out) return HP_ERR_INVALID_ARG;
  return ssim_fwd_launch(A, img, ref, n_tiles, sp->lambda, out, ssim_map, Gm, part, (hipStream_t)stream);
}

extern "C" hp_status hp_ssim_backward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles,
                                            int32_t order, const hp_params* prm, const hp_ssim_params* sp,
                                            const void* mask, const void* ws, size_t ws_bytes,
                                            const float* dL_dloss, float* dL_dimg, void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, ws, ws_bytes, &A, &Gm, &part));
  if (!dL_dloss || !dL_dimg) return HP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, A, img, ref,
                     (const float*)Gm, dL_dloss, dL_dimg);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
