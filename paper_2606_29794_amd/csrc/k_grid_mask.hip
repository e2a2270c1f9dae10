// k_grid_mask.hip -- HEALPix grid tables (tile and quadtree caps) and the
// camera visibility mask M_C of Sec. 3.1.
#include "hp_common.h"

// ---------------------------------------------------------------------------
// Grid: leaf caps (one block per tile, one thread per pixel)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_leaf(int order, int b, float4* cap, float2* sc, int64_t leaf_off) {
  const int64_t t = blockIdx.x;
  const int per = 1 << (2 * b);
  const int tid = threadIdx.x;
  __shared__ double red[4][3];
  __shared__ double cen[3];
  __shared__ double rmax[4];
  double v[3] = {0, 0, 0};
  if (tid < per) hp_pix_dir(order, t * per + tid, v);
  double s0 = v[0], s1 = v[1], s2 = v[2];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
  }
  const int w = tid >> 6;
  if (hp_lane() == 0) { red[w][0] = s0; red[w][1] = s1; red[w][2] = s2; }
  __syncthreads();
  if (tid == 0) {
    double c0 = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    double c1 = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    double c2 = red[0][2] + red[1][2] + red[2][2] + red[3][2];
    double n = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    cen[0] = c0 / n; cen[1] = c1 / n; cen[2] = c2 / n;
  }
  __syncthreads();
  double a = 0;
  if (tid < per) {
    double cx = cen[1] * v[2] - cen[2] * v[1], cy = cen[2] * v[0] - cen[0] * v[2], cz = cen[0] * v[1] - cen[1] * v[0];
    a = atan2(sqrt(cx * cx + cy * cy + cz * cz), cen[0] * v[0] + cen[1] * v[1] + cen[2] * v[2]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a = fmax(a, __shfl_xor(a, off, 64));
  if (hp_lane() == 0) rmax[w] = a;
  __syncthreads();
  if (tid == 0) {
    double R = fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3]));
    float Rf = hp_round_up_f(R);
    cap[leaf_off + t] = make_float4((float)cen[0], (float)cen[1], (float)cen[2], Rf);
    sc[leaf_off + t] = make_float2((float)sin(0.5 * (double)Rf), (float)cos(0.5 * (double)Rf));
  }
}

// Internal node at `level` from its 4 children at level+1: centre = normalised
// sum of child centres, radius covering the child caps plus a slack that keeps
// float32 pruning conservative.
__global__ void k_grid_up(int level, float4* cap, float2* sc) {
  const int64_t n = 12ll << (2 * level);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t off = hp_level_offset(level), coff = hp_level_offset(level + 1);
  double c[3] = {0, 0, 0};
  float4 ch[4];
  for (int k = 0; k < 4; ++k) {
    ch[k] = cap[coff + 4 * i + k];
    c[0] += ch[k].x; c[1] += ch[k].y; c[2] += ch[k].z;
  }
  double nn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  c[0] /= nn; c[1] /= nn; c[2] /= nn;
  double R = 0;
  for (int k = 0; k < 4; ++k) {
    double v[3] = {ch[k].x, ch[k].y, ch[k].z};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double cx = c[1] * v[2] - c[2] * v[1], cy = c[2] * v[0] - c[0] * v[2], cz = c[0] * v[1] - c[1] * v[0];
    double a = atan2(sqrt(cx * cx + cy * cy + cz * cz), (c[0] * v[0] + c[1] * v[1] + c[2] * v[2])) ;
    (void)vn;
    R = fmax(R, a + (double)ch[k].w);
  }
  R += 2e-5;
  float Rf = hp_round_up_f(R);
  cap[off + i] = make_float4((float)c[0], (float)c[1], (float)c[2], Rf);
  sc[off + i] = make_float2((float)sin(0.5 * fmin((double)Rf, M_PI)), (float)cos(0.5 * fmin((double)Rf, M_PI)));
}

extern "C" size_t hp_grid_bytes(int32_t order, int32_t tile_log2) {
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4) return 0;
  return hp_grid_size(hp_geom(order, tile_log2));
}

extern "C" hp_status hp_grid_init(int32_t order, const hp_params* prm, void* grid, size_t grid_bytes, void* stream) {
  if (!prm || !grid) return HP_ERR_INVALID_ARG;
  if (order < 0 || order > HP_MAX_ORDER || prm->tile_log2 < 0 || prm->tile_log2 > 4) return HP_ERR_INVALID_ARG;
  HpGeom g = hp_geom(order, prm->tile_log2);
  if (grid_bytes < hp_grid_size(g)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  HpGridView v = hp_grid_view(grid, g);
  hipLaunchKernelGGL(k_grid_leaf, dim3((unsigned)g.ntile), dim3(256), 0, s, order, g.b, v.cap, v.sc, hp_level_offset(g.kt));
  HP_CHECK_LAUNCH();
  for (int l = g.kt - 1; l >= 0; --l) {
    int64_t n = 12ll << (2 * l);
    hipLaunchKernelGGL(k_grid_up, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, l, v.cap, v.sc);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

// ---------------------------------------------------------------------------
// Mask
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool hp_in_view(int cam, double fx, double fy, const double* t) {
  if (cam == HP_CAM_FULL) return true;
  if (cam == HP_CAM_FISHEYE) {
    // equidistant: incident angle psi from +z; elliptical FoV via w_eff(gamma)
    const double psi = acos(fmin(1.0, fmax(-1.0, t[2])));
    const double rho = sqrt(t[0] * t[0] + t[1] * t[1]);
    double cg = 1.0, sg = 0.0;
    if (rho > 0) { cg = t[0] / rho; sg = t[1] / rho; }
    const double wx = fx / M_PI, wy = fy / M_PI;
    const double weff = sqrt((wx * cg) * (wx * cg) + (wy * sg) * (wy * sg));
    return psi <= 0.5 * M_PI * weff;
  }
  if (!(t[2] > 0)) return false;
  return fabs(t[0]) <= tan(0.5 * fx) * t[2] && fabs(t[1]) <= tan(0.5 * fy) * t[2];
}

// one block per tile: membership bits and count
__global__ __launch_bounds__(256) void k_mask_tiles(int order, int b, int cam, double fx, double fy, uint32_t* bits,
                                                    int32_t* count) {
  const int64_t t = blockIdx.x;
  const int per = 1 << (2 * b);
  const int tid = threadIdx.x;
  bool in = false;
  if (tid < per) {
    if (cam == HP_CAM_FULL) in = true;
    else {
      double v[3];
      hp_pix_dir(order, t * per + tid, v);
      in = hp_in_view(cam, fx, fy, v);
    }
  }
  const uint64_t m = __ballot(in);
  __shared__ int cnt[4];
  const int w = tid >> 6;
  if (hp_lane() == 0) {
    bits[t * 8 + 2 * w] = (uint32_t)m;
    bits[t * 8 + 2 * w + 1] = (uint32_t)(m >> 32);
    cnt[w] = __popcll(m);
  }
  __syncthreads();
  if (tid == 0) count[t] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// single block: exclusive scans of tile counts (pixel slots) and of the
// active-tile flags (compact ids); totals to the header
__global__ __launch_bounds__(1024) void k_mask_scan(int64_t ntile, const int32_t* count, int32_t* start,
                                                    int32_t* compact, int32_t* active_tiles, int64_t* n_active,
                                                    int32_t* n_tiles) {
  __shared__ int64_t s_pix[1024];
  __shared__ int32_t s_til[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (ntile + 1023) / 1024;
  const int64_t lo = tid * chunk, hi = lo + chunk < ntile ? lo + chunk : ntile;
  int64_t sp = 0; int32_t st = 0;
  for (int64_t i = lo; i < hi; ++i) { sp += count[i]; st += count[i] > 0; }
  s_pix[tid] = sp; s_til[tid] = st;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t a = tid >= off ? s_pix[tid - off] : 0;
    int32_t c = tid >= off ? s_til[tid - off] : 0;
    __syncthreads();
    s_pix[tid] += a; s_til[tid] += c;
    __syncthreads();
  }
  int64_t bp = s_pix[tid] - sp;
  int32_t bt = s_til[tid] - st;
  for (int64_t i = lo; i < hi; ++i) {
    start[i] = (int32_t)bp;
    if (count[i] > 0) { compact[i] = bt; active_tiles[bt] = (int32_t)i; ++bt; }
    else compact[i] = -1;
    bp += count[i];
  }
  if (tid == 1023) { *n_active = s_pix[1023]; *n_tiles = s_til[1023]; }
}

__global__ __launch_bounds__(256) void k_mask_pix(int b, const uint32_t* bits, const int32_t* start, int32_t* out) {
  const int64_t t = blockIdx.x;
  const int per = 1 << (2 * b);
  const int tid = threadIdx.x;
  if (tid >= per) return;
  const uint32_t word = bits[t * 8 + (tid >> 5)];
  if (!((word >> (tid & 31)) & 1u)) return;
  int rank = __popc(word & ((1u << (tid & 31)) - 1u));
  for (int k = 0; k < (tid >> 5); ++k) rank += __popc(bits[t * 8 + k]);
  out[start[t] + rank] = (int32_t)(t * per + tid);
}

__global__ void k_mask_nodes_leaf(int64_t ntile, const int32_t* count, uint8_t* node_active, int64_t leaf_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntile) node_active[leaf_off + i] = count[i] > 0;
}
__global__ void k_mask_nodes_up(int level, uint8_t* node_active) {
  const int64_t n = 12ll << (2 * level);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = hp_level_offset(level + 1) + 4 * i;
  node_active[hp_level_offset(level) + i] = node_active[c] | node_active[c + 1] | node_active[c + 2] | node_active[c + 3];
}

extern "C" size_t hp_mask_bytes(int32_t order, int32_t tile_log2) {
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4) return 0;
  return hp_mask_size(hp_geom(order, tile_log2));
}

extern "C" hp_status hp_mask(const hp_view* view, const hp_params* prm, const void* grid, void* mask,
                             size_t mask_bytes, void* stream) {
  if (!view || !prm || !mask) return HP_ERR_INVALID_ARG;
  (void)grid;
  HP_TRY(hp_check_view(view, prm));
  HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (mask_bytes < hp_mask_size(g)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  HpMaskView m = hp_mask_view(mask, g);
  hipLaunchKernelGGL(k_mask_tiles, dim3((unsigned)g.ntile), dim3(256), 0, s, g.order, g.b, view->cam_type,
                     (double)view->fov_x, (double)view->fov_y, m.tile_bits, m.tile_count);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_mask_scan, dim3(1), dim3(1024), 0, s, g.ntile, m.tile_count, m.tile_start, m.tile_compact,
                     m.active_tiles, m.n_active, m.n_tiles);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_mask_pix, dim3((unsigned)g.ntile), dim3(256), 0, s, g.b, m.tile_bits, m.tile_start, m.active_pix);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_mask_nodes_leaf, dim3((unsigned)((g.ntile + 255) / 256)), dim3(256), 0, s, g.ntile, m.tile_count,
                     m.node_active, hp_level_offset(g.kt));
  HP_CHECK_LAUNCH();
  for (int l = g.kt - 1; l >= 0; --l) {
    int64_t n = 12ll << (2 * l);
    hipLaunchKernelGGL(k_mask_nodes_up, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, l, m.node_active);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

extern "C" hp_status hp_mask_counts(const void* mask, int32_t order, int32_t tile_log2, int64_t* n_active,
                                    int32_t* n_tiles, void* stream) {
  if (!mask || !n_active || !n_tiles) return HP_ERR_INVALID_ARG;
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4) return HP_ERR_INVALID_ARG;
  HpMaskView m = hp_mask_view((const char*)mask, hp_geom(order, tile_log2));
  hipStream_t s = (hipStream_t)stream;
  // n_active (int64) and n_tiles (int32) lead the mask's header
  static_assert(sizeof(int64_t) == 8, "header layout");
  char head[16];
  HP_TRY(hp_read_small(head, m.n_active, 16, s));
  int64_t a; int32_t t;
  memcpy(&a, head, 8);
  memcpy(&t, head + ((const char*)m.n_tiles - (const char*)m.n_active), 4);
  *n_active = a; *n_tiles = t;
  return HP_OK;
}

extern "C" const int32_t* hp_mask_active_pix(const void* mask, int32_t order, int32_t tile_log2) {
  if (!mask || order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4) return nullptr;
  return hp_mask_view((const char*)mask, hp_geom(order, tile_log2)).active_pix;
}
