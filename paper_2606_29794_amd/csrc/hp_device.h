// hp_device.h -- device-side building blocks of the HEALPix rasterizer:
// buffer layouts shared by the kernels of this library, HEALPix geometry in
// double precision (Gorski et al. 2005, the grid of Sec. 3.1), the
// face-extended chart used by HEALPix-SSIM (Sec. 4.1) and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hp.h"

#define HP_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// Sizes and layouts
// ---------------------------------------------------------------------------
HP_HD size_t hp_align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct HpGeom {
  int order, b, kt;       // pixel order, log2 tile side, tile order
  int64_t npix, ntile;    // full-sphere pixels and tiles
  int per_tile;           // pixels per tile = 4^b
  int64_t nodes;          // quadtree nodes, levels 0..kt
};

HP_HD HpGeom hp_geom(int order, int tile_log2) {
  HpGeom g;
  g.order = order;
  g.b = tile_log2 < order ? tile_log2 : order;
  g.kt = order - g.b;
  g.npix = 12ll << (2 * order);
  g.ntile = 12ll << (2 * g.kt);
  g.per_tile = 1 << (2 * g.b);
  g.nodes = 12ll * (((int64_t)1 << (2 * (g.kt + 1))) - 1) / 3;
  return g;
}
HP_HD int64_t hp_level_offset(int level) { return 12ll * (((int64_t)1 << (2 * level)) - 1) / 3; }

// grid buffer: node caps (float4: centre xyz, radius) then (sin, cos) of half radius
struct HpGridView {
  float4* cap;
  float2* sc;
};
HP_HD size_t hp_grid_size(const HpGeom& g) { return hp_align256(g.nodes * sizeof(float4)) + hp_align256(g.nodes * sizeof(float2)); }
HP_HD HpGridView hp_grid_view(void* base, const HpGeom& g) {
  HpGridView v;
  char* p = (char*)base;
  v.cap = (float4*)p;
  v.sc = (float2*)(p + hp_align256(g.nodes * sizeof(float4)));
  return v;
}

// mask buffer
struct HpMaskView {
  int64_t* n_active;
  int32_t* n_tiles;
  int32_t* tile_start;    // [ntile] first compact pixel slot of the tile
  int32_t* tile_count;    // [ntile] active pixels in the tile
  int32_t* tile_compact;  // [ntile] compact active tile id or -1
  uint32_t* tile_bits;    // [ntile][8] membership of the tile's pixels (nested order)
  int32_t* active_tiles;  // [ntile] compact id -> tile
  uint8_t* node_active;   // [nodes]
  int32_t* active_pix;    // [npix]
};
HP_HD size_t hp_mask_size(const HpGeom& g) {
  size_t s = 256;
  s += 4 * hp_align256(g.ntile * 4);
  s += hp_align256(g.ntile * 32);
  s += hp_align256(g.nodes);
  s += hp_align256(g.npix * 4);
  return s;
}
template <class P>
HP_HD HpMaskView hp_mask_view(P* base, const HpGeom& g) {
  HpMaskView v;
  char* p = (char*)base;
  v.n_active = (int64_t*)p;
  v.n_tiles = (int32_t*)(p + 8);
  p += 256;
  size_t t4 = hp_align256(g.ntile * 4);
  v.tile_start = (int32_t*)p; p += t4;
  v.tile_count = (int32_t*)p; p += t4;
  v.tile_compact = (int32_t*)p; p += t4;
  v.active_tiles = (int32_t*)p; p += t4;
  v.tile_bits = (uint32_t*)p; p += hp_align256(g.ntile * 32);
  v.node_active = (uint8_t*)p; p += hp_align256(g.nodes);
  v.active_pix = (int32_t*)p;
  return v;
}

// projected buffer: 64-byte record per Gaussian, then depth and radius
//   r0 = (u_x, u_y, u_z, opacity)    unit camera-frame direction
//   r1 = (eo_x, eo_z, ep_x, ep_y)    tangent frame: e_omega = (eo_x, 0, eo_z)
//   r2 = (ep_z, A, B, C)             e_phi = (ep_x, ep_y, ep_z); q = A a^2 + 2 B a b + C b^2
//   r3 = (red, green, blue, sin((r_s + bin_guard) / 2))   the last entry drives the binning
// projected buffer: the 64-byte records, depth [P], radius [P], and disc [P]
// (unit direction, sin of half the tile-test angle r_s + guard: the 16 bytes
// the binning reads, apart from the records so that its gathers share lines)
struct HpProjView {
  float4* rec;
  float* depth;
  float* radius;
  float4* disc;
};
HP_HD size_t hp_proj_size(int64_t P) { return hp_align256(P * 64) + 2 * hp_align256(P * 4) + hp_align256(P * 16); }
template <class T>
HP_HD HpProjView hp_proj_view(T* base, int64_t P) {
  HpProjView v;
  char* p = (char*)base;
  v.rec = (float4*)p;
  v.depth = (float*)(p + hp_align256(P * 64));
  v.radius = (float*)(p + hp_align256(P * 64) + hp_align256(P * 4));
  v.disc = (float4*)(p + hp_align256(P * 64) + 2 * hp_align256(P * 4));
  return v;
}

// ---------------------------------------------------------------------------
// HEALPix NESTED geometry (double precision)
// ---------------------------------------------------------------------------
// bits of x at even positions, bits of y at odd positions
HP_HD uint32_t hp_compact_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}
HP_HD uint32_t hp_spread_bits(uint32_t v) {
  v &= 0x0000ffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
HP_HD void hp_nest_xyf(int order, int64_t p, int* x, int* y, int* f) {
  int64_t npf = (int64_t)1 << (2 * order);
  *f = (int)(p / npf);
  uint32_t q = (uint32_t)(p - (int64_t)(*f) * npf);
  *x = (int)hp_compact_bits(q);
  *y = (int)hp_compact_bits(q >> 1);
}
HP_HD int64_t hp_xyf_nest(int order, int x, int y, int f) {
  return ((int64_t)f << (2 * order)) + (int64_t)(hp_spread_bits((uint32_t)x) | (hp_spread_bits((uint32_t)y) << 1));
}

// Pixel-centre direction in the camera frame (pole = camera +y, longitude
// omega = atan2(t_x, t_z)): t = (sin(theta) sin(phi), z, sin(theta) cos(phi)).
// Face f: row f/4 sets the ring of the face's southern corner (rows 2, 3, 4
// in units of Nside); column f%4 sets its longitude (odd multiples of pi/4 for
// the polar rows, multiples of pi/2 for the equatorial row).
__device__ __forceinline__ void hp_pix_dir(int order, int64_t p, double* t) {
  int x, y, f;
  hp_nest_xyf(order, p, &x, &y, &f);
  const int64_t N = (int64_t)1 << order;
  const int row = f >> 2, col = f & 3;
  const int64_t ring = (int64_t)(row + 2) * N - x - y - 1;   // 1 .. 4N-1 from the north pole
  const int64_t lon_units = (row == 1) ? 2 * col : 2 * col + 1; // face centre longitude in pi/4
  double z, sth, phi;
  if (ring < N || ring > 3 * N) {
    const int64_t nr = ring < N ? ring : 4 * N - ring;        // ring index counted from its pole
    const double tmp = (double)(nr * nr) / (3.0 * (double)(N * N));
    z = ring < N ? 1.0 - tmp : tmp - 1.0;
    sth = sqrt(tmp * (2.0 - tmp));
    // position along the ring: nr pixels per face, centred on the face longitude
    int64_t jp = (lon_units * nr + x - y + 1) / 2;           // 1-based within ring (may wrap)
    phi = ((double)jp - 0.5) * (M_PI / 2.0) / (double)nr;
  } else {
    z = (double)(2 * N - ring) * (2.0 / (3.0 * (double)N));
    sth = sqrt((1.0 - z) * (1.0 + z));
    const int s = (int)((ring - N) & 1);
    int64_t jp = (lon_units * N + x - y + 1 + s) / 2;
    phi = ((double)jp - 0.5 * (1 + s)) * (M_PI / 2.0) / (double)N;
  }
  double sp, cp;
  sincos(phi, &sp, &cp);
  t[0] = sth * sp;
  t[1] = z;
  t[2] = sth * cp;
}

// ---------------------------------------------------------------------------
// Face-extended chart (HEALPix-SSIM neighbourhoods, Sec. 4.1).
// A face-local offset that leaves face f across one edge lands in the
// neighbouring face with its axes turned to line up; across a corner it lands
// in the diagonally opposite face only at four-face vertices (the poles and
// the equatorial corners); at the eight three-face vertices the diagonal
// quadrant does not exist.  Each case is an affine map
//   X = ax x + bx y + kx N + lx,  Y = ay x + by y + ky N + ly
// into face  base + (col + dcol) % 4  (dcol < 0: missing).
// ---------------------------------------------------------------------------
struct HpChartXf {
  int8_t base, dcol, ax, bx, kx, lx, ay, by, ky, ly;
};
// index: row*8 + dir, dir over (sx, sy) in order
// (+1,0) (-1,0) (0,+1) (0,-1) (+1,+1) (-1,-1) (+1,-1) (-1,+1)
__constant__ static const HpChartXf kHpChart[24] = {
    // north row
    {0, 1, 0, 1, 0, 0, -1, 0, 2, -1},   // +x: next polar face, turned
    {4, 0, 1, 0, 1, 0, 0, 1, 0, 0},     // -x: equatorial face below-west
    {0, 3, 0, -1, 2, -1, 1, 0, 0, 0},   // +y: previous polar face, turned
    {4, 1, 1, 0, 0, 0, 0, 1, 1, 0},     // -y: equatorial face below-east
    {0, 2, -1, 0, 2, -1, 0, -1, 2, -1}, // +x+y: across the pole
    {8, 0, 1, 0, 1, 0, 0, 1, 1, 0},     // -x-y: south face across the equatorial vertex
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},    // three-face vertex
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    // equatorial row
    {0, 0, 1, 0, -1, 0, 0, 1, 0, 0},    // +x: polar face above-east
    {8, 3, 1, 0, 1, 0, 0, 1, 0, 0},     // -x: south face below-west
    {0, 3, 1, 0, 0, 0, 0, 1, -1, 0},    // +y: polar face above-west
    {8, 0, 1, 0, 0, 0, 0, 1, 1, 0},     // -y: south face below-east
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},    // +x+y: three-face vertex (north)
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},    // -x-y: three-face vertex (south)
    {4, 1, 1, 0, -1, 0, 0, 1, 1, 0},    // +x-y: next equatorial face
    {4, 3, 1, 0, 1, 0, 0, 1, -1, 0},    // -x+y: previous equatorial face
    // south row
    {4, 1, 1, 0, -1, 0, 0, 1, 0, 0},    // +x: equatorial face above-east
    {8, 3, 0, 1, 0, 0, -1, 0, 0, -1},   // -x: previous polar face, turned
    {4, 0, 1, 0, 0, 0, 0, 1, -1, 0},    // +y: equatorial face above-west
    {8, 1, 0, -1, 0, -1, 1, 0, 0, 0},   // -y: next polar face, turned
    {0, 0, 1, 0, -1, 0, 0, 1, -1, 0},   // +x+y: north face across the equatorial vertex
    {8, 2, -1, 0, 0, -1, 0, -1, 0, -1}, // -x-y: across the south pole
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, -1, 0, 0, 0, 0, 0, 0, 0, 0},
};

// Nested pixel at face-local (x, y) of face f (x, y may be outside [0, N) by
// less than N), or -1 where the chart has no pixel.
__device__ __forceinline__ int64_t hp_chart_pixel(int order, int f, int x, int y) {
  const int N = 1 << order;
  const int sx = x < 0 ? -1 : (x >= N ? 1 : 0);
  const int sy = y < 0 ? -1 : (y >= N ? 1 : 0);
  if (sx == 0 && sy == 0) return hp_xyf_nest(order, x, y, f);
  int dir;
  if (sy == 0) dir = sx > 0 ? 0 : 1;
  else if (sx == 0) dir = sy > 0 ? 2 : 3;
  else if (sx == sy) dir = sx > 0 ? 4 : 5;
  else dir = sx > 0 ? 6 : 7;
  const HpChartXf m = kHpChart[(f >> 2) * 8 + dir];
  if (m.dcol < 0) return -1;
  const int g = m.base + (((f & 3) + m.dcol) & 3);
  const int X = m.ax * x + m.bx * y + m.kx * N + m.lx;
  const int Y = m.ay * x + m.by * y + m.ky * N + m.ly;
  if (X < 0 || X >= N || Y < 0 || Y >= N) return -1;
  return hp_xyf_nest(order, X, Y, g);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int hp_lane() { return (int)__lane_id(); }

// Read-only data addressed by a wave-uniform index: reading through the
// constant address space lets the compiler use scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) float* hp_cfloatp;
typedef const __attribute__((address_space(4))) uint32_t* hp_cu32p;
// the 64-byte record of Gaussian g (see HpProjView) as four float4
__device__ __forceinline__ void hp_load_rec(hp_cfloatp rec, uint32_t g, float4& r0, float4& r1, float4& r2,
                                            float4& r3) {
  const hp_cfloatp p = rec + 16 * (int64_t)g;
  r0 = make_float4(p[0], p[1], p[2], p[3]);
  r1 = make_float4(p[4], p[5], p[6], p[7]);
  r2 = make_float4(p[8], p[9], p[10], p[11]);
  r3 = make_float4(p[12], p[13], p[14], p[15]);
}
__device__ __forceinline__ uint32_t hp_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroups go to the 8 XCDs round-robin by index.  Giving each XCD a
// contiguous range of tiles keeps neighbouring tiles, which share most of
// their data, in the same L2.  A bijection of [0, nb).
__device__ __forceinline__ int hp_xcd_tile(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

template <int CTRL>
__device__ __forceinline__ float hp_dpp(float v) {
  // every source lane of the patterns used here is inside the row, so the
  // bound control setting never applies; it allows fusing into the add
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
// Sums over the 64 lanes of N values at once (all lanes active), wave-uniform
// results: quad butterflies and row mirrors give each 16-lane row its sum,
// then the four row sums are read out and added.  The N reductions advance
// step by step so that independent DPP operations interleave.
template <int N>
__device__ __forceinline__ void hp_wave_totals(float* v) {
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0xB1>(v[m]);   // quad_perm [1,0,3,2]: lane ^ 1
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x4E>(v[m]);   // quad_perm [2,3,0,1]: lane ^ 2
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x141>(v[m]);  // row_half_mirror: quads of a half-row
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x140>(v[m]);  // row_mirror: half-rows of a row
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int x = __float_as_int(v[m]);
    v[m] = (__int_as_float(__builtin_amdgcn_readlane(x, 0)) + __int_as_float(__builtin_amdgcn_readlane(x, 16))) +
           (__int_as_float(__builtin_amdgcn_readlane(x, 32)) + __int_as_float(__builtin_amdgcn_readlane(x, 48)));
  }
}

// Same sums, left in lane 63 only: after the row sums, row_bcast:15 adds
// row r-1's sum into rows 1 and 3, and row_bcast:31 adds lane 31 (rows 0+1)
// into rows 2 and 3, so lane 63 ends with the total of the wave.
template <int N>
__device__ __forceinline__ void hp_wave_totals_lane63(float* v) {
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0xB1>(v[m]);
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x4E>(v[m]);
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x141>(v[m]);
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] += hp_dpp<0x140>(v[m]);
#pragma unroll
  for (int m = 0; m < N; ++m)
    v[m] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[m]), 0x142, 0xa, 0xf, false));
#pragma unroll
  for (int m = 0; m < N; ++m)
    v[m] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[m]), 0x143, 0xc, 0xf, false));
}

// Eight sums over the 64 lanes at once by recursive halving: every exchange
// step moves half of the remaining values to the partner lane group, so the
// 8 x 64 inputs need 4 + 2 + 1 cross-lane moves plus three butterfly adds
// instead of 8 x 6.  gfx950's permlane32 swap pairs lane L with L ^ 32 and
// permlane16 swap pairs L with L ^ 16; a row rotation by 8 pairs L with L ^ 8.
// On return, lane L holds the total of value L >> 3 in all eight lanes of its
// group (L & ~7 .. L | 7).
__device__ __forceinline__ float hp_wave_totals8_spread(const float* v) {
  float w[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    // low half keeps value m, high half keeps value m + 4
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[m]), __float_as_uint(v[m + 4]), false, false);
    w[m] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  float x[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    // even rows keep w[m], odd rows keep w[m + 2]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[m]), __float_as_uint(w[m + 2]), false, false);
    x[m] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // lanes with bit 3 clear keep x[0] and take x[0] of lane L ^ 8; the others
  // keep x[1] and take x[1] of lane L ^ 8
  const bool hi = (hp_lane() & 8) != 0;
  const float send = hi ? x[0] : x[1];
  const float keep = hi ? x[1] : x[0];
  float y = keep + hp_dpp<0x128>(send);  // row_ror:8
  y += hp_dpp<0xB1>(y);
  y += hp_dpp<0x4E>(y);
  y += hp_dpp<0x141>(y);
  return y;
}

// A ninth sum beside hp_wave_totals8_spread: the same exchanges applied to
// one value alone (each swap pairs the value with itself), so every lane ends
// with the wave's total.
__device__ __forceinline__ float hp_wave_total_all(float z) {
  {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(z), __float_as_uint(z), false, false);
    z = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(z), __float_as_uint(z), false, false);
    z = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  z += hp_dpp<0x128>(z);  // row_ror:8
  z += hp_dpp<0xB1>(z);
  z += hp_dpp<0x4E>(z);
  z += hp_dpp<0x141>(z);
  return z;
}

__device__ __forceinline__ float hp_wave_sum(float v) {
  // butterfly over 64 lanes with cross-lane shuffles
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint32_t hp_wave_prefix_u32(uint32_t v, uint32_t* total) {
  // inclusive scan across the wave, returns exclusive; total in *total
  uint32_t x = v;
  const int lane = hp_lane();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}
