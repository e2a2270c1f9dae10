// k_ssim.hip -- HEALPix-SSIM and the training loss of Sec. 4.1.
//
// One workgroup per active tile.  The tile's B x B pixels plus a 5-pixel halo
// are gathered into LDS through the face-extended chart (neighbouring faces
// with their axes turned to line up; the missing quadrant of a three-face
// vertex and inactive pixels carry weight 0).  Dividing the window sums by
// the summed weight renormalises where neighbours are missing.
//
// Windows.  The isotropic chart window exp(-(a^2 + b^2) / (2 sigma^2)) is
// separable on the patch: two 11-tap passes, each thread sliding the window
// along a strip held in registers (one LDS read per input value, four or
// eight outputs per strip).  With zone-specific windows, a pixel of a polar
// cap weighs its neighbours by great-circle distance instead,
// exp(-d^2 / (2 sigma^2 Omega)), Omega = 4 pi / Npix, which is not separable:
// tiles holding such pixels take a direct 121-tap path with the pixel-centre
// directions in LDS.
//
// The backward pass is the transposed window: the chart neighbourhood
// relation is symmetric with equal offset lengths, so the adjoint gathers the
// per-pixel SSIM partials over the same window, each neighbour's partials
// weighted by that neighbour's own window at the pixel.
#include "hp_common.h"

#define SS_R 5
#define SS_W 11

// patch table entries: compact slot, bit 30 set for a polar-cap pixel, -1
// for a missing or inactive neighbour
constexpr int32_t kSsPolarBit = 1 << 30;
constexpr int32_t kSsSlotMask = kSsPolarBit - 1;
// the backward's per-pixel partials: 9 floats at a 12-float (48-byte) stride
constexpr int kSsG = 12;

struct SsimArgs {
  int order, b, kt;
  const int32_t* active_tiles;
  const int32_t* tile_start;
  const int32_t* tile_count;
  const uint32_t* tile_bits;
  int64_t n_active;
  float C1, C2, lam;
  float g[SS_W];   // chart window taps exp(-a^2 / (2 sigma^2)), a = -5..5
  float gsum;      // their sum, accumulated in the order of the passes
  double wscale;   // 1 / (2 sigma^2 Omega): polar windows are exp(-d^2 wscale)
  const int32_t* tables;  // [n_tiles][H*H] patch slots (see k_ssim_tables)
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

// polar cap pixel: ring jr = jrll(f) N - x - y - 1 outside [N, 3N]
__device__ __forceinline__ bool ss_polar(int order, int64_t q) {
  int x, y, f;
  hp_nest_xyf(order, q, &x, &y, &f);
  const int N = 1 << order;
  return f < 4 ? (x + y >= N) : (f >= 8 ? (x + y <= N - 2) : false);
}

// Patch cell (x, y) of gather index i (a bijection of [0, H*H)): the first
// B*B indices are the tile's own pixels in NESTED order, which a fully
// active tile stores contiguously (coalesced loads), the rest the halo row by
// row.
template <int B>
__device__ __forceinline__ void ss_cell(int i, int* cx, int* cy) {
  constexpr int H = B + 2 * SS_R;
  if (i < B * B) {
    *cx = (int)hp_compact_bits((uint32_t)i) + SS_R;
    *cy = (int)hp_compact_bits((uint32_t)i >> 1) + SS_R;
    return;
  }
  int h = i - B * B;
  if (h < SS_R * H) { *cy = h / H; *cx = h % H; return; }  // rows above the tile
  h -= SS_R * H;
  if (h < 2 * SS_R * B) {  // left and right of the tile's rows
    *cy = SS_R + h / (2 * SS_R);
    const int c = h % (2 * SS_R);
    *cx = c < SS_R ? c : c + B;
    return;
  }
  h -= 2 * SS_R * B;
  *cy = SS_R + B + h / H;  // rows below
  *cx = h % H;
}

__device__ __forceinline__ void ss_tile_origin(const SsimArgs& A, int ct, int* f, int* x0, int* y0) {
  const int t = A.active_tiles[ct];
  int tx, ty;
  hp_nest_xyf(A.kt, t, &tx, &ty, f);
  *x0 = tx << A.b;
  *y0 = ty << A.b;
}

// squared great-circle distance between unit vectors u, v (double):
// d = 2 asin(s), s = |u - v| / 2; d^2 = 4 s^2 (asin s / s)^2, the factor as
// its series in s^2 below s^2 = 1/16 (truncation < 1e-9), asin beyond
__device__ __forceinline__ double ss_dist2(const double* u, const double* v) {
  const double dx = u[0] - v[0], dy = u[1] - v[1], dz = u[2] - v[2];
  const double c2 = dx * dx + dy * dy + dz * dz;
  const double s2 = 0.25 * c2;
  if (s2 < 0.0625) {
    const double k = 1.0 + s2 * (1.0 / 3.0 + s2 * (8.0 / 45.0 + s2 * (4.0 / 35.0 + s2 * (128.0 / 1575.0 +
                     s2 * (128.0 / 2079.0 + s2 * (1024.0 / 21021.0))))));
    return c2 * k;
  }
  const double d = 2.0 * asin(fmin(1.0, sqrt(s2)));
  return d * d;
}

// SSIM of one pixel and channel from its normalised window moments, and the
// partials of the backward: d SSIM / d (sum x, sum x^2, sum xy) / Z
__device__ __forceinline__ float ss_index(float C1, float C2, float iZ, float Sx, float Sy, float Sxx, float Syy,
                                          float Sxy, float* G0, float* G1, float* G2) {
  const float mx = Sx * iZ, my = Sy * iZ;
  const float vx = Sxx * iZ - mx * mx, vy = Syy * iZ - my * my;
  const float cxy = Sxy * iZ - mx * my;
  const float An = 2.f * mx * my + C1, Bn = 2.f * cxy + C2;
  const float Ad = mx * mx + my * my + C1, Bd = vx + vy + C2;
  // reciprocals to 1 ulp (v_rcp_f32) instead of IEEE divisions
  const float iAd = __builtin_amdgcn_rcpf(Ad), iBd = __builtin_amdgcn_rcpf(Bd);
  const float iden = iAd * iBd;
  const float s = An * Bn * iden;
  // s(sx, sxx, sxy) with the y sums fixed; sx = mx etc. (normalised)
  const float ds_dmx = (2.f * my * Bn - An * 2.f * my) * iden - s * (2.f * mx * iAd - 2.f * mx * iBd);
  *G0 = ds_dmx * iZ;
  *G1 = (-s * iBd) * iZ;
  *G2 = (2.f * An * iden) * iZ;
  return s;
}

// nested index of patch-interior pixel (x, y) of a tile: x bits at even
// positions, y bits at odd ones
__device__ __forceinline__ int ss_nest_local(int x, int y) {
  auto spread = [](uint32_t v) {
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
  };
  return (int)(spread((uint32_t)x) | (spread((uint32_t)y) << 1));
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// LDS: the gathered patch (mask, x[3], y[3]), the first pass's output
// [16][H][B] (or, on the direct path, the cells' directions), then the
// second pass's output [16][B*B] over the patch's place.
template <int B>
struct SsFwdLds {
  // row pitch HP: 16-byte aligned rows for the strip loads; P1S: the pass-1
  // output's quantity stride, 16 mod 32 words so that the two quantities a
  // half-wave reads in the second pass fall in different banks
  static constexpr int H = B + 2 * SS_R, HP = (H + 3) & ~3, P1S = H * B + ((48 - (H * B) % 32) % 32);
  float in[7][H][HP];
  union {
    float p1[16][P1S];
    double dir[H * H][3];
  };
};

// Forward: SSIM per active pixel and channel; per-block partial sums of SSIM
// and |img - ref|; optionally the per-pixel partials needed by the backward,
// G[m][n] = (d SSIM / d S_m) / Z for m in (sum x, sum x^2, sum xy) x channel.
template <int B, bool ZONES>
__global__ __launch_bounds__(256) void k_ssim_fwd(SsimArgs A, const float* __restrict__ img,
                                                  const float* __restrict__ ref, float* __restrict__ smap,
                                                  float* __restrict__ G, float2* __restrict__ part, int n_tiles) {
  using L = SsFwdLds<B>;
  constexpr int H = L::H;
  __shared__ L s;
  __shared__ float s_red[2][4];
  float(*S)[B * B] = reinterpret_cast<float(*)[B * B]>(&s.in[0][0][0]);  // after pass 1
  const int tid = threadIdx.x;
  constexpr int NG = (H * H + 255) / 256;
  // The workgroup renders tiles l = blockIdx.x, + gridDim.x, ... (a multiple
  // of 8 workgroups, so every l of a workgroup maps to the XCD it runs on),
  // and fetches the next tile's slot table and patch cells while the passes
  // of the current one run, so their latency is not waited out.
  auto load_table = [&](int l, int32_t* e) {
    const int32_t* tab = A.tables + (int64_t)hp_xcd_tile(l, n_tiles) * (H * H);
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int i = tid + 256 * gi;
      e[gi] = i < H * H ? tab[i] : -1;
    }
  };
  auto load_cells = [&](const int32_t* e, float (*v)[6]) {
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int64_t slot = e[gi] & kSsSlotMask;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        v[gi][ch] = e[gi] >= 0 ? img[ch * A.n_active + slot] : 0.f;
        v[gi][3 + ch] = e[gi] >= 0 ? ref[ch * A.n_active + slot] : 0.f;
      }
    }
  };
  int32_t e[NG], en[NG];
  float v[NG][6], vn[NG][6];
  float acc_s = 0.f, acc_l = 0.f;  // this thread's SSIM and L1 sums over the workgroup's tiles
  if ((int)blockIdx.x >= n_tiles) return;
  // one tile: the cells in e / v; with more, the next tile's (ln) are
  // fetched into en / vn during the passes
  auto tile = [&](int l, int ln, bool more) {
    const int ct = hp_xcd_tile(l, n_tiles);
    int f, x0, y0;
    ss_tile_origin(A, ct, &f, &x0, &y0);
    // zone windows: the tile takes the direct path when it holds a polar pixel
    const int N = 1 << A.order;
    // tiles narrower than 8 pixels (orders 0-2) always take the direct path
    constexpr bool kSmall = B < 8;
    const bool direct =
        kSmall || (ZONES && (f < 4 ? (x0 + y0 + 2 * B - 2 >= N) : (f >= 8 ? (x0 + y0 <= N - 2) : false)));
    __syncthreads();  // the previous tile's LDS reads are done
    bool mine_full = true;
  #pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int i = tid + 256 * gi;
      if (i < H * H) {
        int cx, cy;
        ss_cell<B>(i, &cx, &cy);
        mine_full &= e[gi] >= 0;
        s.in[0][cy][cx] = e[gi] >= 0 ? 1.f : 0.f;
  #pragma unroll
        for (int k = 0; k < 6; ++k) s.in[1 + k][cy][cx] = v[gi][k];
        if (ZONES && direct) {
          const int64_t q = hp_chart_pixel(A.order, f, x0 + cx - SS_R, y0 + cy - SS_R);
          double d[3] = {0.0, 0.0, 0.0};
          if (q >= 0) hp_pix_dir(A.order, q, d);
          s.dir[cy * H + cx][0] = d[0];
          s.dir[cy * H + cx][1] = d[1];
          s.dir[cy * H + cx][2] = d[2];
        }
      }
    }
    // every cell of the patch active: the window weights need no mask and sum
    // to (sum of taps)^2 everywhere
    const bool full = __syncthreads_and(mine_full);
    if (more) load_table(ln, en);
    // this thread's pixel: nested local index tid (slot order of a full tile)
    const int px = (int)hp_compact_bits((uint32_t)tid), py = (int)hp_compact_bits((uint32_t)tid >> 1);
    const bool own = tid < B * B;
    float xc[3] = {0.f, 0.f, 0.f}, yc[3] = {0.f, 0.f, 0.f};
    if (own) {
  #pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        xc[ch] = s.in[1 + ch][py + SS_R][px + SS_R];
        yc[ch] = s.in[4 + ch][py + SS_R][px + SS_R];
      }
    }
    float Sm[16];
    if constexpr (!kSmall) if (!direct) {
      // pass 1 along x: item (row r, channel ch, quarter k) slides the window
      // over the 14 cells behind its 4 outputs
      constexpr int Q = B / 4, NI1 = H * 3 * Q;
      for (int it = tid; it < NI1; it += 256) {
        const int r = it / (3 * Q), rem = it % (3 * Q), ch = rem / Q, c0 = 4 * (rem % Q);
        float m[16], x[16], y[16];
  #pragma unroll
        for (int j = 0; j < 16; j += 4) {
          const float4 a = *reinterpret_cast<const float4*>(&s.in[0][r][c0 + j]);
          const float4 bx = *reinterpret_cast<const float4*>(&s.in[1 + ch][r][c0 + j]);
          const float4 by = *reinterpret_cast<const float4*>(&s.in[4 + ch][r][c0 + j]);
          m[j] = a.x; m[j + 1] = a.y; m[j + 2] = a.z; m[j + 3] = a.w;
          x[j] = bx.x; x[j + 1] = bx.y; x[j + 2] = bx.z; x[j + 3] = bx.w;
          y[j] = by.x; y[j + 1] = by.y; y[j + 2] = by.z; y[j + 3] = by.w;
        }
        float o[6][4];
  #pragma unroll
        for (int k = 0; k < 6; ++k)
  #pragma unroll
          for (int u = 0; u < 4; ++u) o[k][u] = 0.f;
        if (full) {
          // m = 1 everywhere: no mask products, no weight sums
  #pragma unroll
          for (int j = 0; j < 14; ++j) {
            const float q5[5] = {x[j], y[j], x[j] * x[j], y[j] * y[j], x[j] * y[j]};
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int a = j - u;
              if (a >= 0 && a < SS_W) {
  #pragma unroll
                for (int k = 0; k < 5; ++k) o[1 + k][u] = fmaf(A.g[a], q5[k], o[1 + k][u]);
              }
            }
          }
        } else {
  #pragma unroll
          for (int j = 0; j < 14; ++j) {
            const float wx = m[j] * x[j], wy = m[j] * y[j];
            const float q5[6] = {m[j], wx, wy, wx * x[j], wy * y[j], wx * y[j]};
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int a = j - u;
              if (a >= 0 && a < SS_W) {
  #pragma unroll
                for (int k = 0; k < 6; ++k) o[k][u] = fmaf(A.g[a], q5[k], o[k][u]);
              }
            }
          }
        }
        // quantity index: 0 weight, 1+ch x, 4+ch y, 7+ch xx, 10+ch yy, 13+ch xy
        if (ch == 0 && !full)
          *reinterpret_cast<float4*>(&s.p1[0][r * B + c0]) = make_float4(o[0][0], o[0][1], o[0][2], o[0][3]);
  #pragma unroll
        for (int k = 1; k < 6; ++k)
          *reinterpret_cast<float4*>(&s.p1[1 + 3 * (k - 1) + ch][r * B + c0]) =
              make_float4(o[k][0], o[k][1], o[k][2], o[k][3]);
      }
      if (more) load_cells(en, vn);
      __syncthreads();
      // pass 2 along y: item (column c, quantity k, half hh) slides over the
      // B/2 + 10 rows behind its B/2 outputs
      constexpr int RO = B / 2, NI2 = B * 16 * 2;
      for (int it = tid; it < NI2; it += 256) {
        const int c = it % B, k = (it / B) % 16, hh = it / (16 * B);
        if (full && k == 0) continue;
        float w[RO + 2 * SS_R];
  #pragma unroll
        for (int j = 0; j < RO + 2 * SS_R; ++j) w[j] = s.p1[k][(hh * RO + j) * B + c];
  #pragma unroll
        for (int u = 0; u < RO; ++u) {
          float acc = 0.f;
  #pragma unroll
          for (int a = 0; a < SS_W; ++a) acc = fmaf(A.g[a], w[u + a], acc);
          S[k][ss_nest_local(c, hh * RO + u)] = acc;   // nested order: read back by pixel tid
        }
      }
      __syncthreads();
      if (own) {
  #pragma unroll
        for (int k = 0; k < 16; ++k) Sm[k] = S[k][tid];
        if (full) Sm[0] = A.gsum * A.gsum;
      }
    }
    if (direct) {
      // direct 121-tap sums: polar pixels (zone windows) weigh by great-circle
      // distance, the others by the chart window
      if (more) load_cells(en, vn);
  #pragma unroll
      for (int k = 0; k < 16; ++k) Sm[k] = 0.f;
      if (own) {
        const bool polar = ZONES && ss_polar(A.order, hp_xyf_nest(A.order, x0 + px, y0 + py, f));
        const double* up = s.dir[(py + SS_R) * H + px + SS_R];
        for (int b = 0; b < SS_W; ++b) {
          for (int a = 0; a < SS_W; ++a) {
            const int cy = py + b, cx = px + a;
            const float m = s.in[0][cy][cx];
            if (m == 0.f) continue;
            const float w = polar ? m * __expf(-(float)(ss_dist2(up, s.dir[cy * H + cx]) * A.wscale))
                                  : m * (A.g[a] * A.g[b]);
            Sm[0] += w;
  #pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
              const float x = s.in[1 + ch][cy][cx], y = s.in[4 + ch][cy][cx];
              const float wx = w * x, wy = w * y;
              Sm[1 + ch] += wx;
              Sm[4 + ch] += wy;
              Sm[7 + ch] = fmaf(wx, x, Sm[7 + ch]);
              Sm[10 + ch] = fmaf(wy, y, Sm[10 + ch]);
              Sm[13 + ch] = fmaf(wx, y, Sm[13 + ch]);
            }
          }
        }
      }
    }
    float ssum = 0.f, lsum = 0.f;
    int64_t slot = -1;
    float gl[kSsG] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (own) {
      slot = ss_slot(A, hp_xyf_nest(A.order, x0 + px, y0 + py, f));
      if (slot >= 0) {
        const float iZ = __builtin_amdgcn_rcpf(Sm[0]);
  #pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          const float sv = ss_index(A.C1, A.C2, iZ, Sm[1 + ch], Sm[4 + ch], Sm[7 + ch], Sm[10 + ch], Sm[13 + ch],
                                    &gl[ch], &gl[3 + ch], &gl[6 + ch]);
          ssum += sv;
          lsum += fabsf(xc[ch] - yc[ch]);
          if (smap) smap[ch * A.n_active + slot] = sv;
        }
      }
    }
    if (G) {
      // the tile's partials leave as one contiguous run: its active pixels
      // hold the slots [start, start + count) (staged in LDS over the first
      // pass's place, once every thread is done reading it)
      const int t = A.active_tiles[ct];
      const int64_t start = A.tile_start[t];
      const int cnt = A.tile_count[t];
      float4* stage = reinterpret_cast<float4*>(&s.p1[0][0]);
      __syncthreads();
      if (slot >= 0) {
        const int loc = (int)(slot - start);
        stage[3 * loc] = make_float4(gl[0], gl[1], gl[2], gl[3]);
        stage[3 * loc + 1] = make_float4(gl[4], gl[5], gl[6], gl[7]);
        stage[3 * loc + 2] = make_float4(gl[8], 0.f, 0.f, 0.f);
      }
      __syncthreads();
      float4* out = reinterpret_cast<float4*>(G + start * kSsG);
      for (int i = tid; i < 3 * cnt; i += 256) out[i] = stage[i];
    }
    acc_s += ssum;
    acc_l += lsum;
  };
  if constexpr (ZONES) {
    // with zone windows every workgroup has one tile (ssim_grid)
    load_table(blockIdx.x, e);
    load_cells(e, v);
    tile(blockIdx.x, 0, false);
  } else {
    load_table(blockIdx.x, e);
    load_cells(e, v);
    for (int l = blockIdx.x; l < n_tiles; l += gridDim.x) {
      const int ln = l + (int)gridDim.x;
      tile(l, ln, ln < n_tiles);
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        e[gi] = en[gi];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[gi][k] = vn[gi][k];
      }
    }
  }
  // the workgroup's (sum of SSIM, sum of |img - ref|) over its tiles
  float red[2] = {acc_s, acc_l};
  hp_wave_totals<2>(red);
  if (hp_lane() == 0) { s_red[0][tid >> 6] = red[0]; s_red[1][tid >> 6] = red[1]; }
  __syncthreads();
  if (tid == 0)
    part[blockIdx.x] = make_float2(s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3],
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

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// The gathered patch; once the first pass has read it (the pass keeps its
// outputs in registers until then), its output [9][P1S] and after that the
// second pass's sums [9][B*B] overlay it.  The cells' directions and polar
// flags are only needed with zone windows.
template <int B, bool ZONES>
struct SsBwdLds {
  static constexpr int H = B + 2 * SS_R, HP = (H + 3) & ~3, P1S = H * B + ((48 - (H * B) % 32) % 32);
  static_assert(B < 8 || 9 * P1S + 9 * B * B <= 9 * H * HP, "first-pass output and sums fit over the patch");
  float in[9][H][HP];
  double dir[ZONES ? H * H : 1][3];
  uint8_t polar[ZONES ? H * H : 1];
};

// dL/dimg_p = dL/dloss * [ (1 - lam) sign(img - ref) / (3n)
//   - lam / (3n) * sum_{q in W(p)} w_q(p) (G0_q + 2 x_p G1_q + y_p G2_q) ]
// with w_q(p) the raw weight of q's window at p
template <int B, bool ZONES>
__global__ __launch_bounds__(256) void k_ssim_bwd(SsimArgs A, const float* __restrict__ img,
                                                  const float* __restrict__ ref, const float* __restrict__ G,
                                                  const float* __restrict__ dL_dloss, float* __restrict__ dimg,
                                                  int n_tiles) {
  using L = SsBwdLds<B, ZONES>;
  constexpr int H = L::H;
  __shared__ L s;
  // over the patch: the first pass's output, then the second pass's sums
  float(*P1)[L::P1S] = reinterpret_cast<float(*)[L::P1S]>(&s.in[0][0][0]);
  float(*S)[B * B] = reinterpret_cast<float(*)[B * B]>(&s.in[0][0][0] + 9 * L::P1S);
  const int tid = threadIdx.x;
  constexpr int NG = (H * H + 255) / 256;
  // tiles l = blockIdx.x, + gridDim.x, ... as in the forward; the next
  // tile's slot table and partials are fetched during the current passes
  auto load_table = [&](int l, int32_t* e) {
    const int32_t* tab = A.tables + (int64_t)hp_xcd_tile(l, n_tiles) * (H * H);
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int i = tid + 256 * gi;
      e[gi] = i < H * H ? tab[i] : -1;
    }
  };
  auto load_cells = [&](const int32_t* e, float (*v)[9]) {
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int64_t slot = e[gi] & kSsSlotMask;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a;
      if (e[gi] >= 0) {
        const float4* gp = reinterpret_cast<const float4*>(G + slot * kSsG);
        a = gp[0]; b = gp[1]; c = gp[2];
      }
      v[gi][0] = a.x; v[gi][1] = a.y; v[gi][2] = a.z; v[gi][3] = a.w;
      v[gi][4] = b.x; v[gi][5] = b.y; v[gi][6] = b.z; v[gi][7] = b.w;
      v[gi][8] = c.x;
    }
  };
  int32_t e[NG], en[NG];
  float v[NG][9], vn[NG][9];
  if ((int)blockIdx.x >= n_tiles) return;
  // one tile: the cells in e / v; with more, the next tile's (ln) are
  // fetched into en / vn during the passes
  auto tile = [&](int l, int ln, bool more) {
    const int ct = hp_xcd_tile(l, n_tiles);
    int f, x0, y0;
    ss_tile_origin(A, ct, &f, &x0, &y0);
    bool any_polar = false;
    __syncthreads();  // the previous tile's LDS reads are done
  #pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int i = tid + 256 * gi;
      if (i < H * H) {
        int cx, cy;
        ss_cell<B>(i, &cx, &cy);
  #pragma unroll
        for (int k = 0; k < 9; ++k) s.in[k][cy][cx] = v[gi][k];
        if (ZONES) {
          const bool pq = e[gi] >= 0 && (e[gi] & kSsPolarBit) != 0;
          s.polar[cy * H + cx] = pq ? 1 : 0;
          any_polar |= pq;
        }
      }
    }
    // the separable pass needs every neighbour's window to be the chart one;
    // tiles narrower than 8 pixels always take the direct path
    constexpr bool kSmall = B < 8;
    bool direct = kSmall;
    if (ZONES) direct = __syncthreads_or(any_polar) || kSmall;
    else __syncthreads();
    if (more) load_table(ln, en);
    const int px = (int)hp_compact_bits((uint32_t)tid), py = (int)hp_compact_bits((uint32_t)tid >> 1);
    float Sm[9];
    if constexpr (!kSmall) if (!direct) {
      constexpr int Q = B / 4, NI1 = H * 9 * Q;
      float o[4][4];  // up to 4 items per thread, 4 outputs each
      int kk[4], rr[4], cc[4];
  #pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int it = tid + 256 * t;
        kk[t] = -1;
        if (it < NI1) {
          const int r = it / (9 * Q), rem = it % (9 * Q), k = rem / Q, c0 = 4 * (rem % Q);
          float v[16];
  #pragma unroll
          for (int j = 0; j < 16; j += 4) {
            const float4 a = *reinterpret_cast<const float4*>(&s.in[k][r][c0 + j]);
            v[j] = a.x; v[j + 1] = a.y; v[j + 2] = a.z; v[j + 3] = a.w;
          }
  #pragma unroll
          for (int u = 0; u < 4; ++u) {
            float acc = 0.f;
  #pragma unroll
            for (int a = 0; a < SS_W; ++a) acc = fmaf(A.g[a], v[u + a], acc);
            o[t][u] = acc;
          }
          kk[t] = k; rr[t] = r; cc[t] = c0;
        }
      }
      __syncthreads();  // every read of the patch is done: the output goes over it
  #pragma unroll
      for (int t = 0; t < 4; ++t)
        if (kk[t] >= 0)
          *reinterpret_cast<float4*>(&P1[kk[t]][rr[t] * B + cc[t]]) = make_float4(o[t][0], o[t][1], o[t][2], o[t][3]);
      if (more) load_cells(en, vn);
      __syncthreads();
      constexpr int RO = B / 2, NI2 = B * 9 * 2;
      for (int it = tid; it < NI2; it += 256) {
        const int c = it % B, k = (it / B) % 9, hh = it / (9 * B);
        float w[RO + 2 * SS_R];
  #pragma unroll
        for (int j = 0; j < RO + 2 * SS_R; ++j) w[j] = P1[k][(hh * RO + j) * B + c];
  #pragma unroll
        for (int u = 0; u < RO; ++u) {
          float acc = 0.f;
  #pragma unroll
          for (int a = 0; a < SS_W; ++a) acc = fmaf(A.g[a], w[u + a], acc);
          S[k][ss_nest_local(c, hh * RO + u)] = acc;
        }
      }
      __syncthreads();
      if (tid < B * B) {
  #pragma unroll
        for (int k = 0; k < 9; ++k) Sm[k] = S[k][tid];
      }
    }
    if (direct) {
      if (more) load_cells(en, vn);
      // directions of the patch cells, for the polar windows
      if (ZONES) {
        for (int i = tid; i < H * H; i += 256) {
          const int cx = i % H, cy = i / H;
          const int64_t q = hp_chart_pixel(A.order, f, x0 + cx - SS_R, y0 + cy - SS_R);
          double d[3] = {0.0, 0.0, 0.0};
          if (q >= 0) hp_pix_dir(A.order, q, d);
          s.dir[i][0] = d[0];
          s.dir[i][1] = d[1];
          s.dir[i][2] = d[2];
        }
        __syncthreads();
      }
  #pragma unroll
      for (int k = 0; k < 9; ++k) Sm[k] = 0.f;
      if (tid < B * B) {
        const double* up = ZONES ? s.dir[(py + SS_R) * H + px + SS_R] : nullptr;
        for (int b = 0; b < SS_W; ++b) {
          for (int a = 0; a < SS_W; ++a) {
            const int cy = py + b, cx = px + a;
            // q's own window at p: the great-circle Gaussian for a polar q,
            // the (symmetric) chart taps otherwise
            const float w = (ZONES && s.polar[cy * H + cx])
                                ? __expf(-(float)(ss_dist2(up, s.dir[ZONES ? cy * H + cx : 0]) * A.wscale))
                                : A.g[a] * A.g[b];
  #pragma unroll
            for (int k = 0; k < 9; ++k) Sm[k] = fmaf(w, s.in[k][cy][cx], Sm[k]);
          }
        }
      }
    }
    const int64_t slot = tid < B * B ? ss_slot(A, hp_xyf_nest(A.order, x0 + px, y0 + py, f)) : -1;
    if (slot >= 0) {
      const float up = *dL_dloss;
      const float inv3n = 1.f / (3.f * (float)A.n_active);
  #pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float x = img[ch * A.n_active + slot], y = ref[ch * A.n_active + slot];
        const float dssim = Sm[0 * 3 + ch] + 2.f * x * Sm[1 * 3 + ch] + y * Sm[2 * 3 + ch];
        const float sgn = (float)((x > y) - (x < y));
        dimg[ch * A.n_active + slot] = up * inv3n * ((1.f - A.lam) * sgn - A.lam * dssim);
      }
    }
  };
  if constexpr (ZONES) {
    // with zone windows every workgroup has one tile (ssim_grid)
    load_table(blockIdx.x, e);
    load_cells(e, v);
    tile(blockIdx.x, 0, false);
  } else {
    load_table(blockIdx.x, e);
    load_cells(e, v);
    for (int l = blockIdx.x; l < n_tiles; l += gridDim.x) {
      const int ln = l + (int)gridDim.x;
      tile(l, ln, ln < n_tiles);
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        e[gi] = en[gi];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[gi][k] = vn[gi][k];
      }
    }
  }
}

// Patch tables: for every active tile and patch cell (in gather order), the
// compact slot of the chart neighbour (-1: missing or inactive), with bit 30
// set when that neighbour lies in a polar cap.  Image independent: built once
// per mask and reused by every forward and backward.
template <int B>
__global__ __launch_bounds__(256) void k_ssim_tables(SsimArgs A, int32_t* __restrict__ tables) {
  constexpr int H = B + 2 * SS_R;
  const int ct = blockIdx.x;
  int f, x0, y0;
  ss_tile_origin(A, ct, &f, &x0, &y0);
  for (int i = threadIdx.x; i < H * H; i += 256) {
    int cx, cy;
    ss_cell<B>(i, &cx, &cy);
    const int64_t q = hp_chart_pixel(A.order, f, x0 + cx - SS_R, y0 + cy - SS_R);
    const int64_t slot = ss_slot(A, q);
    tables[(int64_t)ct * H * H + i] = slot < 0 ? -1 : ((int32_t)slot | (ss_polar(A.order, q) ? kSsPolarBit : 0));
  }
}

static int ss_patch(int b) { const int H = (1 << b) + 2 * SS_R; return H * H; }

static size_t ssim_ws_size(int64_t n_active, int64_t ntile) {
  return hp_align256((size_t)kSsG * n_active * 4) + hp_align256((size_t)ntile * sizeof(float2));
}

extern "C" size_t hp_ssim_workspace_bytes(int32_t order, int32_t tile_log2, int64_t n_active) {
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4 || n_active < 0) return 0;
  return ssim_ws_size(n_active, hp_geom(order, tile_log2).ntile);
}

extern "C" size_t hp_ssim_tables_bytes(int32_t order, int32_t tile_log2, int32_t n_tiles) {
  if (order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4 || n_tiles < 0) return 0;
  return hp_align256((size_t)n_tiles * ss_patch(hp_geom(order, tile_log2).b) * 4);
}

static hp_status ssim_mask_args(int32_t order, const hp_params* prm, const void* mask, int64_t n_active,
                                int32_t n_tiles, SsimArgs* A) {
  HP_TRY(hp_check_params(prm));
  if (!mask) return HP_ERR_INVALID_ARG;
  if (order < 0 || order > HP_MAX_ORDER) return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(order, prm->tile_log2);
  // tiles of 1 to 16 pixels a side (tiles under 8 pixels take the direct path)
  if (g.b < 0 || g.b > 4) return HP_ERR_UNSUPPORTED;
  if (n_tiles <= 0 || n_tiles > g.ntile || n_active <= 0 || n_active > g.npix) return HP_ERR_INVALID_ARG;
  const HpMaskView mv = hp_mask_view((const char*)mask, g);
  A->order = order; A->b = g.b; A->kt = g.kt;
  A->active_tiles = mv.active_tiles; A->tile_start = mv.tile_start; A->tile_count = mv.tile_count;
  A->tile_bits = mv.tile_bits; A->n_active = n_active;
  return HP_OK;
}

extern "C" hp_status hp_ssim_tables(const hp_params* prm, const void* mask, int32_t order, int64_t n_active,
                                    int32_t n_tiles, int32_t* tables, size_t tables_bytes, void* stream) {
  SsimArgs A;
  HP_TRY(ssim_mask_args(order, prm, mask, n_active, n_tiles, &A));
  if (!tables) return HP_ERR_INVALID_ARG;
  if (tables_bytes < hp_ssim_tables_bytes(order, prm->tile_log2, n_tiles)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  switch (A.b) {
    case 4: hipLaunchKernelGGL(k_ssim_tables<16>, dim3((unsigned)n_tiles), dim3(256), 0, s, A, tables); break;
    case 3: hipLaunchKernelGGL(k_ssim_tables<8>, dim3((unsigned)n_tiles), dim3(256), 0, s, A, tables); break;
    case 2: hipLaunchKernelGGL(k_ssim_tables<4>, dim3((unsigned)n_tiles), dim3(256), 0, s, A, tables); break;
    case 1: hipLaunchKernelGGL(k_ssim_tables<2>, dim3((unsigned)n_tiles), dim3(256), 0, s, A, tables); break;
    default: hipLaunchKernelGGL(k_ssim_tables<1>, dim3((unsigned)n_tiles), dim3(256), 0, s, A, tables); break;
  }
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// shared argument checks and set-up of the three entry points
static hp_status ssim_setup(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                            const hp_params* prm, const hp_ssim_params* sp, const void* mask, const int32_t* tables,
                            const void* ws, size_t ws_bytes, SsimArgs* A, float** Gm, float2** part) {
  HP_TRY(ssim_mask_args(order, prm, mask, n_active, n_tiles, A));
  if (!sp || !ws || !tables || !img || !ref) return HP_ERR_INVALID_ARG;
  if (!(sp->sigma > 0) || !(sp->C1 > 0) || !(sp->C2 > 0) || !(sp->lambda >= 0 && sp->lambda <= 1) ||
      (sp->zones != 0 && sp->zones != 1))
    return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(order, prm->tile_log2);
  if (ws_bytes < ssim_ws_size(n_active, g.ntile)) return HP_ERR_CAPACITY;
  A->tables = tables;
  A->C1 = sp->C1; A->C2 = sp->C2; A->lam = sp->lambda;
  A->gsum = 0.f;
  for (int a = 0; a < SS_W; ++a) {
    const double d = a - SS_R;
    A->g[a] = (float)exp(-d * d / (2.0 * (double)sp->sigma * (double)sp->sigma));
    A->gsum += A->g[a];
  }
  const double omega = 4.0 * M_PI / (double)g.npix;
  A->wscale = 1.0 / (2.0 * (double)sp->sigma * (double)sp->sigma * omega);
  *Gm = (float*)ws;
  *part = (float2*)((char*)ws + hp_align256((size_t)kSsG * n_active * 4));
  return HP_OK;
}

// Workgroups of the forward and backward: with the separable windows, three
// per CU (what the LDS patch allows; a multiple of 8), each looping over
// tiles; with zone windows one per tile, since their direct-path tiles cost
// several times the others and a fixed share per workgroup would leave the
// load uneven.
static unsigned ssim_grid(int32_t n_tiles, bool zones) {
  const int32_t g = 3 * 256;
  return (unsigned)(zones || n_tiles <= g ? n_tiles : g);
}
// the backward's patch and pass outputs share their LDS: four workgroups per
// CU (what its registers allow)
static unsigned ssim_bwd_grid(int32_t n_tiles, bool zones) {
  const int32_t g = 4 * 256;
  return (unsigned)(zones || n_tiles <= g ? n_tiles : g);
}

template <int B>
static hp_status ssim_fwd_launch_b(const SsimArgs& A, bool zones, const float* img, const float* ref,
                                   int32_t n_tiles, float* ssim_map, float* Gm, float2* part, hipStream_t s) {
  const dim3 grid(ssim_grid(n_tiles, zones));
  if (zones)
    hipLaunchKernelGGL((k_ssim_fwd<B, true>), grid, dim3(256), 0, s, A, img, ref, ssim_map, Gm, part, (int)n_tiles);
  else
    hipLaunchKernelGGL((k_ssim_fwd<B, false>), grid, dim3(256), 0, s, A, img, ref, ssim_map, Gm, part, (int)n_tiles);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

static hp_status ssim_fwd_launch(const SsimArgs& A, bool zones, const float* img, const float* ref, int32_t n_tiles,
                                 float lam, float* out, float* ssim_map, float* Gm, float2* part, hipStream_t s) {
  switch (A.b) {
    case 4: HP_TRY(ssim_fwd_launch_b<16>(A, zones, img, ref, n_tiles, ssim_map, Gm, part, s)); break;
    case 3: HP_TRY(ssim_fwd_launch_b<8>(A, zones, img, ref, n_tiles, ssim_map, Gm, part, s)); break;
    case 2: HP_TRY(ssim_fwd_launch_b<4>(A, zones, img, ref, n_tiles, ssim_map, Gm, part, s)); break;
    case 1: HP_TRY(ssim_fwd_launch_b<2>(A, zones, img, ref, n_tiles, ssim_map, Gm, part, s)); break;
    default: HP_TRY(ssim_fwd_launch_b<1>(A, zones, img, ref, n_tiles, ssim_map, Gm, part, s)); break;
  }
  // one partial per forward workgroup
  hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(1024), 0, s, (const float2*)part, (int)ssim_grid(n_tiles, zones),
                     A.n_active, lam, out);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

template <int B>
static hp_status ssim_bwd_launch_b(const SsimArgs& A, bool zones, const float* img, const float* ref,
                                   int32_t n_tiles, const float* Gm, const float* dL_dloss, float* dL_dimg,
                                   hipStream_t s) {
  const dim3 grid(ssim_bwd_grid(n_tiles, zones));
  if (zones)
    hipLaunchKernelGGL((k_ssim_bwd<B, true>), grid, dim3(256), 0, s, A, img, ref, Gm, dL_dloss, dL_dimg, (int)n_tiles);
  else
    hipLaunchKernelGGL((k_ssim_bwd<B, false>), grid, dim3(256), 0, s, A, img, ref, Gm, dL_dloss, dL_dimg,
                       (int)n_tiles);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

static hp_status ssim_bwd_launch(const SsimArgs& A, bool zones, const float* img, const float* ref, int32_t n_tiles,
                                 const float* Gm, const float* dL_dloss, float* dL_dimg, hipStream_t s) {
  switch (A.b) {
    case 4: return ssim_bwd_launch_b<16>(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s);
    case 3: return ssim_bwd_launch_b<8>(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s);
    case 2: return ssim_bwd_launch_b<4>(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s);
    case 1: return ssim_bwd_launch_b<2>(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s);
    default: return ssim_bwd_launch_b<1>(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s);
  }
}

extern "C" hp_status hp_ssim(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                             const hp_params* prm, const hp_ssim_params* sp, const void* mask, const int32_t* tables,
                             float* out, float* ssim_map, const float* dL_dloss, float* dL_dimg, void* ws,
                             size_t ws_bytes, void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, tables, ws, ws_bytes, &A, &Gm, &part));
  if (!out || (dL_dloss && !dL_dimg)) return HP_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const bool zones = sp->zones != 0;
  HP_TRY(ssim_fwd_launch(A, zones, img, ref, n_tiles, sp->lambda, out, ssim_map, dL_dloss ? Gm : nullptr, part, s));
  if (dL_dloss) HP_TRY(ssim_bwd_launch(A, zones, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, s));
  return HP_OK;
}

extern "C" hp_status hp_ssim_forward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles,
                                           int32_t order, const hp_params* prm, const hp_ssim_params* sp,
                                           const void* mask, const int32_t* tables, float* out, float* ssim_map,
                                           void* ws, size_t ws_bytes, void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, tables, ws, ws_bytes, &A, &Gm, &part));
  if (!out) return HP_ERR_INVALID_ARG;
  return ssim_fwd_launch(A, sp->zones != 0, img, ref, n_tiles, sp->lambda, out, ssim_map, Gm, part,
                         (hipStream_t)stream);
}

extern "C" hp_status hp_ssim_backward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles,
                                            int32_t order, const hp_params* prm, const hp_ssim_params* sp,
                                            const void* mask, const int32_t* tables, const void* ws, size_t ws_bytes,
                                            const float* dL_dloss, float* dL_dimg, void* stream) {
  SsimArgs A;
  float* Gm;
  float2* part;
  HP_TRY(ssim_setup(img, ref, n_active, n_tiles, order, prm, sp, mask, tables, ws, ws_bytes, &A, &Gm, &part));
  if (!dL_dloss || !dL_dimg) return HP_ERR_INVALID_ARG;
  return ssim_bwd_launch(A, sp->zones != 0, img, ref, n_tiles, Gm, dL_dloss, dL_dimg, (hipStream_t)stream);
}
