// hp_sort_impl.h -- device-wide exclusive scan and stable LSD radix sort of
// (uint32 key, uint32 value) pairs whose element count may live in device
// memory: the binning sizes its later steps from counts it has just computed
// on the GPU, so nothing here waits for the host.
//
// Both run on a grid fixed at launch from a capacity (an upper bound of the
// count): block b of G takes the contiguous run of 4096-element tiles
// [b T / G, (b + 1) T / G), T = ceil(n / 4096), with n read on the device.
// Wave-level scans use DPP row shifts and row broadcasts; the sort ranks keys
// with wave ballots on the digit bits.
#pragma once

#include "hp_common.h"

namespace hpsort {
namespace {  // internal linkage: each translation unit keeps its own kernels

constexpr int kThreads = 256;              // 4 waves
constexpr int kItems = 16;                 // per thread and tile
constexpr int kTile = kThreads * kItems;   // 4096 elements per tile
constexpr int kMaxGrid = 1024;
static_assert(kMaxGrid <= 4 * kThreads, "k_radix_digit_scan holds a row of at most 4 entries per thread");

// element count: min(*n, cap) (cap when n is null)
__device__ __forceinline__ int64_t dev_count(const uint64_t* n, int64_t cap) {
  if (!n) return cap;
  const uint64_t v = *n;
  return v < (uint64_t)cap ? (int64_t)v : cap;
}

inline unsigned grid_for(int64_t cap) {
  const int64_t t = (cap + kTile - 1) / kTile;
  return (unsigned)(t < 1 ? 1 : (t > kMaxGrid ? kMaxGrid : t));
}

// tiles of block b: [t0, t1)
__device__ __forceinline__ void block_tiles(int64_t n, int64_t* t0, int64_t* t1, int64_t tile = kTile) {
  const int64_t T = (n + tile - 1) / tile, G = gridDim.x, b = blockIdx.x;
  *t0 = T * b / G;
  *t1 = T * (b + 1) / G;
}

// The radix passes work on tiles of 1024 keys (4 per thread): a million keys
// make ~1000 workgroups, enough to keep every CU busy, where 4096-key tiles
// left one 4-wave workgroup per CU.
constexpr int kRadixTile = 1024;

inline unsigned radix_grid(int64_t cap) {
  const int64_t t = (cap + kRadixTile - 1) / kRadixTile;
  return (unsigned)(t < 1 ? 1 : (t > kMaxGrid ? kMaxGrid : t));
}

// ---------------------------------------------------------------------------
// wave and block scans
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, BOUND);
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<CTRL, ROW_MASK, BOUND>((uint32_t)v);
  const uint32_t hi = dpp_u32<CTRL, ROW_MASK, BOUND>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_any(uint32_t v) { return dpp_u32<CTRL, ROW_MASK, BOUND>(v); }
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint64_t dpp_any(uint64_t v) { return dpp_u64<CTRL, ROW_MASK, BOUND>(v); }

// Inclusive scan over the 64 lanes (all active): Hillis-Steele inside each
// 16-lane row with row_shr 1, 2, 4, 8 (lanes whose source lies before the row
// start add 0), then row_bcast:15 adds the last lane of rows 0 and 2 into rows
// 1 and 3, and row_bcast:31 adds lane 31 (rows 0 + 1) into rows 2 and 3.
template <class T>
__device__ __forceinline__ T wave_inclusive(T x) {
  x += dpp_any<0x111, 0xf, true>(x);
  x += dpp_any<0x112, 0xf, true>(x);
  x += dpp_any<0x114, 0xf, true>(x);
  x += dpp_any<0x118, 0xf, true>(x);
  x += dpp_any<0x142, 0xa, false>(x);
  x += dpp_any<0x143, 0xc, false>(x);
  return x;
}

// Exclusive scan over the 256 threads of a block; *total gets the block's
// sum.  s_w: 4 elements of LDS.
template <class T>
__device__ __forceinline__ T block_exclusive(T v, T* total, T* s_w) {
  const int w = threadIdx.x >> 6;
  const T inc = wave_inclusive<T>(v);
  if (hp_lane() == 63) s_w[w] = inc;
  __syncthreads();
  const T w0 = s_w[0], w1 = s_w[1], w2 = s_w[2], w3 = s_w[3];
  __syncthreads();  // s_w may be rewritten by the caller's next round
  T base = 0;
  if (w > 0) base += w0;
  if (w > 1) base += w1;
  if (w > 2) base += w2;
  *total = w0 + w1 + w2 + w3;
  return base + inc - v;
}

// ---------------------------------------------------------------------------
// scan: out[i] = sum of in[0 .. i), *grand = sum of all (n from the device)
// ---------------------------------------------------------------------------
template <class T, class In>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const In* __restrict__ in, const uint64_t* __restrict__ cnt,
                                                          int64_t cap, T* __restrict__ sums) {
  __shared__ T s_w[4];
  const int64_t n = dev_count(cnt, cap);
  int64_t t0, t1;
  block_tiles(n, &t0, &t1);
  T acc = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * kTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = base + (int64_t)k * kThreads;
      if (i < n) acc += (T)in[i];
    }
  }
  T total;
  block_exclusive<T>(acc, &total, s_w);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// every block adds the sums of the blocks before it, then scans its tiles
// with a running carry: a tile is loaded striped (coalesced) into LDS, each
// thread scans 16 consecutive elements of it, and the results leave striped
// again.  LDS element i sits at i + i / 16, so that the 16-element runs of
// neighbouring threads start in different banks.
template <class T, class In>
__global__ __launch_bounds__(kThreads) void k_scan_down(const In* in, T* out, const uint64_t* __restrict__ cnt,
                                                        int64_t cap, const T* __restrict__ sums, T* grand,
                                                        int64_t* count_out, const uint32_t* __restrict__ over) {
  __shared__ T s_w[4];
  __shared__ T s_x[kTile + kTile / kItems];
  const int64_t n = dev_count(cnt, cap);
  int64_t t0, t1;
  block_tiles(n, &t0, &t1);
  // prefix of the block sums before this block (and all of them)
  T pre = 0, all = 0;
  for (int j = threadIdx.x; j < (int)gridDim.x; j += kThreads) {
    const T s = sums[j];
    all += s;
    if (j < (int)blockIdx.x) pre += s;
  }
  T carry, tot_all;
  block_exclusive<T>(pre, &carry, s_w);
  block_exclusive<T>(all, &tot_all, s_w);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    if (grand) *grand = tot_all;
    if (count_out) *count_out = *over ? INT64_MAX : (int64_t)tot_all;
  }
  const int run = (int)threadIdx.x * (kItems + 1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t tb = t * kTile;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int i = k * kThreads + (int)threadIdx.x;
      s_x[i + i / kItems] = tb + i < n ? (T)in[tb + i] : T(0);
    }
    __syncthreads();
    T v[kItems];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = s_x[run + k];
      acc += v[k];
    }
    T tile_total;
    T ex = block_exclusive<T>(acc, &tile_total, s_w) + carry;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      s_x[run + k] = ex;
      ex += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int i = k * kThreads + (int)threadIdx.x;
      if (tb + i < n) out[tb + i] = s_x[i + i / kItems];
    }
    __syncthreads();  // the next tile's loads reuse s_x
    carry += tile_total;
  }
}

template <class T>
inline size_t scan_ws_bytes(int64_t cap) {
  return hp_align256((size_t)grid_for(cap) * sizeof(T));
}

// Exclusive scan of the first min(*cnt, cap) elements of `in` (converted to
// T) into `out` (in place allowed); *grand (device, nullable) receives the
// total.  cnt null: cap elements.  With count_out (device, nullable; then
// `over` too) *count_out receives the total as int64, or INT64_MAX when *over
// is set.
template <class T, class In>
inline hp_status scan_exclusive(const In* in, T* out, const uint64_t* cnt, int64_t cap, T* grand, void* ws,
                                hipStream_t s, int64_t* count_out = nullptr, const uint32_t* over = nullptr) {
  if (cap < 0) return HP_ERR_INVALID_ARG;
  const unsigned G = grid_for(cap);
  T* sums = (T*)ws;
  hipLaunchKernelGGL((k_scan_reduce<T, In>), dim3(G), dim3(kThreads), 0, s, in, cnt, cap, sums);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_scan_down<T, In>), dim3(G), dim3(kThreads), 0, s, in, out, cnt, cap, (const T*)sums, grand,
                     count_out, over);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
// digit histogram of each block's tiles, digit-major: hist[digit * G + block]
// (k_radix_digit_scan then turns every digit's row into the block offsets
// within that digit)
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         const uint64_t* __restrict__ cnt, int64_t cap, int shift,
                                                         int bits, uint32_t* __restrict__ hist, int64_t* mark) {
  __shared__ uint32_t s_h[256];
  if (mark && blockIdx.x == 0 && threadIdx.x == 0) *mark = INT64_MAX;
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1;
  for (int d = threadIdx.x; d < radix; d += kThreads) s_h[d] = 0;
  __syncthreads();
  const int64_t n = dev_count(cnt, cap);
  int64_t t0, t1;
  block_tiles(n, &t0, &t1, kRadixTile);
  const int64_t lo = t0 * kRadixTile, hi = t1 * kRadixTile < n ? t1 * kRadixTile : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) atomicAdd(&s_h[(keys[i] >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kThreads) hist[(int64_t)d * gridDim.x + blockIdx.x] = s_h[d];
}

// One workgroup per digit d: the row hist[d * G .. d * G + G) becomes its
// exclusive scan (where each block's keys of digit d start among all keys of
// digit d) and dtot[d] the digit's total.  G <= kMaxGrid = 4 * kThreads, so
// every thread holds four consecutive entries of the row.
__global__ __launch_bounds__(kThreads) void k_radix_digit_scan(uint32_t* __restrict__ hist, int G,
                                                               uint32_t* __restrict__ dtot) {
  __shared__ uint32_t s_w[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * G;
  const int j0 = 4 * (int)threadIdx.x;
  uint32_t v[4], acc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = j0 + k < G ? row[j0 + k] : 0u;
    acc += v[k];
  }
  uint32_t total;
  uint32_t ex = block_exclusive<uint32_t>(acc, &total, s_w);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (j0 + k < G) row[j0 + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = total;
}

// Stable scatter of each block's tiles, in order.  Per tile, wave w owns the
// contiguous items [w*256, (w+1)*256) and ranks them in 4 rounds of 64:
// equal digits inside a round are matched by ballots on the digit bits, and a
// running count per digit, private to the wave, carries the rank across
// rounds.  The tile is then placed in LDS sorted by digit, so that the global
// writes go out as contiguous runs per digit, and the block's running digit
// offsets advance by the tile's digit counts.
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ vals,
                                                            const uint64_t* __restrict__ cnt, int64_t cap, int shift,
                                                            int bits, const uint32_t* __restrict__ offs,
                                                            const uint32_t* __restrict__ dtot,
                                                            uint32_t* __restrict__ okeys, uint32_t* __restrict__ ovals) {
  constexpr int kWaveItems = kRadixTile / 4;  // 256
  constexpr int kRounds = kWaveItems / 64;     // 4
  __shared__ uint32_t s_cnt[4][256];
  __shared__ uint32_t s_loc[256];
  __shared__ uint32_t s_goff[256];
  __shared__ uint32_t s_wsum[4];
  __shared__ uint32_t s_key[kRadixTile];
  __shared__ uint32_t s_val[kRadixTile];
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1;
  const int tid = threadIdx.x, lane = hp_lane(), w = tid >> 6;
  const int64_t n = dev_count(cnt, cap);
  int64_t t0, t1;
  block_tiles(n, &t0, &t1, kRadixTile);
  // the block's first output position per digit: the keys of all smaller
  // digits (an exclusive scan of the digit totals; radix <= kThreads) plus
  // those of digit d in the blocks before this one
  {
    uint32_t all;
    const uint32_t dpre = block_exclusive<uint32_t>(tid < radix ? dtot[tid] : 0u, &all, s_wsum);
    if (tid < radix) s_goff[tid] = dpre + offs[(int64_t)tid * gridDim.x + blockIdx.x];
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t t = t0; t < t1; ++t) {
    for (int k = tid; k < 4 * 256; k += kThreads) (&s_cnt[0][0])[k] = 0;
    __syncthreads();
    const int64_t base = t * kRadixTile;
    uint32_t rk[kRounds], kk[kRounds], vv[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t i = base + (int64_t)w * kWaveItems + r * 64 + lane;
      const bool valid = i < n;
      const uint32_t key = valid ? keys[i] : 0u;
      kk[r] = key;
      vv[r] = valid ? (vals ? vals[i] : (uint32_t)i) : 0u;  // no values: each key's index
      const uint32_t d = (key >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      uint32_t before = 0;
      if (valid) before = s_cnt[w][d];
      rk[r] = before + (uint32_t)__popcll(peers & lt);
      const int leader = __ffsll((unsigned long long)peers) - 1;
      if (valid && lane == leader) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: per-wave exclusive offsets and the tile-local start of the digit
    uint32_t tot = 0;
    if (tid < radix) {
      const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
      s_cnt[0][tid] = 0;
      s_cnt[1][tid] = c0;
      s_cnt[2][tid] = c0 + c1;
      s_cnt[3][tid] = c0 + c1 + c2;
      tot = c0 + c1 + c2 + c3;
    }
    uint32_t all;
    const uint32_t loc = block_exclusive<uint32_t>(tot, &all, s_wsum);
    if (tid < radix) s_loc[tid] = loc;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t i = base + (int64_t)w * kWaveItems + r * 64 + lane;
      if (i < n) {
        const uint32_t d = (kk[r] >> shift) & mask;
        const uint32_t lp = s_loc[d] + s_cnt[w][d] + rk[r];
        s_key[lp] = kk[r];
        s_val[lp] = vv[r];
      }
    }
    __syncthreads();
    const int nloc = (int)(n - base < kRadixTile ? n - base : kRadixTile);
    for (int lp = tid; lp < nloc; lp += kThreads) {
      const uint32_t key = s_key[lp];
      const uint32_t d = (key >> shift) & mask;
      const uint32_t g = s_goff[d] + ((uint32_t)lp - s_loc[d]);
      okeys[g] = key;
      ovals[g] = s_val[lp];
    }
    __syncthreads();
    // the tile's digit counts move the block's offsets on
    if (tid < radix) s_goff[tid] += tot;
  }
}

// keys[i] = src[i], vals[i] = i
__global__ void k_keys_iota(const uint32_t* __restrict__ src, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            const uint64_t* __restrict__ cnt, int64_t cap, int64_t* mark) {
  if (mark && blockIdx.x == 0 && threadIdx.x == 0) *mark = INT64_MAX;
  const int64_t n = dev_count(cnt, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = src[i];
    vals[i] = (uint32_t)i;
  }
}

__global__ void k_copy_u32(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, const uint64_t* __restrict__ cnt,
                           int64_t cap) {
  const int64_t n = dev_count(cnt, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

inline unsigned copy_grid(int64_t cap) {
  const int64_t b = (cap + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

inline size_t radix_ws_bytes(int64_t cap) {
  const int64_t h = (int64_t)radix_grid(cap) * 256;
  return 2 * hp_align256((size_t)(cap > 0 ? cap : 1) * 4) + hp_align256((size_t)h * 4) + hp_align256(256 * 4);
}

// Stable sort of the first min(*cnt, cap) (key, value) pairs by the low
// `nbits` bits of the key (cnt null: cap pairs).  The result is left in
// (keys, vals), or, when out_keys / out_vals are given, in whichever of
// (keys, vals) and the workspace's second buffer the last pass wrote
// (returned through them; no copy back).  With first_keys, the input keys are
// read from there and each element's value is its index: keys and vals are
// then outputs only.  With mark (device, nullable), the sort's first kernel
// also sets *mark = INT64_MAX (a caller's "not yet counted" flag, set by the
// first kernel of its sequence); first_keys is required then.
inline hp_status radix_sort(uint32_t* keys, uint32_t* vals, const uint64_t* cnt, int64_t cap, int nbits, void* ws,
                            hipStream_t s, uint32_t** out_keys = nullptr, uint32_t** out_vals = nullptr,
                            const uint32_t* first_keys = nullptr, int64_t* mark = nullptr) {
  if (out_keys) *out_keys = keys;
  if (out_vals) *out_vals = vals;
  if (mark && (!first_keys || cap <= 0)) return HP_ERR_INVALID_ARG;
  if (cap <= 0) return HP_OK;
  if (cap == 1 || nbits <= 0) {
    if (first_keys) {
      hipLaunchKernelGGL(k_keys_iota, dim3(copy_grid(cap)), dim3(256), 0, s, first_keys, keys, vals, cnt, cap, mark);
      HP_CHECK_LAUNCH();
    }
    return HP_OK;
  }
  const int passes = (nbits + 7) / 8;
  const int bits = (nbits + passes - 1) / passes;
  const unsigned G = radix_grid(cap);
  char* p = (char*)ws;
  uint32_t* k2 = (uint32_t*)p; p += hp_align256((size_t)cap * 4);
  uint32_t* v2 = (uint32_t*)p; p += hp_align256((size_t)cap * 4);
  uint32_t* hist = (uint32_t*)p; p += hp_align256((size_t)G * 256 * 4);
  uint32_t* dtot = (uint32_t*)p;
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * bits;
    const int b = (shift + bits <= nbits) ? bits : nbits - shift;
    const uint32_t* src_k = (pass == 0 && first_keys) ? first_keys : ka;
    const uint32_t* src_v = (pass == 0 && first_keys) ? nullptr : va;
    hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kThreads), 0, s, src_k, cnt, cap, shift, b, hist,
                       pass == 0 ? mark : nullptr);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_radix_digit_scan, dim3(1u << b), dim3(kThreads), 0, s, hist, (int)G, dtot);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(kThreads), 0, s, src_k, src_v, cnt, cap, shift, b,
                       (const uint32_t*)hist, (const uint32_t*)dtot, kb, vb);
    HP_CHECK_LAUNCH();
    uint32_t* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  if (out_keys && out_vals) {
    *out_keys = ka;
    *out_vals = va;
    return HP_OK;
  }
  if (ka != keys) {
    hipLaunchKernelGGL(k_copy_u32, dim3(copy_grid(cap)), dim3(256), 0, s, (const uint32_t*)ka, keys, cnt, cap);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_copy_u32, dim3(copy_grid(cap)), dim3(256), 0, s, (const uint32_t*)va, vals, cnt, cap);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

}  // namespace
}  // namespace hpsort
