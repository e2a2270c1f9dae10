// hp_sort_impl.h -- device-wide exclusive scan and stable LSD radix sort of
// (uint32 key, uint32 value) pairs, used for the depth order of Gaussians and
// the per-tile sort of (tile, Gaussian) pairs.
#pragma once

#include "hp_common.h"

namespace hpsort {
namespace {  // internal linkage: each translation unit keeps its own kernels

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;                       // per thread
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096 per block
constexpr int kMaxScanBlocks = kScanThreads * 16;     // second level capacity

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 pairs per block

// ---------------------------------------------------------------------------
// scan
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* total) {
  // 1024 threads = 16 waves
  __shared__ T s_w[16];
  const int lane = hp_lane(), w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  if (w == 0) {
    T t = lane < (int)(blockDim.x >> 6) ? s_w[lane] : T(0);
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      T y = __shfl_up(t, off, 64);
      if (lane >= off) t += y;
    }
    if (lane < 16) s_w[lane] = t;
  }
  __syncthreads();
  T wave_base = w > 0 ? s_w[w - 1] : T(0);
  *total = s_w[(blockDim.x >> 6) - 1];
  __syncthreads();
  return wave_base + x - v;
}

// per block: exclusive scan of its 4096 elements (in place into out) and the block sum
template <class T, class In>
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const In* __restrict__ in, T* __restrict__ out, int64_t n,
                                                             T* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? (T)in[base + k] : T(0);
    acc += v[k];
  }
  T total;
  T ex = block_exclusive_scan<T>(acc, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of the block sums (up to kMaxScanBlocks), total to *grand
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(T* sums, int64_t nb, T* grand) {
  const int per = (int)((nb + kScanThreads - 1) / kScanThreads);
  const int64_t lo = (int64_t)threadIdx.x * per;
  T acc = 0;
  for (int k = 0; k < per; ++k)
    if (lo + k < nb) acc += sums[lo + k];
  T total;
  T ex = block_exclusive_scan<T>(acc, &total);
  for (int k = 0; k < per; ++k)
    if (lo + k < nb) {
      T s = sums[lo + k];
      sums[lo + k] = ex;
      ex += s;
    }
  if (threadIdx.x == 0 && grand) *grand = total;
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T* __restrict__ out, int64_t n, const T* __restrict__ sums) {
  const T add = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] += add;
}

template <class T>
inline size_t scan_ws_bytes(int64_t n) {
  return hp_align256((size_t)((n + kScanTile - 1) / kScanTile + 1) * sizeof(T));
}

// exclusive scan of n elements of `in` (converted to T) into `out`; *grand
// (device, nullable) receives the total.  n <= kScanTile * kMaxScanBlocks.
template <class T, class In>
inline hp_status scan_exclusive(const In* in, T* out, int64_t n, T* grand, void* ws, hipStream_t s) {
  if (n <= 0) return HP_OK;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb > kMaxScanBlocks) return HP_ERR_UNSUPPORTED;
  T* sums = (T*)ws;
  hipLaunchKernelGGL((k_scan_local<T, In>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_scan_sums<T>), dim3(1), dim3(kScanThreads), 0, s, sums, nb, grand);
  HP_CHECK_LAUNCH();
  if (nb > 1) {
    hipLaunchKernelGGL((k_scan_add<T>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, n, sums);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
// digit histogram of each block's 4096 keys: hist[d * nblocks + block]
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                             int bits, uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t s_h[256];
  const int radix = 1 << bits;
  for (int d = threadIdx.x; d < radix; d += kSortThreads) s_h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint32_t mask = (uint32_t)radix - 1;
#pragma unroll 4
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < radix; d += kSortThreads) hist[(int64_t)d * nblocks + blockIdx.x] = s_h[d];
}

// Stable scatter.  Wave w of a block owns the contiguous items
// [w*1024, (w+1)*1024) of the block's 4096 and ranks them in 16 rounds of 64:
// equal digits inside a round are matched by ballots on the digit bits, and a
// running count per digit, private to the wave, carries the rank across
// rounds.  After one barrier the per-wave counts become per-wave offsets and
// the block's items are placed in LDS sorted by digit, so that the final
// writes go out as contiguous runs per digit.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* __restrict__ keys,
                                                                const uint32_t* __restrict__ vals, int64_t n,
                                                                int shift, int bits, const uint32_t* __restrict__ offs,
                                                                int64_t nblocks, uint32_t* __restrict__ okeys,
                                                                uint32_t* __restrict__ ovals) {
  constexpr int kWaveItems = kSortTile / 4;  // 1024
  constexpr int kRounds = kWaveItems / 64;   // 16
  __shared__ uint32_t s_cnt[4][256];
  __shared__ uint32_t s_loc[256];
  __shared__ uint32_t s_goff[256];
  __shared__ uint32_t s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1;
  const int tid = threadIdx.x, lane = hp_lane(), w = tid >> 6;
  for (int k = tid; k < 4 * 256; k += kSortThreads) (&s_cnt[0][0])[k] = 0;
  for (int d = tid; d < radix; d += kSortThreads) s_goff[d] = offs[(int64_t)d * nblocks + blockIdx.x];
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t rk[kRounds], kk[kRounds], vv[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + (int64_t)w * kWaveItems + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t key = valid ? keys[i] : 0u;
    kk[r] = key;
    vv[r] = valid ? vals[i] : 0u;
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
  // per digit: per-wave exclusive offsets and the block-local start of the digit
  uint32_t tot = 0;
  if (tid < radix) {
    const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
    s_cnt[0][tid] = 0;
    s_cnt[1][tid] = c0;
    s_cnt[2][tid] = c0 + c1;
    s_cnt[3][tid] = c0 + c1 + c2;
    tot = c0 + c1 + c2 + c3;
  }
  // exclusive scan of the digit totals over the (<= 256) digits
  {
    uint32_t x = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __shared__ uint32_t s_wsum[4];
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < w; ++k) add += s_wsum[k];
    if (tid < radix) s_loc[tid] = add + x - tot;
  }
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
  const int64_t nloc = n - base < kSortTile ? n - base : kSortTile;
  for (int lp = tid; lp < nloc; lp += kSortThreads) {
    const uint32_t key = s_key[lp];
    const uint32_t d = (key >> shift) & mask;
    const uint32_t g = s_goff[d] + ((uint32_t)lp - s_loc[d]);
    okeys[g] = key;
    ovals[g] = s_val[lp];
  }
}

__global__ void k_copy_u32(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

inline size_t radix_ws_bytes(int64_t n) {
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  const int64_t h = 256 * (nb > 0 ? nb : 1);
  return 2 * hp_align256((size_t)n * 4) + hp_align256((size_t)h * 4) + scan_ws_bytes<uint32_t>(h);
}

// Stable sort of (keys, vals) by the low `nbits` bits of the key; the result
// ends in keys/vals.
// Stable sort of n (key, value) pairs by the low nbits of the key.  The
// result is left in (keys, vals), or, when out_keys / out_vals are given, in
// whichever of (keys, vals) and the workspace's second buffer the last pass
// wrote (returned through them; no copy back).
inline hp_status radix_sort(uint32_t* keys, uint32_t* vals, int64_t n, int nbits, void* ws, hipStream_t s,
                            uint32_t** out_keys = nullptr, uint32_t** out_vals = nullptr) {
  if (out_keys) *out_keys = keys;
  if (out_vals) *out_vals = vals;
  if (n <= 1 || nbits <= 0) return HP_OK;
  const int passes = (nbits + 7) / 8;
  const int bits = (nbits + passes - 1) / passes;
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  char* p = (char*)ws;
  uint32_t* k2 = (uint32_t*)p; p += hp_align256((size_t)n * 4);
  uint32_t* v2 = (uint32_t*)p; p += hp_align256((size_t)n * 4);
  uint32_t* hist = (uint32_t*)p; p += hp_align256((size_t)256 * nb * 4);
  void* sws = p;
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * bits;
    const int b = (shift + bits <= nbits) ? bits : nbits - shift;
    const int64_t nh = (int64_t)(1 << b) * nb;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, n, shift, b, hist, nb);
    HP_CHECK_LAUNCH();
    HP_TRY((scan_exclusive<uint32_t, uint32_t>(hist, hist, nh, (uint32_t*)nullptr, sws, s)));
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, va, n, shift, b, hist, nb,
                       kb, vb);
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
    hipLaunchKernelGGL(k_copy_u32, dim3(hp_blocks(n, 256)), dim3(256), 0, s, ka, keys, n);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_copy_u32, dim3(hp_blocks(n, 256)), dim3(256), 0, s, va, vals, n);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

}  // namespace
}  // namespace hpsort
