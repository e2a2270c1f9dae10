// k_sort.hip -- stage 2b of Alg. 1: sort the (tile, Gaussian) pairs by tile
// (stable, so the depth order in which they were emitted is kept inside each
// tile) and identify each tile's range [start_t, end_t).
#include "hp_sort_impl.h"

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, int64_t n, uint32_t n_tiles,
                              uint32_t* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (k >= n_tiles) return;  // a key past the caller's tile count has no range slot
  if (i == 0 || keys[i - 1] != k) ranges[2 * (int64_t)k] = (uint32_t)i;
  if (i == n - 1 || keys[i + 1] != k) ranges[2 * (int64_t)k + 1] = (uint32_t)(i + 1);
}

static int bits_for(int64_t count) {
  int b = 0;
  while (((int64_t)1 << b) < count) ++b;
  return b;
}

extern "C" size_t hp_sort_workspace_bytes(int64_t n_pairs, int32_t n_tiles) {
  (void)n_tiles;
  if (n_pairs < 0) return 0;
  return hpsort::radix_ws_bytes(n_pairs);
}

extern "C" hp_status hp_sort(uint32_t* keys, uint32_t* vals, int64_t n_pairs, int32_t n_tiles, uint32_t* tile_ranges,
                             void* ws, size_t ws_bytes, void* stream) {
  if (n_pairs < 0 || n_tiles < 0 || n_pairs > ((int64_t)1 << 31)) return HP_ERR_INVALID_ARG;
  if (n_tiles > 0 && !tile_ranges) return HP_ERR_INVALID_ARG;
  if (n_pairs > 0 && (!keys || !vals || !ws)) return HP_ERR_INVALID_ARG;
  if (ws_bytes < hpsort::radix_ws_bytes(n_pairs)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(hp_blocks(2 * (int64_t)n_tiles, 256)), dim3(256), 0, s, tile_ranges,
                       2 * (int64_t)n_tiles, 0u);
    HP_CHECK_LAUNCH();
  }
  if (n_pairs == 0) return HP_OK;
  HP_TRY(hpsort::radix_sort(keys, vals, n_pairs, bits_for(n_tiles), ws, s));
  hipLaunchKernelGGL(k_tile_ranges, dim3(hp_blocks(n_pairs, 256)), dim3(256), 0, s, keys, n_pairs, (uint32_t)n_tiles,
                     tile_ranges);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
