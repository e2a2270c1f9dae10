// k_sort.hip -- stage 2b of Alg. 1: sort the (tile, Gaussian) pairs by tile
// (stable, so the depth order in which they were emitted is kept inside each
// tile) and identify each tile's range [start_t, end_t).  The pair count is
// read on the device, so the call does not wait for the binning to finish.
#include "hp_sort_impl.h"

namespace {

// the count to sort: *n_pairs when it fits the buffers, else nothing
__global__ void k_sort_count(const int64_t* __restrict__ n_pairs, int64_t capacity, uint64_t* __restrict__ n_eff) {
  const int64_t n = *n_pairs;
  *n_eff = (n >= 0 && n <= capacity) ? (uint64_t)n : 0ull;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ n_eff, uint32_t n_tiles,
                              uint32_t* __restrict__ ranges) {
  const int64_t n = (int64_t)*n_eff;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= n_tiles) continue;  // a key past the caller's tile count has no range slot
    if (i == 0 || keys[i - 1] != k) ranges[2 * (int64_t)k] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != k) ranges[2 * (int64_t)k + 1] = (uint32_t)(i + 1);
  }
}

int bits_for(int64_t count) {
  int b = 0;
  while (((int64_t)1 << b) < count) ++b;
  return b;
}

}  // namespace

extern "C" size_t hp_sort_workspace_bytes(int64_t capacity, int32_t n_tiles) {
  (void)n_tiles;
  if (capacity < 0) return 0;
  return 256 + hpsort::radix_ws_bytes(capacity);
}

extern "C" hp_status hp_sort(uint32_t* keys, uint32_t* vals, const int64_t* n_pairs, int64_t capacity, int32_t n_tiles,
                             uint32_t* tile_ranges, void* ws, size_t ws_bytes, void* stream) {
  if (capacity < 0 || n_tiles < 0 || capacity > ((int64_t)1 << 31)) return HP_ERR_INVALID_ARG;
  if (!n_pairs || !ws || (n_tiles > 0 && !tile_ranges) || (capacity > 0 && (!keys || !vals))) return HP_ERR_INVALID_ARG;
  if (ws_bytes < hp_sort_workspace_bytes(capacity, n_tiles)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  uint64_t* n_eff = (uint64_t*)ws;
  void* sort_ws = (char*)ws + 256;
  hipLaunchKernelGGL(k_sort_count, dim3(1), dim3(1), 0, s, n_pairs, capacity, n_eff);
  HP_CHECK_LAUNCH();
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(hp_blocks(2 * (int64_t)n_tiles, 256)), dim3(256), 0, s, tile_ranges,
                       2 * (int64_t)n_tiles, 0u);
    HP_CHECK_LAUNCH();
  }
  if (capacity == 0) return HP_OK;
  HP_TRY(hpsort::radix_sort(keys, vals, n_eff, capacity, bits_for(n_tiles), sort_ws, s));
  hipLaunchKernelGGL(k_tile_ranges, dim3(hpsort::copy_grid(capacity)), dim3(256), 0, s, (const uint32_t*)keys,
                     (const uint64_t*)n_eff, (uint32_t)n_tiles, tile_ranges);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
