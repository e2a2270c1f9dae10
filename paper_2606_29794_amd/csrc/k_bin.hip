// k_bin.hip -- stage 2a of Alg. 1: tile assignment (QueryDisc) and pair
// emission.  Tile t is assigned to Gaussian i when the angle between t's cap
// centre and i's direction is at most r_s,i + R_t + guard; the NESTED
// quadtree of caps (each containing its children's) is walked depth-first
// without a stack, pruning subtrees whose cap misses the disc or that hold no
// active pixel.  Gaussians are processed in order of radial depth so that the
// pair list is depth-ordered, which the stable tile sort then preserves.
#include "hp_sort_impl.h"

// Work is split in two so that no lane walks a large Gaussian alone:
//  coarse: each Gaussian walks the quadtree from the 12 faces down to the
//          split level Ls = kt - 3 and lists the nodes that pass ("tasks");
//  fine:   each task walks its subtree (at most 64 tiles) down to the tiles.
// Both walks run twice (count, then write at scanned offsets) so that tasks
// and pairs stay in depth order.
constexpr int kSplitDepth = 3;

struct BinWs {
  uint32_t* dkey;    // [P] depth bits, then sorted
  uint32_t* order;   // [P] Gaussian ids in depth order
  uint32_t* tcount;  // [P] tasks per Gaussian (depth order)
  uint32_t* toff;    // [P] exclusive scan of tcount
  uint32_t* task_g;  // [cap_t] Gaussian of each task
  uint32_t* task_n;  // [cap_t] node index at the split level
  uint32_t* pcount;  // [cap_t] pairs per task
  uint64_t* poff;    // [cap_t] exclusive scan of pcount
  uint32_t* t_total; // device scalars: task total (u32), pair total (u64)
  uint64_t* p_total;
  void* sort_ws;
  void* scan_ws;
  int64_t cap_t;
};

static int64_t task_capacity(int64_t P) { return 16 * P + (1 << 20); }

static size_t bin_ws_size(int64_t P) {
  const int64_t ct = task_capacity(P);
  return 4 * hp_align256(P * 4) + 3 * hp_align256(ct * 4) + hp_align256(ct * 8) + 256 +
         hpsort::radix_ws_bytes(P) + hpsort::scan_ws_bytes<uint64_t>(ct > P ? ct : P);
}

static BinWs bin_ws(void* base, int64_t P) {
  BinWs w;
  const int64_t ct = task_capacity(P);
  char* p = (char*)base;
  w.dkey = (uint32_t*)p; p += hp_align256(P * 4);
  w.order = (uint32_t*)p; p += hp_align256(P * 4);
  w.tcount = (uint32_t*)p; p += hp_align256(P * 4);
  w.toff = (uint32_t*)p; p += hp_align256(P * 4);
  w.task_g = (uint32_t*)p; p += hp_align256(ct * 4);
  w.task_n = (uint32_t*)p; p += hp_align256(ct * 4);
  w.pcount = (uint32_t*)p; p += hp_align256(ct * 4);
  w.poff = (uint64_t*)p; p += hp_align256(ct * 8);
  w.t_total = (uint32_t*)p;
  w.p_total = (uint64_t*)(p + 128);
  p += 256;
  w.sort_ws = p; p += hpsort::radix_ws_bytes(P);
  w.scan_ws = p;
  w.cap_t = ct;
  return w;
}

__global__ void k_depth_keys(int64_t P, const float* __restrict__ depth, uint32_t* __restrict__ key,
                             uint32_t* __restrict__ id) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  key[i] = __float_as_uint(depth[i]);  // positive floats order as unsigned ints; +inf (culled) last
  id[i] = (uint32_t)i;
}

struct BinTables {
  const float4* cap;
  const float2* sc;
  const uint8_t* node_active;  // null: every node holds active pixels (full sphere)
  const int32_t* tile_compact;
  int kt, ls;
};

// cap test of node `node`: angle(centre, u) <= R + r_s + guard, as a chord
// comparison: |c - u|^2 <= 4 sin^2((R + theta)/2), always true past pi
__device__ __forceinline__ bool node_pass(const BinTables& T, int64_t node, float ux, float uy, float uz, float sg,
                                          float cg) {
  if (T.node_active && !T.node_active[node]) return false;
  const float4 c = T.cap[node];
  const float2 h = T.sc[node];
  const float dx = c.x - ux, dy = c.y - uy, dz = c.z - uz;
  const float chord2 = dx * dx + dy * dy + dz * dz;
  const float sh = h.x * cg + h.y * sg;  // sin((R + theta) / 2)
  const float ch = h.y * cg - h.x * sg;  // cos((R + theta) / 2)
  return (ch <= 0.f) || (chord2 <= 4.f * sh * sh);
}

// Stackless depth-first walk of the implicit quadtree (node (l, i) has
// children 4i..4i+3 at level l+1; level 0 holds the 12 faces) from root
// (l0, i0) -- or from all 12 faces when l0 < 0 -- down to level `stop`; calls
// f(i) for every passing node at `stop`.
template <class F>
__device__ __forceinline__ void quad_walk(const BinTables& T, int l0, int64_t i0, int stop, float ux, float uy, float uz,
                                          float sg, float cg, F&& f) {
  const bool forest = l0 < 0;
  const int lroot = forest ? 0 : l0;
  int l = lroot;
  int64_t i = forest ? 0 : i0;
  int64_t loff = hp_level_offset(l);
  while (true) {
    if (node_pass(T, loff + i, ux, uy, uz, sg, cg)) {
      if (l == stop) {
        f(i);
      } else {
        loff += 12ll << (2 * l);
        ++l;
        i *= 4;
        continue;
      }
    }
    while (l > lroot && (i & 3) == 3) {
      --l;
      loff -= 12ll << (2 * l);
      i >>= 2;
    }
    if (l == lroot) {
      if (forest && i < 11) {
        ++i;
        continue;
      }
      break;
    }
    ++i;
  }
}

__device__ __forceinline__ void gauss_dir(const float4* rec, const float* radius, uint32_t gid, float guard, float* u,
                                          float* sg, float* cg, bool* ok) {
  const float rs = radius[gid];
  *ok = rs > 0.f;
  if (!*ok) return;
  const float4 r0 = rec[4 * (int64_t)gid];
  u[0] = r0.x; u[1] = r0.y; u[2] = r0.z;
  sincosf(0.5f * (rs + guard), sg, cg);
}

// coarse walk: tasks of Gaussian order[k]
template <bool EMIT>
__global__ __launch_bounds__(256) void k_bin_coarse(int64_t P, const uint32_t* __restrict__ order,
                                                    const float4* __restrict__ rec, const float* __restrict__ radius,
                                                    BinTables T, float guard, uint32_t* __restrict__ tcount,
                                                    const uint32_t* __restrict__ toff, uint32_t* __restrict__ task_g,
                                                    uint32_t* __restrict__ task_n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint32_t gid = order[k];
  float u[3], sg, cg;
  bool ok;
  gauss_dir(rec, radius, gid, guard, u, &sg, &cg, &ok);
  if (!ok) {
    if (!EMIT) tcount[k] = 0;
    return;
  }
  uint32_t cnt = 0;
  const uint32_t base = EMIT ? toff[k] : 0;
  quad_walk(T, -1, 0, T.ls, u[0], u[1], u[2], sg, cg, [&](int64_t i) {
    if (EMIT) {
      task_g[base + cnt] = gid;
      task_n[base + cnt] = (uint32_t)i;
    }
    ++cnt;
  });
  if (!EMIT) tcount[k] = cnt;
}

// fine walk: pairs of task t
template <bool EMIT>
__global__ __launch_bounds__(256) void k_bin_fine(const uint32_t* __restrict__ n_tasks, int64_t cap_t,
                                                  const uint32_t* __restrict__ task_g,
                                                  const uint32_t* __restrict__ task_n, const float4* __restrict__ rec,
                                                  const float* __restrict__ radius, BinTables T, float guard,
                                                  uint32_t* __restrict__ pcount, const uint64_t* __restrict__ poff,
                                                  const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                  uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)*n_tasks;
  if (t >= nt || t >= cap_t) return;
  if (EMIT && *n_pairs > capacity) return;
  const uint32_t gid = task_g[t];
  float u[3], sg, cg;
  bool ok;
  gauss_dir(rec, radius, gid, guard, u, &sg, &cg, &ok);
  uint32_t cnt = 0;
  const uint64_t base = EMIT ? poff[t] : 0;
  quad_walk(T, T.ls, task_n[t], T.kt, u[0], u[1], u[2], sg, cg, [&](int64_t i) {
    if (EMIT) {
      keys[base + cnt] = (uint32_t)T.tile_compact[i];
      vals[base + cnt] = gid;
    }
    ++cnt;
  });
  if (!EMIT) pcount[t] = cnt;
}

__global__ void k_store_total(const uint64_t* grand, int64_t* n_pairs) { *n_pairs = (int64_t)*grand; }
__global__ void k_store_zero(int64_t* n_pairs) { *n_pairs = 0; }

extern "C" size_t hp_bin_workspace_bytes(int64_t P) { return P < 0 ? 0 : bin_ws_size(P) + 256; }

extern "C" hp_status hp_bin(int32_t phase, const void* projected, int64_t P, const hp_view* view, const hp_params* prm,
                            const void* grid, const void* mask, uint32_t* keys, uint32_t* vals, int64_t capacity,
                            int64_t* n_pairs, void* ws, size_t ws_bytes, void* stream) {
  if (phase < HP_BIN_COUNT || phase > HP_BIN_ALL) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_view(view, prm));
  if (P < 0 || P > ((int64_t)1 << 31) - 1 || capacity < 0) return HP_ERR_INVALID_ARG;
  if (!projected || !grid || !mask || !n_pairs || !ws) return HP_ERR_INVALID_ARG;
  if ((phase & HP_BIN_EMIT) && capacity > 0 && (!keys || !vals)) return HP_ERR_INVALID_ARG;
  if (ws_bytes < bin_ws_size(P)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  const HpProjView pv = hp_proj_view((const char*)projected, P);
  const HpGridView gv = hp_grid_view((void*)grid, g);
  const HpMaskView mv = hp_mask_view((const char*)mask, g);
  BinWs w = bin_ws(ws, P);
  const int ls = g.kt > kSplitDepth ? g.kt - kSplitDepth : 0;
  BinTables T{gv.cap, gv.sc, view->cam_type == HP_CAM_FULL ? nullptr : mv.node_active, mv.tile_compact, g.kt, ls};
  const unsigned fine_blocks = hp_blocks(w.cap_t, 256);
  if (phase & HP_BIN_COUNT) {
    if (P == 0) {
      hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, n_pairs);
      HP_CHECK_LAUNCH();
      return HP_OK;
    }
    hipLaunchKernelGGL(k_depth_keys, dim3(hp_blocks(P, 256)), dim3(256), 0, s, P, pv.depth, w.dkey, w.order);
    HP_CHECK_LAUNCH();
    HP_TRY(hpsort::radix_sort(w.dkey, w.order, P, 32, w.sort_ws, s));
    hipLaunchKernelGGL((k_bin_coarse<false>), dim3(hp_blocks(P, 256)), dim3(256), 0, s, P, w.order, pv.rec, pv.radius,
                       T, prm->bin_guard, w.tcount, (const uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr);
    HP_CHECK_LAUNCH();
    HP_TRY((hpsort::scan_exclusive<uint32_t, uint32_t>(w.tcount, w.toff, P, w.t_total, w.scan_ws, s)));
    // the number of tasks must fit the workspace: read it back once
    uint32_t nt = 0;
    if (hipMemcpyAsync(&nt, w.t_total, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return HP_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return HP_ERR_DEVICE;
    if ((int64_t)nt > w.cap_t) return HP_ERR_CAPACITY;
    hipLaunchKernelGGL((k_bin_coarse<true>), dim3(hp_blocks(P, 256)), dim3(256), 0, s, P, w.order, pv.rec, pv.radius,
                       T, prm->bin_guard, w.tcount, w.toff, w.task_g, w.task_n);
    HP_CHECK_LAUNCH();
    if (nt > 0) {
      hipLaunchKernelGGL((k_bin_fine<false>), dim3(hp_blocks(nt, 256)), dim3(256), 0, s, (const uint32_t*)w.t_total,
                         w.cap_t, w.task_g, w.task_n, pv.rec, pv.radius, T, prm->bin_guard, w.pcount,
                         (const uint64_t*)nullptr, (const int64_t*)nullptr, (int64_t)0, (uint32_t*)nullptr,
                         (uint32_t*)nullptr);
      HP_CHECK_LAUNCH();
      HP_TRY((hpsort::scan_exclusive<uint64_t, uint32_t>(w.pcount, w.poff, nt, w.p_total, w.scan_ws, s)));
      hipLaunchKernelGGL(k_store_total, dim3(1), dim3(1), 0, s, (const uint64_t*)w.p_total, n_pairs);
    } else {
      hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, n_pairs);
    }
    HP_CHECK_LAUNCH();
  }
  if ((phase & HP_BIN_EMIT) && P > 0) {
    (void)fine_blocks;
    // the task count is read on the device; the grid covers the capacity bound
    // only up to the tasks present when the count phase ran on this stream
    uint32_t nt = 0;
    if (hipMemcpyAsync(&nt, w.t_total, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return HP_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return HP_ERR_DEVICE;
    if (nt > 0) {
      hipLaunchKernelGGL((k_bin_fine<true>), dim3(hp_blocks(nt, 256)), dim3(256), 0, s, (const uint32_t*)w.t_total,
                         w.cap_t, w.task_g, w.task_n, pv.rec, pv.radius, T, prm->bin_guard, w.pcount, w.poff, n_pairs,
                         capacity, keys, vals);
      HP_CHECK_LAUNCH();
    }
  }
  return HP_OK;
}
