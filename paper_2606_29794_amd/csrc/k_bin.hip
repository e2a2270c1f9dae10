// k_bin.hip -- stage 2a of Alg. 1: tile assignment (QueryDisc) and pair
// emission.  Tile t is assigned to Gaussian i when the angle between t's cap
// centre and i's direction is at most r_s,i + R_t + guard; the NESTED
// quadtree of caps (each containing its children's) is walked depth-first
// without a stack, pruning subtrees whose cap misses the disc or that hold no
// active pixel.  Gaussians are processed in order of radial depth so that the
// pair list is depth-ordered, which the stable tile sort then preserves.
#include "hp_sort_impl.h"
#include <type_traits>

// Work is split in two so that no lane walks a large Gaussian alone:
//  coarse: each Gaussian walks the quadtree from the 12 faces down to the
//          split level Ls = kt - 3 and lists the nodes that pass ("tasks");
//  fine:   one wave per task tests the (at most 64) tiles below its node.
// Both walks run twice (count, then write at scanned offsets) so that tasks
// and pairs stay in depth order.
constexpr int kSplitDepth = 3;

struct BinWs {
  uint32_t* dkey;    // [P] depth bits, then sorted
  uint32_t* order;   // [P] Gaussian ids in depth order
  uint32_t* tcount;  // [P] tasks per Gaussian (depth order)
  uint64_t* toff;    // [P] exclusive scan of tcount (64-bit: the total may pass 2^32)
  uint32_t* task_g;  // [cap_t] Gaussian of each task
  uint32_t* task_n;  // [cap_t] node index at the split level
  uint32_t* pcount;  // [cap_t] pairs per task
  uint64_t* pmask;   // [cap_t] tiles hit below the task's node (bit per leaf)
  uint64_t* poff;    // [cap_t] exclusive scan of pcount
  // device scalars
  uint64_t* t_total;  // tasks wanted (scan total)
  uint64_t* nt;       // tasks kept: min(t_total, cap_t)
  uint64_t* p_total;  // pairs
  uint64_t* ncol;     // (chunk, leaf) count entries to scan (sorted emission)
  uint32_t* over;     // 1 when the tasks exceeded cap_t
  void* sort_ws;
  void* scan_ws;
  int64_t cap_t;
};

static int64_t task_capacity(int64_t P) { return 16 * P + (1 << 20); }

static size_t bin_ws_size(int64_t P) {
  const int64_t ct = task_capacity(P);
  return 3 * hp_align256(P * 4) + hp_align256(P * 8) + 3 * hp_align256(ct * 4) + 2 * hp_align256(ct * 8) + 256 +
         hpsort::radix_ws_bytes(P) + hpsort::scan_ws_bytes<uint64_t>(ct > P ? ct : P);
}

static BinWs bin_ws(void* base, int64_t P) {
  BinWs w;
  const int64_t ct = task_capacity(P);
  char* p = (char*)base;
  w.dkey = (uint32_t*)p; p += hp_align256(P * 4);
  w.order = (uint32_t*)p; p += hp_align256(P * 4);
  w.tcount = (uint32_t*)p; p += hp_align256(P * 4);
  w.toff = (uint64_t*)p; p += hp_align256(P * 8);
  w.task_g = (uint32_t*)p; p += hp_align256(ct * 4);
  w.task_n = (uint32_t*)p; p += hp_align256(ct * 4);
  w.pcount = (uint32_t*)p; p += hp_align256(ct * 4);
  w.pmask = (uint64_t*)p; p += hp_align256(ct * 8);
  w.poff = (uint64_t*)p; p += hp_align256(ct * 8);
  w.t_total = (uint64_t*)p;
  w.nt = (uint64_t*)(p + 8);
  w.p_total = (uint64_t*)(p + 16);
  w.ncol = (uint64_t*)(p + 24);
  w.over = (uint32_t*)(p + 32);
  p += 256;
  w.sort_ws = p; p += hpsort::radix_ws_bytes(P);
  w.scan_ws = p;
  w.cap_t = ct;
  return w;
}

// tasks kept and the overflow flag, from the scanned task total
__global__ void k_task_clamp(const uint64_t* __restrict__ t_total, int64_t cap_t, uint64_t* __restrict__ nt,
                             uint32_t* __restrict__ over) {
  const uint64_t t = *t_total;
  *over = t > (uint64_t)cap_t ? 1u : 0u;
  *nt = t > (uint64_t)cap_t ? (uint64_t)cap_t : t;
}

struct BinTables {
  const float4* cap;
  const float2* sc;
  const uint8_t* node_active;  // null: every node holds active pixels (full sphere)
  const uint8_t* leaf_active;  // never null: active flags of every node (all set for the full sphere)
  const int32_t* tile_compact;
  int kt, ls;
  // (sin, cos) of half an angle added to every Gaussian's test angle: (0, 1)
  // for the binning itself, a margin when the pairs are candidates for a
  // narrower query that filters them afterwards
  float wsin, wcos;
};

// Cap test: angle(cap centre c, u) <= R + theta as a chord comparison,
// |c - u|^2 <= (2 sin((R + theta) / 2))^2, always true once R + theta >= pi
// (cos((R + theta) / 2) <= 0).  (sR, cR) = (sin R/2, cos R/2) of the cap,
// (sg, cg) = (sin theta/2, cos theta/2) of the Gaussian (theta = r_s + guard).
// Every binning kernel tests through this one function with explicit FMAs,
// so the sorted and the unsorted emission take identical decisions.
__device__ __forceinline__ bool hp_cap_test(float cx, float cy, float cz, float sR, float cR, float ux, float uy,
                                            float uz, float sg, float cg) {
  const float dx = cx - ux, dy = cy - uy, dz = cz - uz;
  const float chord2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float sh2 = fmaf(2.f * sR, cg, (2.f * cR) * sg);  // 2 sin((R + theta) / 2)
  const float ch = fmaf(cR, cg, -(sR * sg));               // cos((R + theta) / 2)
  return (ch <= 0.f) | (chord2 <= sh2 * sh2);
}

// The same test without the cos((R + theta) / 2) <= 0 branch, for callers
// that know R + theta < pi: when cos(theta / 2) > sin(R / 2) + 1e-5 the
// half-angle sum is below pi / 2 by a margin far beyond the rounding of ch,
// so the branch cannot fire and both forms decide alike.
__device__ __forceinline__ bool hp_cap_test_near(float cx, float cy, float cz, float sR, float cR, float ux, float uy,
                                                 float uz, float sg, float cg) {
  const float dx = cx - ux, dy = cy - uy, dz = cz - uz;
  const float chord2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float sh2 = fmaf(2.f * sR, cg, (2.f * cR) * sg);
  return chord2 <= sh2 * sh2;
}
constexpr float kNearMargin = 1e-5f;

// largest value of v over the wave (all lanes active)
__device__ __forceinline__ float hp_wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// cap test of node `node` (inactive nodes fail)
__device__ __forceinline__ bool node_pass(const BinTables& T, int64_t node, float ux, float uy, float uz, float sg,
                                          float cg) {
  if (T.node_active && !T.node_active[node]) return false;
  const float4 c = T.cap[node];
  const float2 h = T.sc[node];
  return hp_cap_test(c.x, c.y, c.z, h.x, h.y, ux, uy, uz, sg, cg);
}

// Stackless depth-first walk of the implicit quadtree (node (l, i) has
// children 4i..4i+3 at level l+1; level 0 holds the 12 faces) from root
// (l0, i0) -- or from all 12 faces when l0 < 0 -- down to level `stop`; calls
// f(i) for every passing node at `stop`.
template <class Pass, class F>
__device__ __forceinline__ void quad_walk(int l0, int64_t i0, int stop, Pass&& pass, F&& f) {
  const bool forest = l0 < 0;
  const int lroot = forest ? 0 : l0;
  int l = lroot;
  int64_t i = forest ? 0 : i0;
  int64_t loff = hp_level_offset(l);
  while (true) {
    if (pass(loff + i)) {
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

// (sin, cos) of half the test angle widened by the table's margin: the sum
// of half-angles, exact (bit for bit) when the margin is zero
__device__ __forceinline__ void widen_half(float wsin, float wcos, float* sg, float* cg) {
  const float s0 = *sg, c0 = *cg;
  *sg = fmaf(s0, wcos, c0 * wsin);
  *cg = fmaf(c0, wcos, -(s0 * wsin));
}

// direction and (sin, cos) of half the test angle r_s + guard (the sine is
// precomputed in the Gaussian's disc entry; the half angle is at most pi/2,
// so the cosine is the non-negative root), widened by the table's margin.
// A culled Gaussian (r_s = 0) has an all-zero disc entry, so the sine alone
// tells it apart (a kept one has r_s > 0 and a positive sine): one gather
// per Gaussian, not two.
__device__ __forceinline__ void gauss_dir(const float4* disc, const float* radius, uint32_t gid, const BinTables& T,
                                          float* u, float* sg, float* cg, bool* ok) {
  (void)radius;
  const hp_cfloatp r = (hp_cfloatp)disc + 4 * (int64_t)gid;
  *ok = r[3] > 0.f;
  if (!*ok) return;
  u[0] = r[0]; u[1] = r[1]; u[2] = r[2];
  *sg = r[3];
  *cg = sqrtf(fmaxf(0.f, 1.f - *sg * *sg));
  widen_half(T.wsin, T.wcos, sg, cg);
}

// coarse walk: tasks of Gaussian order[k].  With `slots` (slot-major
// [kSlots][P]) the count walk also keeps the first kSlots task nodes, and the
// emit pass copies them instead of walking again when they are all there.
constexpr int kSlots = 16;
constexpr int kTopNodes = 252;  // quadtree levels 0..2

// The quadtree's top levels (faces and two more: 252 nodes) in LDS, where
// every walk starts.  Returns how many are there.  The caller synchronises.
struct TopNodes {
  float4 cap[kTopNodes];
  float2 sc[kTopNodes];
  uint8_t act[kTopNodes];
};
__device__ __forceinline__ int load_top_nodes(const BinTables& T, TopNodes& S) {
  const int64_t nlev = hp_level_offset(T.ls + 1);  // nodes of levels 0..ls
  const int ntop = (int)(nlev < kTopNodes ? nlev : kTopNodes);
  for (int t = threadIdx.x; t < ntop; t += blockDim.x) {
    S.cap[t] = T.cap[t];
    S.sc[t] = T.sc[t];
    S.act[t] = T.node_active ? T.node_active[t] : (uint8_t)1;
  }
  return ntop;
}

// largest sin(R/2) over the LDS copy's nodes below the faces (levels 1-2), for
// the near-test guard; called by every lane after the copy is synchronised
__device__ __forceinline__ float top_srmax(const TopNodes& S, int ntop) {
  float m = 0.f;
  for (int t = 12 + hp_lane(); t < ntop; t += 64) m = fmaxf(m, S.sc[t].x);
  return hp_wave_max(m);
}

// Calls emit(i) for the passing nodes i at level T.ls, in increasing order,
// of the Gaussian with direction u and half test angle (sg, cg): the top
// levels are tested from the LDS copy, deeper ones from memory.  Level 1 (48
// nodes) is tested by every lane in the same order, which keeps the wave
// converged where a walk from the 12 faces would diverge at once; below a
// passing level-1 node the children are tested in order (level 2) and deeper
// levels are walked depth-first.
// srmax: top_srmax of the LDS copy.  When every walking lane of the wave has
// cos(theta / 2) > srmax + margin, the LDS nodes take the near test.
template <class Emit>
__device__ __forceinline__ void coarse_nodes(const BinTables& T, const TopNodes& S, int ntop, float srmax,
                                             const float* u, float sg, float cg, Emit&& emit) {
  const bool near = __builtin_amdgcn_ballot_w64(!(cg > srmax + kNearMargin)) == 0;
  auto pass = [&](int64_t node) -> bool {
    if (node < ntop) {
      if (!S.act[node]) return false;
      const float4 c = S.cap[node];
      const float2 h = S.sc[node];
      return near && node >= 12 ? hp_cap_test_near(c.x, c.y, c.z, h.x, h.y, u[0], u[1], u[2], sg, cg)
                                : hp_cap_test(c.x, c.y, c.z, h.x, h.y, u[0], u[1], u[2], sg, cg);
    }
    return node_pass(T, node, u[0], u[1], u[2], sg, cg);
  };
  if (T.ls == 0) {
    for (int f = 0; f < 12; ++f)
      if (pass(f)) emit(f);
    return;
  }
  uint64_t m1 = 0;
#pragma unroll 4
  for (int j = 0; j < 48; ++j) m1 |= pass(12 + j) ? (1ull << j) : 0ull;
  while (m1 != 0) {
    const int j = __builtin_ctzll(m1);
    m1 &= m1 - 1;
    if (T.ls == 1) {
      emit(j);
      continue;
    }
    for (int c = 0; c < 4; ++c) {
      const int64_t i2 = 4 * (int64_t)j + c;
      if (T.ls == 2) {
        if (pass(60 + i2)) emit(i2);
      } else {
        quad_walk(2, i2, T.ls, pass, emit);
      }
    }
  }
}

template <bool EMIT>
__global__ __launch_bounds__(256) void k_bin_coarse(int64_t P, const uint32_t* __restrict__ order,
                                                    const float4* __restrict__ disc, const float* __restrict__ radius,
                                                    BinTables T, float guard, uint32_t* __restrict__ tcount,
                                                    const uint64_t* __restrict__ toff, int64_t cap_t,
                                                    uint32_t* __restrict__ task_g, uint32_t* __restrict__ task_n,
                                                    uint32_t* __restrict__ slots) {
  __shared__ TopNodes S;
  const int ntop = load_top_nodes(T, S);
  __syncthreads();
  const float srmax = top_srmax(S, ntop);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint32_t gid = order[k];
  // the emit pass writes a Gaussian's tasks at its scanned offset, and none
  // past the task capacity (the count pass then flagged the overflow)
  const uint64_t base = EMIT ? toff[k] : 0ull;
  const uint32_t room = EMIT ? (base >= (uint64_t)cap_t ? 0u
                                : (uint32_t)min((uint64_t)tcount[k], (uint64_t)cap_t - base))
                             : 0u;
  if (EMIT && slots) {
    const uint32_t cnt = tcount[k];
    if (cnt <= (uint32_t)kSlots) {
      for (uint32_t j = 0; j < room; ++j) {
        task_g[base + j] = gid;
        task_n[base + j] = slots[(int64_t)j * P + k];
      }
      return;
    }
  }
  float u[3], sg, cg;
  bool ok;
  gauss_dir(disc, radius, gid, T, u, &sg, &cg, &ok);
  if (!ok) {
    if (!EMIT) tcount[k] = 0;
    return;
  }
  uint32_t cnt = 0;
  coarse_nodes(T, S, ntop, srmax, u, sg, cg, [&](int64_t i) {
    if (EMIT && cnt < room) {
      task_g[base + cnt] = gid;
      task_n[base + cnt] = (uint32_t)i;
    }
    if (!EMIT && slots && cnt < (uint32_t)kSlots) slots[(int64_t)cnt * P + k] = (uint32_t)i;
    ++cnt;
  });
  if (!EMIT) tcount[k] = cnt;
}

// ---- task list in node order without a sort --------------------------------
// For split levels of at most kHistNodes nodes.  The count walk also counts
// each workgroup's tasks per node into a node-major histogram [nn][G] (G
// workgroups of 256 Gaussians in depth order).  An exclusive scan of the
// histogram (each node's row scanned by its own workgroup, then the node
// offsets added) gives every (node, workgroup) its first slot, and the scatter
// pass writes each task straight to its place: that slot plus the number of
// the workgroup's earlier Gaussians with a task at the node.  A Gaussian has
// at most one task per node, so this is the order a stable sort of the
// depth-ordered tasks by node gives.
constexpr int kHistNodes = 768;
static_assert(kHistNodes <= 4 * 256, "k_task_segments takes four nodes per thread");

__global__ __launch_bounds__(256) void k_task_count(int64_t P, const uint32_t* __restrict__ order,
                                                    const float4* __restrict__ disc, const float* __restrict__ radius,
                                                    BinTables T, uint32_t* __restrict__ tcount,
                                                    uint32_t* __restrict__ slots, int nn, uint32_t* __restrict__ hist) {
  __shared__ TopNodes S;
  __shared__ uint32_t s_cnt[kHistNodes];
  const int ntop = load_top_nodes(T, S);
  for (int n = threadIdx.x; n < nn; n += blockDim.x) s_cnt[n] = 0u;
  __syncthreads();
  const float srmax = top_srmax(S, ntop);
  const int gb = blockIdx.x;
  const int64_t k = (int64_t)gb * blockDim.x + threadIdx.x;
  if (k < P) {
    const uint32_t gid = order[k];
    float u[3], sg, cg;
    bool ok;
    gauss_dir(disc, radius, gid, T, u, &sg, &cg, &ok);
    uint32_t cnt = 0;
    if (ok) {
      coarse_nodes(T, S, ntop, srmax, u, sg, cg, [&](int64_t i) {
        if (cnt < (uint32_t)kSlots) slots[(int64_t)cnt * P + k] = (uint32_t)i;
        atomicAdd(&s_cnt[i], 1u);
        ++cnt;
      });
    }
    tcount[k] = cnt;
  }
  __syncthreads();
  const int64_t G = gridDim.x;
  for (int n = threadIdx.x; n < nn; n += blockDim.x) hist[(int64_t)n * G + gb] = s_cnt[n];
}

// One workgroup per node n: the histogram row hist[n][0..G) becomes its
// exclusive scan hoff[n][0..G) (where workgroup b's tasks at node n start
// among the node's tasks) and rowtot[n] the node's task count.  The node
// offsets (an exclusive scan of rowtot) follow in k_task_segments.
__global__ __launch_bounds__(256) void k_hist_rows(const uint32_t* __restrict__ hist, int64_t G,
                                                   uint64_t* __restrict__ hoff, uint64_t* __restrict__ rowtot) {
  __shared__ uint64_t s_w[4];
  constexpr int kItems = 16;
  const uint32_t* row = hist + (int64_t)blockIdx.x * G;
  uint64_t* out = hoff + (int64_t)blockIdx.x * G;
  uint64_t carry = 0;
  for (int64_t t0 = 0; t0 < G; t0 += 256 * kItems) {
    const int64_t j0 = t0 + (int64_t)kItems * threadIdx.x;
    uint32_t v[kItems];
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = j0 + k < G ? row[j0 + k] : 0u;
      acc += v[k];
    }
    uint64_t tot;
    uint64_t ex = hpsort::block_exclusive<uint64_t>(acc, &tot, s_w) + carry;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (j0 + k < G) out[j0 + k] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Dynamic LDS per node: the workgroup's first slot (8 B), 256 membership
// bits (which of the workgroup's Gaussians have a task at the node), the
// node's first place in the workgroup's staging run (4 B) and the bit counts
// before each of the 8 words (8 x 1 B): 52 B.
constexpr int kScatterLdsPerNode = 52;
// tasks of one workgroup staged in LDS in node order, then written out in
// runs; a workgroup with more writes its tasks directly
constexpr int kStage = 2048;

__global__ __launch_bounds__(256) void k_task_scatter(int64_t P, const uint32_t* __restrict__ order,
                                                      const float4* __restrict__ disc,
                                                      const float* __restrict__ radius, BinTables T,
                                                      const uint32_t* __restrict__ tcount,
                                                      const uint32_t* __restrict__ slots, int nn,
                                                      const uint64_t* __restrict__ hoff,
                                                      const uint64_t* __restrict__ node_off, int64_t cap_t,
                                                      uint32_t* __restrict__ task_g) {
  extern __shared__ uint64_t s_dyn[];
  uint64_t* s_off = s_dyn;                            // [nn]
  uint32_t* s_bits = (uint32_t*)(s_dyn + nn);         // [nn][8]
  uint32_t* s_start = s_bits + 8 * nn;                // [nn]
  uint8_t* s_pre = (uint8_t*)(s_start + nn);          // [nn][8]
  __shared__ TopNodes S;
  __shared__ uint32_t s_gid[kStage];
  __shared__ uint16_t s_node[kStage];
  __shared__ uint32_t s_w[4];
  const int ntop = load_top_nodes(T, S);
  const int64_t G = gridDim.x;
  for (int n = threadIdx.x; n < nn; n += blockDim.x) s_off[n] = node_off[n] + hoff[(int64_t)n * G + blockIdx.x];
  for (int i = threadIdx.x; i < 8 * nn; i += blockDim.x) s_bits[i] = 0u;
  __syncthreads();
  const float srmax = top_srmax(S, ntop);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < P;
  const uint32_t cnt = live ? tcount[k] : 0u;
  const uint32_t gid = live ? order[k] : 0u;
  const int w = threadIdx.x >> 5;
  const uint32_t bit = 1u << (threadIdx.x & 31);
  // the Gaussian's nodes: from the count walk's slots, or walked again when
  // it had more than kSlots
  auto each_node = [&](auto&& f) {
    if (cnt <= (uint32_t)kSlots) {
      for (uint32_t j = 0; j < cnt; ++j) f((int64_t)slots[(int64_t)j * P + k]);
      return;
    }
    float u[3], sg, cg;
    bool ok;
    gauss_dir(disc, radius, gid, T, u, &sg, &cg, &ok);
    if (ok) coarse_nodes(T, S, ntop, srmax, u, sg, cg, f);
  };
  if (cnt) each_node([&](int64_t i) { atomicOr(&s_bits[8 * i + w], bit); });
  __syncthreads();
  // per node (thread t: nodes 4t .. 4t + 3): counts before each word, and
  // the node's place in the workgroup's node-ordered run
  uint32_t tot[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = 4 * (int)threadIdx.x + q;
    uint32_t a = 0;
    if (n < nn) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        s_pre[8 * n + j] = (uint8_t)a;
        a += (uint32_t)__popc(s_bits[8 * n + j]);
      }
    }
    tot[q] = a;
    sum += a;
  }
  uint32_t total;
  uint32_t ex = hpsort::block_exclusive<uint32_t>(sum, &total, s_w);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = 4 * (int)threadIdx.x + q;
    if (n < nn) s_start[n] = ex;
    ex += tot[q];
  }
  __syncthreads();
  const bool staged = total <= (uint32_t)kStage;
  if (cnt) {
    each_node([&](int64_t i) {
      const uint32_t r = (uint32_t)s_pre[8 * i + w] + (uint32_t)__popc(s_bits[8 * i + w] & (bit - 1u));
      if (staged) {
        const uint32_t lp = s_start[i] + r;
        s_gid[lp] = gid;
        s_node[lp] = (uint16_t)i;
      } else {
        const uint64_t pos = s_off[i] + r;
        if (pos < (uint64_t)cap_t) task_g[pos] = gid;
      }
    });
  }
  if (staged) {
    __syncthreads();
    // consecutive threads write consecutive places of each node's run
    for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
      const int n = s_node[t];
      const uint64_t pos = s_off[n] + (t - s_start[n]);
      if (pos < (uint64_t)cap_t) task_g[pos] = s_gid[t];
    }
  }
}

// One workgroup: every node's first task (an exclusive scan of the node task
// counts, into node_off), the task total and overflow flag, every node's task
// segment (clamped to the capacity), its chunks of 64 tasks and their
// offsets, and the number of (chunk, leaf) columns.  After an overflow no
// chunk is made.
__global__ __launch_bounds__(256) void k_task_segments(int nn, const uint64_t* __restrict__ rowtot,
                                                       uint64_t* __restrict__ node_off, int64_t cap_t, int depth,
                                                       uint64_t* __restrict__ t_total, uint64_t* __restrict__ nt,
                                                       uint32_t* __restrict__ over, uint32_t* __restrict__ seg,
                                                       uint32_t* __restrict__ choff, uint64_t* __restrict__ ncol) {
  __shared__ uint64_t s_w64[4];
  __shared__ uint32_t s_w[4];
  // nodes 4t .. 4t + 3 of thread t
  uint64_t cnt[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = 4 * (int)threadIdx.x + q;
    cnt[q] = n < nn ? rowtot[n] : 0ull;
    sum += cnt[q];
  }
  uint64_t tot;
  uint64_t pre = hpsort::block_exclusive<uint64_t>(sum, &tot, s_w64);
  const bool ov = tot > (uint64_t)cap_t;
  const uint64_t lim = ov ? (uint64_t)cap_t : tot;
  uint32_t nch[4], csum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = 4 * (int)threadIdx.x + q;
    nch[q] = 0u;
    if (n < nn) {
      node_off[n] = pre;
      uint64_t s0 = pre, s1 = pre + cnt[q];
      s0 = s0 < lim ? s0 : lim;
      s1 = s1 < lim ? s1 : lim;
      seg[2 * n] = (uint32_t)s0;
      seg[2 * n + 1] = (uint32_t)s1;
      nch[q] = ov ? 0u : (uint32_t)((s1 - s0 + 63) / 64);
    }
    pre += cnt[q];
    csum += nch[q];
  }
  uint32_t total;
  uint32_t ex = hpsort::block_exclusive<uint32_t>(csum, &total, s_w);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = 4 * (int)threadIdx.x + q;
    if (n < nn) choff[n] = ex;
    ex += nch[q];
  }
  if (threadIdx.x == 0) {
    choff[nn] = total;
    *ncol = (uint64_t)total << (2 * depth);
    *t_total = tot;
    *nt = lim;
    *over = ov ? 1u : 0u;
  }
}

// fine stage: one lane per tile below a task's node (64 tiles three levels
// down).  A wave takes 64 consecutive tasks at a time (their Gaussian and
// node ids in one coalesced load, then read out lane by lane) and issues the
// loads of kFineGroup tasks before testing any of them, so that many memory
// requests are in flight per wave.  The count pass keeps each task's 64-bit
// hit mask; the emit pass only turns masks into pairs, each hit written at
// its rank among the task's hits so that the pairs of a task are contiguous
// and tasks stay in depth order.
constexpr int kFineGroup = 8;

__device__ __forceinline__ uint64_t hp_readlane64(uint64_t v, int i) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), i);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void k_bin_fine_count(const uint64_t* __restrict__ n_tasks, int64_t cap_t,
                                                        const uint32_t* __restrict__ task_g,
                                                        const uint32_t* __restrict__ task_n,
                                                        const float4* __restrict__ disc, BinTables T,
                                                        uint64_t* __restrict__ pmask, uint32_t* __restrict__ pcount) {
  int64_t nt = (int64_t)*n_tasks;
  if (nt > cap_t) nt = cap_t;
  const int lane = hp_lane();
  const int depth = T.kt - T.ls;  // 0..3 levels below the task node
  const bool leaf_lane = lane < (1 << (2 * depth));
  const int leaf_mask = (1 << (2 * depth)) - 1;
  const int64_t leaf_off = hp_level_offset(T.kt);
  const int64_t nch = (nt + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  // the 64 tasks' discs, one gather per lane, read back as LDS broadcasts
  __shared__ float4 s_disc[4][64];
  const int wv = threadIdx.x >> 6;
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + hp_uniform(threadIdx.x >> 6); c < nch; c += waves) {
    const int64_t t0 = c << 6;
    const int nin = nt - t0 < 64 ? (int)(nt - t0) : 64;
    const uint32_t tg = lane < nin ? task_g[t0 + lane] : 0u;
    const uint32_t tn = lane < nin ? task_n[t0 + lane] : 0u;
    __builtin_amdgcn_wave_barrier();  // the previous chunk's reads are done
    s_disc[wv][lane] = lane < nin ? disc[tg] : make_float4(0.f, 0.f, 0.f, 0.f);
    __builtin_amdgcn_wave_barrier();
    uint64_t mine = 0;
    for (int i0 = 0; i0 < nin; i0 += kFineGroup) {
      float3 cap[kFineGroup];  // cap centre (the radius enters through sc)
      float2 sc[kFineGroup];
      uint32_t act[kFineGroup];
      float ux[kFineGroup], uy[kFineGroup], uz[kFineGroup], sg[kFineGroup];
#pragma unroll
      for (int q = 0; q < kFineGroup; ++q) {
        // past the chunk's end the last task is loaded again; its result is dropped
        const int i = i0 + q < nin ? i0 + q : nin - 1;
        // lanes past the node's leaves (depth < 3) load a valid leaf and drop it
        const int64_t node = leaf_off + ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)tn, i) << (2 * depth)) +
                             (lane & leaf_mask);
        const float4 d = s_disc[wv][i];  // same address on every lane: a broadcast
        ux[q] = d.x; uy[q] = d.y; uz[q] = d.z; sg[q] = d.w;
        const float* cp = (const float*)(T.cap + node);
        cap[q] = make_float3(cp[0], cp[1], cp[2]);
        sc[q] = T.sc[node];
        act[q] = (uint32_t)T.leaf_active[node];
      }
#pragma unroll
      for (int q = 0; q < kFineGroup; ++q) {
        const float cg = sqrtf(fmaxf(0.f, 1.f - sg[q] * sg[q]));
        const bool hit = leaf_lane && (act[q] != 0u) &&
                         hp_cap_test(cap[q].x, cap[q].y, cap[q].z, sc[q].x, sc[q].y, ux[q], uy[q], uz[q], sg[q], cg);
        const uint64_t m = __ballot(hit);
        if (lane == i0 + q) mine = m;
      }
    }
    if (lane < nin) {
      pmask[t0 + lane] = mine;
      pcount[t0 + lane] = (uint32_t)__popcll(mine);
    }
  }
}

__global__ __launch_bounds__(256) void k_bin_fine_emit(const uint64_t* __restrict__ n_tasks, int64_t cap_t,
                                                       const uint32_t* __restrict__ task_g,
                                                       const uint32_t* __restrict__ task_n, BinTables T,
                                                       const uint64_t* __restrict__ pmask,
                                                       const uint64_t* __restrict__ poff,
                                                       const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                       uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int64_t nt = (int64_t)*n_tasks;
  if (nt > cap_t) nt = cap_t;
  if (*n_pairs > capacity) return;
  const int lane = hp_lane();
  const int depth = T.kt - T.ls;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t nch = (nt + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + hp_uniform(threadIdx.x >> 6); c < nch; c += waves) {
    const int64_t t0 = c << 6;
    const int nin = nt - t0 < 64 ? (int)(nt - t0) : 64;
    const uint32_t tg = lane < nin ? task_g[t0 + lane] : 0u;
    const uint32_t tn = lane < nin ? task_n[t0 + lane] : 0u;
    const uint64_t mk = lane < nin ? pmask[t0 + lane] : 0ull;
    const uint64_t of = lane < nin ? poff[t0 + lane] : 0ull;
    for (int i0 = 0; i0 < nin; i0 += kFineGroup) {
      // all addresses and values of the group first, then only stores: no
      // register that an in-flight store reads is written before it drains
      int32_t comp[kFineGroup];
      uint32_t gv[kFineGroup];
      uint32_t* kp[kFineGroup];
      uint32_t* vp[kFineGroup];
      bool hit[kFineGroup];
#pragma unroll
      for (int q = 0; q < kFineGroup; ++q) {
        const int i = i0 + q < nin ? i0 + q : nin - 1;
        const uint64_t m = i0 + q < nin ? hp_readlane64(mk, i) : 0ull;
        const int64_t leaf = ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)tn, i) << (2 * depth)) + lane;
        hit[q] = ((m >> lane) & 1ull) != 0;
        comp[q] = hit[q] ? T.tile_compact[leaf] : 0;
        const uint64_t at = hp_readlane64(of, i) + (uint64_t)__popcll(m & below);
        kp[q] = keys + at;
        vp[q] = vals + at;
        gv[q] = (uint32_t)__builtin_amdgcn_readlane((int)tg, i);
      }
      // wait once for the group's gathers (vmcnt 0; expcnt and lgkmcnt left
      // at their maxima), so that the masked stores below need no waits
      __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
      for (int q = 0; q < kFineGroup; ++q) {
        if (hit[q]) {
          *kp[q] = (uint32_t)comp[q];
          *vp[q] = gv[q];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pairs straight into per-tile depth order (no sort of the pairs).  Every
// task names one node at the split level and one Gaussian.  After a stable
// sort of the tasks by node, the pairs of tile t = (node n, leaf b) are the
// tasks of n's segment whose test on leaf b passes, in depth order.  Each
// segment is cut into chunks of 64 tasks; a wave per chunk keeps one leaf per
// lane and tests the chunk's tasks one after the other, collecting for leaf b
// the 64-bit column W_b of hits.  popcount(W_b) per (chunk, leaf), laid out
// tile-major -- for each node, for each leaf, its chunks in order -- and
// scanned, gives every (chunk, leaf) its first output slot; inside a chunk
// the task at bit j writes at popcount(W_b below j).
// ---------------------------------------------------------------------------
__global__ void k_seg_ranges(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ n_dev, uint32_t nn,
                             uint32_t* __restrict__ seg) {
  const int64_t n = (int64_t)*n_dev;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= nn) continue;
    if (i == 0 || keys[i - 1] != k) seg[2 * (int64_t)k] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != k) seg[2 * (int64_t)k + 1] = (uint32_t)(i + 1);
  }
}

__global__ void k_seg_chunks(const uint32_t* __restrict__ seg, uint32_t nn, uint32_t* __restrict__ nch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) nch[i] = (seg[2 * i + 1] - seg[2 * i] + 63) / 64;
}

__global__ void k_fill_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// node of every chunk: workgroup n fills the chunks [choff[n], choff[n+1])
__global__ void k_chunk_nodes(const uint32_t* __restrict__ choff, uint32_t* __restrict__ cnode) {
  const uint32_t n = blockIdx.x, c1 = choff[n + 1];
  for (uint32_t c = choff[n] + threadIdx.x; c < c1; c += blockDim.x) cnode[c] = n;
}

struct ChunkInfo {
  uint32_t node, local, nchn, t0, ntask;
};
__device__ __forceinline__ ChunkInfo chunk_info(const uint32_t* choff, const uint32_t* seg, const uint32_t* cnode,
                                                uint32_t c) {
  ChunkInfo ci;
  ci.node = hp_uniform(((hp_cu32p)cnode)[c]);
  const uint32_t c0 = hp_uniform(((hp_cu32p)choff)[ci.node]);
  ci.nchn = hp_uniform(((hp_cu32p)choff)[ci.node + 1]) - c0;
  ci.local = c - c0;
  const uint32_t s0 = hp_uniform(((hp_cu32p)seg)[2 * ci.node]), s1 = hp_uniform(((hp_cu32p)seg)[2 * ci.node + 1]);
  ci.t0 = s0 + 64 * ci.local;
  ci.ntask = s1 - ci.t0 < 64 ? s1 - ci.t0 : 64;
  return ci;
}

// The chunks of the calling wave.  Workgroup b runs on XCD b mod 8, so XCD
// x takes the contiguous range [x n / 8, (x + 1) n / 8), shared by the waves
// of its workgroups.  Neighbouring chunks belong to the same or neighbouring
// quadtree nodes, whose tasks gather the same Gaussians' records and write
// the same tiles' lists: within one XCD they meet in one L2.  With fewer than
// 8 workgroups every wave strides over all chunks.
struct ChunkRange {
  uint32_t first, end, stride;
};
__device__ __forceinline__ ChunkRange xcd_chunks(uint32_t n) {
  // the wave index is uniform, which the compiler cannot see: without the
  // readfirstlane every chunk index (and the node search below) would live
  // in vector registers, with a vector load per search step
  const uint32_t nb = gridDim.x, wpb = blockDim.x >> 6, w = hp_uniform(threadIdx.x >> 6);
  ChunkRange r;
  if (nb < 8u) {
    r.first = blockIdx.x * wpb + w;
    r.end = n;
    r.stride = nb * wpb;
    return r;
  }
  const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
  const uint32_t nbx = (nb - x + 7u) / 8u;  // workgroups b < nb with b mod 8 = x
  r.first = (uint32_t)((uint64_t)n * x / 8u) + k * wpb + w;
  r.end = (uint32_t)((uint64_t)n * (x + 1u) / 8u);
  r.stride = nbx * wpb;
  return r;
}

// per chunk: the hit columns W_b (kept) and their popcounts, tile-major
__global__ __launch_bounds__(256) void k_bin_cols(const uint32_t* __restrict__ choff, uint32_t nn,
                                                  const uint32_t* __restrict__ seg, const uint32_t* __restrict__ cnode,
                                                  const uint32_t* __restrict__ tgid,
                                                  const float4* __restrict__ disc, BinTables T,
                                                  uint64_t* __restrict__ wcol, uint32_t* __restrict__ cnt) {
  const uint32_t nchunks = hp_uniform(((hp_cu32p)choff)[nn]);
  const int lane = hp_lane();
  const int depth = T.kt - T.ls;
  const int nleaf = 1 << (2 * depth);
  const bool leaf_lane = lane < nleaf;
  const int64_t leaf_off = hp_level_offset(T.kt);
  // the chunk's 64 tasks' discs, one per lane, published for the whole wave:
  // (direction, sin) and cos of half the widened test angle
  __shared__ float4 s_disc[4][64];
  __shared__ float s_cg[4][64];
  const int wv = threadIdx.x >> 6;
  const ChunkRange cr = xcd_chunks(nchunks);
  for (uint32_t c = cr.first; c < cr.end; c += cr.stride) {
    const ChunkInfo ci = chunk_info(choff, seg, cnode, c);
    const uint32_t ntask = hp_uniform(ci.ntask);
    // this lane's leaf below the chunk's node (lanes past the leaves test a
    // valid leaf and drop the result)
    const int64_t leaf = leaf_off + ((int64_t)ci.node << (2 * depth)) + (lane & (nleaf - 1));
    const float* cp = (const float*)(T.cap + leaf);
    const float cx = cp[0], cy = cp[1], cz = cp[2];
    const float2 h = T.sc[leaf];
    const bool act = leaf_lane && T.leaf_active[leaf] != 0;
    const uint32_t tg = (uint32_t)lane < ntask ? tgid[ci.t0 + lane] : 0u;
    // every task's disc in one gather (lane j: task j); (sin, cos) of
    // (r_s + guard) / 2 by the same expressions as the rest of the binning
    // (identical decisions)
    const float4 dl = (uint32_t)lane < ntask ? disc[tg] : make_float4(0.f, 0.f, 0.f, 0.f);
    float sgl = dl.w;
    float cgl = sqrtf(fmaxf(0.f, 1.f - sgl * sgl));
    widen_half(T.wsin, T.wcos, &sgl, &cgl);
    __builtin_amdgcn_wave_barrier();  // the previous chunk's reads are done
    s_disc[wv][lane] = make_float4(dl.x, dl.y, dl.z, sgl);
    s_cg[wv][lane] = cgl;
    __builtin_amdgcn_wave_barrier();
    // tasks far from the antipodal case for every leaf of the node, as a wave
    // mask: groups of such tasks take the near test (hp_cap_test_near),
    // which decides alike; a Gaussian whose disc covers nearly the whole
    // sphere keeps the full test
    const float srl = hp_wave_max(h.x);
    const uint64_t nearmask = __builtin_amdgcn_ballot_w64(!((uint32_t)lane < ntask) || cgl > srl + kNearMargin);
    // bits of tasks 0..31 and 32..63 are kept apart so that every set is a
    // 32-bit select-or
    uint32_t Wh[2] = {0u, 0u};
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const uint32_t jend = ntask < 32u * (half + 1) ? ntask : 32u * (half + 1);
      for (uint32_t j0 = 32u * half; j0 < jend; j0 += kFineGroup) {
        // entries past the chunk's end are read too (stale or zero LDS, in
        // bounds) and their bits dropped, so the reads take fixed offsets
        auto group = [&](auto near_tag) {
          constexpr bool NEAR = decltype(near_tag)::value;
          float ux[kFineGroup], uy[kFineGroup], uz[kFineGroup], sg[kFineGroup], cg[kFineGroup];
#pragma unroll
          for (int q = 0; q < kFineGroup; ++q) {
            const float4 d = s_disc[wv][j0 + q];  // same address on every lane: a broadcast
            ux[q] = d.x; uy[q] = d.y; uz[q] = d.z; sg[q] = d.w;
            cg[q] = s_cg[wv][j0 + q];
          }
#pragma unroll
          for (int q = 0; q < kFineGroup; ++q) {
            const bool in = NEAR ? hp_cap_test_near(cx, cy, cz, h.x, h.y, ux[q], uy[q], uz[q], sg[q], cg[q])
                                 : hp_cap_test(cx, cy, cz, h.x, h.y, ux[q], uy[q], uz[q], sg[q], cg[q]);
            const uint32_t bit = j0 + q < jend ? (1u << ((j0 + q) & 31u)) : 0u;
            Wh[half] |= in ? bit : 0u;
          }
        };
        if (((nearmask >> j0) & 0xffull) == 0xffull)
          group(std::true_type{});
        else
          group(std::false_type{});
      }
    }
    const uint64_t W = act ? ((uint64_t)Wh[1] << 32) | Wh[0] : 0ull;
    if (leaf_lane) {
      wcol[(int64_t)c * 64 + lane] = W;
      const int64_t flat = (int64_t)(c - ci.local) * nleaf + (int64_t)lane * ci.nchn + ci.local;
      cnt[flat] = (uint32_t)__popcll(W);
    }
  }
}

// Per chunk: every hit of leaf b's column goes to its slot in tile (node, b).
// The chunk's hits are numbered in (leaf, task) order: column lane b lists
// its hits (column and task, lowest task first) in LDS at their numbers,
// and the wave then writes 64 of them per store, lane k taking hit o + k,
// whose rank in its column gives the slot.  So each store instruction is
// full (the slots of one column are consecutive), where a store per column
// would carry ~10 lanes.
constexpr int kMaxChunkHits = 64 * 64;

// (start, end) of every active tile from the scanned column counts; the end
// of the last tile of the last node is the total.  When nothing is emitted
// (the pairs exceed the capacity, or the count has not completed) every
// range is empty, so that a render over them reads no list entry.  Written
// by the emission kernel's threads, strided over its grid.
struct TileRanges {
  int32_t n_tiles;
  const int32_t* active_tiles;
  const uint64_t* ncol;   // (chunk, leaf) count entries
  const uint64_t* total;  // pairs
  uint32_t* ranges;
};
__device__ __forceinline__ void write_tile_ranges(const TileRanges& R, int depth, const uint32_t* __restrict__ choff,
                                                  const uint64_t* __restrict__ start, bool none) {
  const int nleaf = 1 << (2 * depth);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < R.n_tiles;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (none) {
      R.ranges[2 * k] = 0u;
      R.ranges[2 * k + 1] = 0u;
      continue;
    }
    const int t = R.active_tiles[k];
    const uint32_t n = (uint32_t)t >> (2 * depth), b = (uint32_t)t & (uint32_t)(nleaf - 1);
    const int64_t c0 = choff[n], nchn = (int64_t)choff[n + 1] - c0;
    const uint64_t nc = *R.ncol;
    const uint64_t i0 = (uint64_t)(c0 * nleaf + b * nchn), i1 = (uint64_t)(c0 * nleaf + (b + 1) * nchn);
    R.ranges[2 * k] = (uint32_t)(i0 < nc ? start[i0] : *R.total);
    R.ranges[2 * k + 1] = (uint32_t)(i1 < nc ? start[i1] : *R.total);
  }
}

__global__ __launch_bounds__(256) void k_bin_emit_sorted(const uint32_t* __restrict__ choff, uint32_t nn,
                                                         const uint32_t* __restrict__ seg,
                                                         const uint32_t* __restrict__ cnode,
                                                         const uint32_t* __restrict__ tgid, int depth,
                                                         const uint64_t* __restrict__ wcol,
                                                         const uint64_t* __restrict__ start,
                                                         const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                         uint32_t* __restrict__ vals, TileRanges tr) {
  const bool none = *n_pairs > capacity;
  write_tile_ranges(tr, depth, choff, start, none);
  if (none) return;
  __shared__ uint64_t s_base[4][64];
  __shared__ uint32_t s_g[4][64], s_off[4][64];
  __shared__ uint16_t s_hit[4][kMaxChunkHits];  // column << 8 | task of every hit number
  const uint32_t nchunks = hp_uniform(((hp_cu32p)choff)[nn]);
  const int lane = hp_lane();
  const int wv = threadIdx.x >> 6;
  const int nleaf = 1 << (2 * depth);
  const bool leaf_lane = lane < nleaf;
  const ChunkRange cr = xcd_chunks(nchunks);
  // a chunk's columns, output slots and Gaussian ids
  auto fetch = [&](uint32_t c, uint64_t* W, uint64_t* base, uint32_t* g) {
    const ChunkInfo ci = chunk_info(choff, seg, cnode, c);
    *W = leaf_lane ? wcol[(int64_t)c * 64 + lane] : 0ull;
    *base = leaf_lane ? start[(int64_t)(c - ci.local) * nleaf + (int64_t)lane * ci.nchn + ci.local] : 0ull;
    *g = (uint32_t)lane < ci.ntask ? tgid[ci.t0 + lane] : 0u;
  };
  uint32_t c = cr.first;
  if (c >= cr.end) return;
  uint64_t W, base;
  uint32_t g;
  fetch(c, &W, &base, &g);
  while (true) {
    // the next chunk's loads go out before this chunk's stores
    const uint32_t cn = c + cr.stride;
    const bool more = cn < cr.end;
    uint64_t Wn = 0ull, basen = 0ull;
    uint32_t gn = 0u;
    if (more) fetch(cn, &Wn, &basen, &gn);
    const uint32_t cnt = (uint32_t)__popcll(W);
    const uint32_t incl = hpsort::wave_inclusive<uint32_t>(cnt);
    const uint32_t off = incl - cnt;
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    // column lane b: its hits at numbers off, off + 1, ... (every number
    // below tot written once)
    {
      uint64_t w = W;
      const uint32_t col = (uint32_t)lane << 8;
      for (uint32_t r = off; w != 0; ++r) {
        s_hit[wv][r] = (uint16_t)(col | (uint32_t)__builtin_ctzll(w));
        w &= w - 1;
      }
    }
    s_base[wv][lane] = base;
    s_g[wv][lane] = g;
    s_off[wv][lane] = off;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = (uint32_t)lane; k < tot; k += 64) {
      const uint32_t e = s_hit[wv][k];
      const uint32_t b = e >> 8;
      vals[s_base[wv][b] + (k - s_off[wv][b])] = s_g[wv][e & 0xffu];
    }
    __builtin_amdgcn_wave_barrier();  // this chunk's LDS reads are done
    if (!more) break;
    c = cn;
    W = Wn;
    base = basen;
    g = gn;
  }
}

// number of (chunk, leaf) count entries: chunks x leaves per node
__global__ void k_col_count(const uint32_t* __restrict__ choff, uint32_t nn, int depth, uint64_t* __restrict__ ncol) {
  *ncol = (uint64_t)choff[nn] << (2 * depth);
}

__global__ void k_store_zero(int64_t* n_pairs) { *n_pairs = 0; }

// one wave per 64 tasks, at most 8192 blocks of 4 waves that loop over them
static unsigned fine_grid(int64_t nt) {
  const int64_t blocks = ((nt + 63) / 64 + 3) / 4;
  return (unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
}

// Depth order, coarse walk and task list (shared by both emissions): tasks
// (Gaussian, node at the split level) in order of radial depth; *w.nt holds
// their number and *w.over whether they exceeded the workspace's capacity.
// Its first kernel also sets *n_pairs = INT64_MAX: until the count completes,
// the count says that nothing may be emitted.
static hp_status depth_order(const HpProjView& pv, int64_t P, BinWs& w, int64_t* n_pairs, hipStream_t s) {
  // positive floats order as unsigned ints (+inf, a culled Gaussian, last):
  // the sort reads the depths' bits as its keys
  return hpsort::radix_sort(w.dkey, w.order, nullptr, P, 32, w.sort_ws, s, nullptr, nullptr,
                            reinterpret_cast<const uint32_t*>(pv.depth), n_pairs);
}

static hp_status bin_tasks(const HpProjView& pv, int64_t P, const BinTables& T, float guard, BinWs& w, uint32_t* slots,
                           int64_t* n_pairs, hipStream_t s) {
  HP_TRY(depth_order(pv, P, w, n_pairs, s));
  hipLaunchKernelGGL((k_bin_coarse<false>), dim3(hp_blocks(P, 256)), dim3(256), 0, s, P, w.order, pv.disc, pv.radius,
                     T, guard, w.tcount, (const uint64_t*)nullptr, w.cap_t, (uint32_t*)nullptr, (uint32_t*)nullptr,
                     slots);
  HP_CHECK_LAUNCH();
  HP_TRY((hpsort::scan_exclusive<uint64_t, uint32_t>(w.tcount, w.toff, nullptr, P, w.t_total, w.scan_ws, s)));
  hipLaunchKernelGGL(k_task_clamp, dim3(1), dim3(1), 0, s, (const uint64_t*)w.t_total, w.cap_t, w.nt, w.over);
  HP_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_bin_coarse<true>), dim3(hp_blocks(P, 256)), dim3(256), 0, s, P, w.order, pv.disc, pv.radius,
                     T, guard, w.tcount, (const uint64_t*)w.toff, w.cap_t, w.task_g, w.task_n, slots);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

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
  BinTables T{gv.cap, gv.sc, view->cam_type == HP_CAM_FULL ? nullptr : mv.node_active, mv.node_active,
              mv.tile_compact, g.kt, ls, 0.f, 1.f};
  if (phase & HP_BIN_COUNT) {
    if (P == 0) {
      hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, n_pairs);
      HP_CHECK_LAUNCH();
      return HP_OK;
    }
    HP_TRY(bin_tasks(pv, P, T, prm->bin_guard, w, nullptr, n_pairs, s));
    // per task: its 64-bit hit mask and count; the counts scanned into offsets
    hipLaunchKernelGGL(k_bin_fine_count, dim3(fine_grid(w.cap_t)), dim3(256), 0, s, (const uint64_t*)w.nt, w.cap_t,
                       w.task_g, w.task_n, pv.disc, T, w.pmask, w.pcount);
    HP_CHECK_LAUNCH();
    // the pair total goes to *n_pairs with the scan (a count no buffer holds
    // when the tasks overflowed: the emission kernels then write nothing)
    HP_TRY((hpsort::scan_exclusive<uint64_t, uint32_t>(w.pcount, w.poff, w.nt, w.cap_t, w.p_total, w.scan_ws, s,
                                                       n_pairs, (const uint32_t*)w.over)));
  }
  if ((phase & HP_BIN_EMIT) && P > 0) {
    // the task count is read on the device; the grid covers the capacity bound
    hipLaunchKernelGGL(k_bin_fine_emit, dim3(fine_grid(w.cap_t)), dim3(256), 0, s, (const uint64_t*)w.nt, w.cap_t,
                       w.task_g, w.task_n, T, (const uint64_t*)w.pmask, (const uint64_t*)w.poff, n_pairs, capacity,
                       keys, vals);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

// ---- sorted emission: workspace and entry point -----------------------------
struct SortedWs {
  void* tsort_ws;    // radix sort of the tasks by node
  uint32_t* seg;     // [nn][2] task segment of every node
  uint32_t* nch;     // [nn] chunks per node
  uint32_t* choff;   // [nn + 1] first chunk of every node, total last
  uint32_t* cnt;     // [L] hits per (chunk, leaf), tile-major
  uint64_t* start;   // [L] exclusive scan of cnt: first output slot
  uint64_t* wcol;    // [nchunk_max][64] hit columns
  uint32_t* slots;   // [kSlots][P] first task nodes of every Gaussian (coarse walk)
  uint32_t* cnode;   // [nchunk_max] node of every chunk
  void* scan_ws;
  int64_t nn, nchunk_max, L;
};

static void sorted_dims(int64_t P, const HpGeom& g, int64_t* nn, int64_t* nchunk_max, int64_t* L) {
  const int ls = g.kt > kSplitDepth ? g.kt - kSplitDepth : 0;
  const int depth = g.kt - ls;
  *nn = 12ll << (2 * ls);
  *nchunk_max = task_capacity(P) / 64 + *nn + 1;
  *L = *nchunk_max * (1ll << (2 * depth));
}

static size_t sorted_ws_size(int64_t P, const HpGeom& g) {
  int64_t nn, ncm, L;
  sorted_dims(P, g, &nn, &ncm, &L);
  return hpsort::radix_ws_bytes(task_capacity(P)) + hp_align256(nn * 8) + hp_align256(nn * 4) +
         hp_align256((nn + 1) * 4) + hp_align256(L * 4) + hp_align256(L * 8) + hp_align256(ncm * 64 * 8) +
         hp_align256((size_t)kSlots * P * 4) + hp_align256((size_t)ncm * 4) +
         hpsort::scan_ws_bytes<uint64_t>(L > nn ? L : nn);
}

static SortedWs sorted_ws(void* base, int64_t P, const HpGeom& g) {
  SortedWs w;
  sorted_dims(P, g, &w.nn, &w.nchunk_max, &w.L);
  char* p = (char*)base;
  w.tsort_ws = p; p += hpsort::radix_ws_bytes(task_capacity(P));
  w.seg = (uint32_t*)p; p += hp_align256(w.nn * 8);
  w.nch = (uint32_t*)p; p += hp_align256(w.nn * 4);
  w.choff = (uint32_t*)p; p += hp_align256((w.nn + 1) * 4);
  w.cnt = (uint32_t*)p; p += hp_align256(w.L * 4);
  w.start = (uint64_t*)p; p += hp_align256(w.L * 8);
  w.wcol = (uint64_t*)p; p += hp_align256(w.nchunk_max * 64 * 8);
  w.slots = (uint32_t*)p; p += hp_align256((size_t)kSlots * P * 4);
  w.cnode = (uint32_t*)p; p += hp_align256((size_t)w.nchunk_max * 4);
  w.scan_ws = p;
  return w;
}

extern "C" size_t hp_bin_sorted_workspace_bytes(int64_t P, int32_t order, int32_t tile_log2) {
  if (P < 0 || order < 0 || order > HP_MAX_ORDER || tile_log2 < 0 || tile_log2 > 4) return 0;
  const HpGeom g = hp_geom(order, tile_log2);
  return bin_ws_size(P) + sorted_ws_size(P, g) + 512;
}

// one wave per chunk, at most kChunkBlocks blocks of 4 waves looping over the
// chunks (measured on config 2: 8192 blocks beat one resident round of 2048)
constexpr int64_t kChunkBlocks = 8192;
static unsigned chunk_grid(int64_t nchunks) {
  const int64_t blocks = (nchunks + 3) / 4;
  return (unsigned)(blocks < kChunkBlocks ? (blocks > 0 ? blocks : 1) : kChunkBlocks);
}

// The sorted emission with every Gaussian's test angle widened by `widen`
// radians (0: the binning of hp_bin_sorted).  No step waits for the host:
// every count that sizes a later step is read on the device, and the grids
// are sized from the workspace's bounds.
hp_status hp_bin_sorted_widened(int32_t phase, const void* projected, int64_t P, const hp_view* view,
                                const hp_params* prm, const void* grid, const void* mask, uint32_t* vals,
                                uint32_t* tile_ranges, int32_t n_tiles, int64_t capacity, int64_t* n_pairs, void* ws,
                                size_t ws_bytes, void* stream, double widen) {
  if (phase < HP_BIN_COUNT || phase > HP_BIN_ALL) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_view(view, prm));
  if (P < 0 || P > ((int64_t)1 << 31) - 1 || capacity < 0 || capacity > ((int64_t)1 << 32) - 1 || n_tiles < 0)
    return HP_ERR_INVALID_ARG;
  if (!projected || !grid || !mask || !n_pairs || !ws) return HP_ERR_INVALID_ARG;
  if ((phase & HP_BIN_EMIT) && ((capacity > 0 && !vals) || (n_tiles > 0 && !tile_ranges))) return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_tiles > g.ntile) return HP_ERR_INVALID_ARG;
  if (ws_bytes < hp_bin_sorted_workspace_bytes(P, view->order, prm->tile_log2)) return HP_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  const HpProjView pv = hp_proj_view((const char*)projected, P);
  const HpGridView gv = hp_grid_view((void*)grid, g);
  const HpMaskView mv = hp_mask_view((const char*)mask, g);
  BinWs w = bin_ws(ws, P);
  SortedWs sw = sorted_ws((char*)ws + hp_align256(bin_ws_size(P)), P, g);
  const int ls = g.kt > kSplitDepth ? g.kt - kSplitDepth : 0;
  const int depth = g.kt - ls;
  BinTables T{gv.cap, gv.sc, view->cam_type == HP_CAM_FULL ? nullptr : mv.node_active, mv.node_active,
              mv.tile_compact, g.kt, ls, (float)sin(0.5 * widen), (float)cos(0.5 * widen)};
  const uint32_t nn = (uint32_t)sw.nn;
  if (phase & HP_BIN_COUNT) {
    if (P == 0) {
      hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, n_pairs);
      HP_CHECK_LAUNCH();
      return HP_OK;
    }
    // until the count below completes, *n_pairs says that nothing may be
    // emitted (set by the depth sort's first kernel)
    if (sw.nn <= kHistNodes) {
      // tasks written in node order straight from the walk (no task sort);
      // the histogram lives in task_n and its row scans, node counts and node
      // offsets in poff, which this path does not otherwise use
      // (nn x G + 2 nn <= 3 (P + 255) + 1536 <= task capacity)
      HP_TRY(depth_order(pv, P, w, n_pairs, s));
      const unsigned G = hp_blocks(P, 256);
      const int nni = (int)sw.nn;
      uint32_t* hist = w.task_n;
      uint64_t* hoff = w.poff;
      hipLaunchKernelGGL(k_task_count, dim3(G), dim3(256), 0, s, P, (const uint32_t*)w.order, pv.disc, pv.radius, T,
                         w.tcount, sw.slots, nni, hist);
      HP_CHECK_LAUNCH();
      // per node: the row scan of the histogram and the node's task count
      // (after the histogram in poff), then the node offsets
      uint64_t* rowtot = hoff + (int64_t)nni * G;
      uint64_t* node_off = rowtot + nni;
      hipLaunchKernelGGL(k_hist_rows, dim3(nni), dim3(256), 0, s, (const uint32_t*)hist, (int64_t)G, hoff, rowtot);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_task_segments, dim3(1), dim3(256), 0, s, nni, (const uint64_t*)rowtot, node_off, w.cap_t,
                         depth, w.t_total, w.nt, w.over, sw.seg, sw.choff, w.ncol);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_task_scatter, dim3(G), dim3(256), (size_t)nni * kScatterLdsPerNode, s, P,
                         (const uint32_t*)w.order, pv.disc, pv.radius, T, (const uint32_t*)w.tcount,
                         (const uint32_t*)sw.slots, nni, (const uint64_t*)hoff, (const uint64_t*)node_off, w.cap_t,
                         w.task_g);
      HP_CHECK_LAUNCH();
    } else {
      HP_TRY(bin_tasks(pv, P, T, prm->bin_guard, w, sw.slots, n_pairs, s));
      // stable sort of the tasks by node; segments and chunk offsets per node
      int nbits = 0;
      while (((int64_t)1 << nbits) < sw.nn) ++nbits;
      // the sorted node keys are only needed here: read them where the last
      // pass left them; the Gaussian ids go back to task_g for the emit phase
      uint32_t *snode = w.task_n, *sgid = w.task_g;
      HP_TRY(hpsort::radix_sort(w.task_n, w.task_g, w.nt, w.cap_t, nbits, sw.tsort_ws, s, &snode, &sgid));
      if (sgid != w.task_g) {
        hipLaunchKernelGGL(hpsort::k_copy_u32, dim3(hpsort::copy_grid(w.cap_t)), dim3(256), 0, s, (const uint32_t*)sgid,
                           w.task_g, (const uint64_t*)w.nt, w.cap_t);
        HP_CHECK_LAUNCH();
      }
      hipLaunchKernelGGL(k_fill_zero_u32, dim3(hp_blocks(2 * sw.nn, 256)), dim3(256), 0, s, sw.seg, 2 * sw.nn);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_seg_ranges, dim3(hpsort::copy_grid(w.cap_t)), dim3(256), 0, s, (const uint32_t*)snode,
                         (const uint64_t*)w.nt, nn, sw.seg);
      HP_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_seg_chunks, dim3(hp_blocks(sw.nn, 256)), dim3(256), 0, s, sw.seg, nn, sw.nch);
      HP_CHECK_LAUNCH();
      HP_TRY((hpsort::scan_exclusive<uint32_t, uint32_t>(sw.nch, sw.choff, nullptr, sw.nn, sw.choff + sw.nn, sw.scan_ws,
                                                         s)));
      // hit columns and their counts (every count entry of the chunks present
      // is written), scanned in tile-major order into output slots
      hipLaunchKernelGGL(k_col_count, dim3(1), dim3(1), 0, s, (const uint32_t*)sw.choff, nn, depth, w.ncol);
      HP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_chunk_nodes, dim3(nn), dim3(256), 0, s, (const uint32_t*)sw.choff, sw.cnode);
    HP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bin_cols, dim3(chunk_grid(sw.nchunk_max)), dim3(256), 0, s, (const uint32_t*)sw.choff, nn,
                       (const uint32_t*)sw.seg, (const uint32_t*)sw.cnode, (const uint32_t*)w.task_g, pv.disc, T,
                       sw.wcol, sw.cnt);
    HP_CHECK_LAUNCH();
    // the pair total goes to *n_pairs with the scan (a count no buffer holds
    // when the tasks overflowed: the emission kernels then write nothing)
    HP_TRY((hpsort::scan_exclusive<uint64_t, uint32_t>(sw.cnt, sw.start, w.ncol, sw.L, w.p_total, sw.scan_ws, s,
                                                       n_pairs, (const uint32_t*)w.over)));
  }
  if ((phase & HP_BIN_EMIT) && P > 0) {
    // the chunk count is read on the device: launch for the workspace's bound
    // the emission also writes the tile ranges
    const TileRanges tr{n_tiles, mv.active_tiles, (const uint64_t*)w.ncol, (const uint64_t*)w.p_total, tile_ranges};
    hipLaunchKernelGGL(k_bin_emit_sorted, dim3(chunk_grid(sw.nchunk_max)), dim3(256), 0, s, (const uint32_t*)sw.choff,
                       nn, (const uint32_t*)sw.seg, (const uint32_t*)sw.cnode, (const uint32_t*)w.task_g, depth,
                       (const uint64_t*)sw.wcol, (const uint64_t*)sw.start, (const int64_t*)n_pairs, capacity, vals, tr);
    HP_CHECK_LAUNCH();
  } else if ((phase & HP_BIN_EMIT) && n_tiles > 0) {
    hipLaunchKernelGGL(k_fill_zero_u32, dim3(hp_blocks(2 * (int64_t)n_tiles, 256)), dim3(256), 0, s, tile_ranges,
                       2 * (int64_t)n_tiles);
    HP_CHECK_LAUNCH();
  }
  return HP_OK;
}

extern "C" hp_status hp_bin_sorted(int32_t phase, const void* projected, int64_t P, const hp_view* view,
                                   const hp_params* prm, const void* grid, const void* mask, uint32_t* vals,
                                   uint32_t* tile_ranges, int32_t n_tiles, int64_t capacity, int64_t* n_pairs,
                                   void* ws, size_t ws_bytes, void* stream) {
  return hp_bin_sorted_widened(phase, projected, P, view, prm, grid, mask, vals, tile_ranges, n_tiles, capacity,
                               n_pairs, ws, ws_bytes, stream, 0.0);
}
