// k_query.hip -- the paper's own tile queries (Sec. 3.3; Alg. 2 NESTED
// quadtree traversal, Alg. 3 RING sequential scan) at search depth f, as
// per-tile lists for the renderer.
//
// Both queries decide on centres at the query order kq = kt + log2 f, so their
// tile sets are narrower than the binning of hp_bin_sorted and can leave out
// tiles a Gaussian reaches (the aliasing of coarse queries in the ablation).
// Instead of a ring walk or a stack per Gaussian, membership is evaluated tile
// by tile: Gaussian i's set holds tile t exactly when one of t's query points
// passes the test the query applies to it --
//   RING:   a pixel of order kq on a ring whose latitude lies within r_s of
//           the disc centre's, at a position inside the ring's window
//           [floor, ceil] of Eq. ring_phi_range (whole ring when the ring lies
//           inside the disc);
//   NESTED: a node of order kt .. kq whose centre lies within r_s (what the
//           traversal reports when PixRad bounds the distance from a node
//           centre to its descendants' centres at order kq).
// Candidates are the pairs of hp_bin_sorted with every test angle widened by a
// margin that contains both sets (one ring step for RING, plus the distance
// from a query point to the nearest pixel centre of its tile); they arrive in
// per-tile depth order, and one block per tile keeps the entries that pass,
// compacting the tile's list in place, so the order is preserved.
#include "hp_common.h"

namespace {

constexpr int kMaxPts = 341;    // nodes of orders kt .. kt + 4 below one tile
constexpr int kMaxRings = 31;   // rings crossing one tile at f = 16

struct QueryArgs {
  int mode, kq, fl, order_t;
  const int32_t* active_tiles;
  const float4* disc;   // (direction, sin((r_s + guard) / 2)) per Gaussian
  const float* radius;
  uint32_t* vals;
  uint32_t* ranges;
  const int64_t* n_pairs;
  int64_t capacity;
  unsigned long long* n_kept;
};

// ring ir (1 .. 4N-1 from the north pole) at order kq: latitude, its cosine,
// number of pixels and the offset (in pixels) of pixel 0's centre from
// longitude 0
__device__ void ring_geom(int64_t N, int64_t ir, double* lat, double* clat, int* nring, float* off) {
  const double s6 = 2.449489742783178;  // sqrt(6)
  if (ir < N || ir > 3 * N) {
    const int64_t i = ir < N ? ir : 4 * N - ir;
    const double th = 2.0 * asin((double)i / ((double)N * s6));  // 1 - |z| = 2 sin^2(theta / 2)
    *lat = ir < N ? 0.5 * M_PI - th : th - 0.5 * M_PI;
    *clat = sin(th);
    *nring = (int)(4 * i);
    *off = 0.5f;
  } else {
    const double z = (double)(2 * N - ir) * (2.0 / (3.0 * (double)N));
    *lat = asin(z);
    *clat = sqrt((1.0 - z) * (1.0 + z));
    *nring = (int)(4 * N);
    *off = ((ir - N) & 1) ? 0.f : 0.5f;
  }
}

// ring and 0-based position along it of nested pixel p at order kq
__device__ void pix_ring(int kq, int64_t p, int64_t* ring, int* pos, int* x_minus_y) {
  int x, y, f;
  hp_nest_xyf(kq, p, &x, &y, &f);
  const int64_t N = (int64_t)1 << kq;
  const int row = f >> 2, col = f & 3;
  const int64_t ir = (int64_t)(row + 2) * N - x - y - 1;
  const int64_t lon = (row == 1) ? 2 * col : 2 * col + 1;
  int64_t jp, nring;
  if (ir < N || ir > 3 * N) {
    const int64_t nr = ir < N ? ir : 4 * N - ir;
    jp = (lon * nr + x - y + 1) / 2;
    nring = 4 * nr;
  } else {
    const int64_t s = (ir - N) & 1;
    jp = (lon * N + x - y + 1 + s) / 2;
    nring = 4 * N;
  }
  if (jp > nring) jp -= nring;
  if (jp < 1) jp += nring;
  *ring = ir;
  *pos = (int)(jp - 1);
  *x_minus_y = x - y;
}

// One ring crossing a tile at the query order, for the RING test.  The
// tile's pixels on it are a run of positions; the window of Eq. ring_phi_range
// ([floor, ceil] of its ends in pixel units) holds pixel ip exactly when
// |omega - lambda_ip| < d_omega + step (lambda_ip its centre longitude, step
// = 2 pi / nring), so it meets the run exactly when the longitude distance
// from omega to the run's interval widened by one step on both sides,
// [lambda_first - step, lambda_last + step], is below d_omega.
struct RingSlot {
  float sh, ch;    // sin, cos of half the ring's latitude
  float clat;      // cos of its latitude
  float sm, cm;    // sin, cos of half the widened interval's middle longitude
  float shw, chw;  // sin, cos of half its half-width
  int whole;       // the widened interval covers the ring (or the tile has no pixel on it: -1)
};

// RING membership of the tile for a Gaussian with direction u and
// hrs = sin^2(r_s / 2).  With hav x = sin^2(x / 2):
//   num = hav r_s - hav(lat_r - lat_c),  den = cos lat_c cos lat_r,
//   hav d_omega = num / den  (Eq. ring_phi_range in haversine form),
// so the ring lies in the disc's z range when |sin((lat_r - lat_c) / 2)| <=
// sin(r_s / 2), wholly inside the disc when num >= den, meets it nowhere when
// num <= 0, and otherwise the run is hit when den hav(distance) < num.  Every
// small angle enters as the sine of its half, formed as a difference of
// products of half-angle sines and cosines: no cancellation for small discs,
// and no transcendental per ring.
__device__ __forceinline__ bool ring_hit(const RingSlot* S, int nslot, float ux, float uy, float uz, float hrs) {
  const float clat_c = sqrtf(fmaf(ux, ux, uz * uz));
  // half of the centre's latitude: its cosine is at least 1/sqrt(2)
  const float cc = sqrtf(fmaf(0.5f, clat_c, 0.5f));
  const float sc = uy / (2.f * cc);
  const float srs = sqrtf(hrs);
  float sw, cw;  // half of the centre's longitude
  sincosf(0.5f * atan2f(ux, uz), &sw, &cw);
  for (int j = 0; j < nslot; ++j) {
    const RingSlot r = S[j];
    if (r.whole < 0) continue;
    const float sd = fmaf(r.sh, cc, -(r.ch * sc));  // sin((lat_r - lat_c) / 2)
    if (fabsf(sd) > srs) continue;                  // outside the disc's z range
    const float num = fmaf(-sd, sd, hrs);
    const float den = clat_c * r.clat;
    if (num >= den) return true;   // the whole ring lies in the disc (also at the poles)
    if (!(num > 0.f)) continue;    // d_omega = 0: no pixel
    if (r.whole) return true;
    // y = |omega - middle| reduced to [0, pi]: sin(y / 2), cos(y / 2)
    const float a = fabsf(fmaf(sw, r.cm, -(cw * r.sm)));
    const float b = fabsf(fmaf(cw, r.cm, sw * r.sm));
    if (a <= r.shw) return true;   // inside the widened interval
    const float sdist = fmaf(a, r.chw, -(b * r.shw));  // sin((y - half-width) / 2)
    if (den * (sdist * sdist) < num) return true;
  }
  return false;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_query_filter(QueryArgs A) {
  if (*A.n_pairs > A.capacity) return;  // the candidates were not written
  __shared__ float4 s_pt[MODE == HP_QUERY_NESTED ? kMaxPts : 1];
  __shared__ RingSlot s_ring[MODE == HP_QUERY_RING ? kMaxRings : 1];
  __shared__ uint32_t s_key[kMaxRings], s_len[kMaxRings];
  __shared__ uint32_t s_wcnt[4];
  const int k = hp_xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int64_t t = A.active_tiles[k];
  const int tid = threadIdx.x;
  const int f = 1 << A.fl, nsub = f * f;
  int npts = 0, nslot = 0;
  if (MODE == HP_QUERY_NESTED) {
    // centres of the nodes of orders kt .. kq below t, coarsest first
    npts = (4 * nsub - 1) / 3;
    for (int j = tid; j < npts; j += blockDim.x) {
      int o = 0, base = 0;
      while (j >= base + (1 << (2 * o))) { base += 1 << (2 * o); ++o; }
      double v[3];
      hp_pix_dir(A.order_t + o, (t << (2 * o)) + (j - base), v);
      s_pt[j] = make_float4((float)v[0], (float)v[1], (float)v[2], 0.f);
    }
  } else {
    // rings crossing t at order kq: ring_min is that of the tile's south
    // corner pixel; each ring holds a run of the tile's pixels
    nslot = 2 * f - 1;
    int xt, yt, ft;
    hp_nest_xyf(A.order_t, t, &xt, &yt, &ft);
    const int64_t N = (int64_t)1 << A.kq;
    const int64_t ring_min = (int64_t)((ft >> 2) + 2) * N - ((int64_t)xt * f + f - 1) - ((int64_t)yt * f + f - 1) - 1;
    if (tid < nslot) { s_key[tid] = 0xffffffffu; s_len[tid] = 0u; }
    __syncthreads();
    if (tid < nsub) {
      int64_t ir;
      int pos, xmy;
      pix_ring(A.kq, (t << (2 * A.fl)) + tid, &ir, &pos, &xmy);
      const int j = (int)(ir - ring_min);
      // first pixel of the run: the smallest x - y (positions grow with it)
      atomicMin(&s_key[j], ((uint32_t)(xmy + 16384) << 17) | (uint32_t)pos);
      atomicAdd(&s_len[j], 1u);
    }
    __syncthreads();
    if (tid < nslot) {
      double lat, clat;
      int nring;
      float off;
      ring_geom(N, ring_min + tid, &lat, &clat, &nring, &off);
      const int len = (int)s_len[tid];
      const int start = len ? (int)(s_key[tid] & 0x1ffffu) : 0;
      const double step = 2.0 * M_PI / (double)nring;
      const double mid = ((double)start + 0.5 * (double)(len - 1) + (double)off) * step;
      const double hw = 0.5 * (double)(len + 1) * step;
      RingSlot r;
      r.sh = (float)sin(0.5 * lat);
      r.ch = (float)cos(0.5 * lat);
      r.clat = (float)clat;
      r.sm = (float)sin(0.5 * mid);
      r.cm = (float)cos(0.5 * mid);
      r.shw = (float)sin(0.5 * (hw < M_PI ? hw : M_PI));
      r.chw = (float)cos(0.5 * (hw < M_PI ? hw : M_PI));
      r.whole = len == 0 ? -1 : (hw >= M_PI ? 1 : 0);
      s_ring[tid] = r;
    }
  }
  __syncthreads();

  const uint32_t s = A.ranges[2 * k], e = A.ranges[2 * k + 1];
  const int lane = hp_lane(), wv = tid >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t kept = 0;
  for (uint32_t base = s; base < e; base += blockDim.x) {
    const uint32_t idx = base + (uint32_t)tid;
    const bool have = idx < e;
    const uint32_t g = have ? A.vals[idx] : 0u;
    bool keep = false;
    if (have) {
      const float4 r0 = A.disc[g];
      const float rs = A.radius[g];
      if (MODE == HP_QUERY_NESTED) {
        const float c = 2.f * sinf(0.5f * rs);
        const float thr = c * c;
        for (int j = 0; j < npts && !keep; ++j) {
          const float4 p = s_pt[j];
          const float dx = p.x - r0.x, dy = p.y - r0.y, dz = p.z - r0.z;
          keep = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= thr;
        }
      } else {
        const float hs = sinf(0.5f * rs);
        keep = ring_hit(s_ring, nslot, r0.x, r0.y, r0.z, hs * hs);
      }
    }
    // every entry of this chunk has been read (the tests used them); the
    // kept ones move down to the tile's next free slots, in order
    const uint64_t m = __ballot(keep);
    if (lane == 0) s_wcnt[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = kept;
    for (int w = 0; w < wv; ++w) off += s_wcnt[w];
    const uint32_t tot = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    if (keep) A.vals[s + off + (uint32_t)__popcll(m & below)] = g;
    kept += tot;
    __syncthreads();
  }
  if (tid == 0) {
    A.ranges[2 * k + 1] = s + kept;
    if (A.n_kept) atomicAdd(A.n_kept, (unsigned long long)kept);
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

}  // namespace

extern "C" size_t hp_bin_query_workspace_bytes(int64_t P, int32_t order, int32_t tile_log2) {
  return hp_bin_sorted_workspace_bytes(P, order, tile_log2);
}

extern "C" hp_status hp_bin_query(int32_t phase, int32_t mode, int32_t f, const void* projected, int64_t P,
                                  const hp_view* view, const hp_params* prm, const void* grid, const void* mask,
                                  uint32_t* vals, uint32_t* tile_ranges, int32_t n_tiles, int64_t capacity,
                                  int64_t* n_pairs, int64_t* n_kept, void* ws, size_t ws_bytes, void* stream) {
  if (mode != HP_QUERY_RING && mode != HP_QUERY_NESTED) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_view(view, prm));
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  int fl = 0;
  while (fl < 5 && (1 << fl) < f) ++fl;
  if (f < 1 || (1 << fl) != f || fl > g.b) return HP_ERR_INVALID_ARG;  // query order at most the pixel order
  const int kq = g.kt + fl;
  // margin: one ring step at the query order (RING), plus the distance from a
  // query point to the nearest pixel centre of its tile (at most a pixel
  // radius, below 1.2 / Nside), plus float slack
  const double step = mode == HP_QUERY_RING ? M_PI / (2.0 * (double)((int64_t)1 << kq)) : 0.0;
  const double widen = step + 1.2 / (double)((int64_t)1 << view->order) + 1e-4;
  HP_TRY(hp_bin_sorted_widened(phase, projected, P, view, prm, grid, mask, vals, tile_ranges, n_tiles, capacity,
                               n_pairs, ws, ws_bytes, stream, widen));
  if (!(phase & HP_BIN_EMIT)) return HP_OK;
  hipStream_t s = (hipStream_t)stream;
  if (n_kept) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, n_kept);
    HP_CHECK_LAUNCH();
  }
  if (P == 0 || n_tiles == 0) return HP_OK;
  const HpProjView pv = hp_proj_view((const char*)projected, P);
  const HpMaskView mv = hp_mask_view((const char*)mask, g);
  QueryArgs A{mode, kq, fl, g.kt, mv.active_tiles, pv.disc, pv.radius, vals, tile_ranges, n_pairs, capacity,
              (unsigned long long*)n_kept};
  if (mode == HP_QUERY_RING)
    hipLaunchKernelGGL(k_query_filter<HP_QUERY_RING>, dim3((unsigned)n_tiles), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL(k_query_filter<HP_QUERY_NESTED>, dim3((unsigned)n_tiles), dim3(256), 0, s, A);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
