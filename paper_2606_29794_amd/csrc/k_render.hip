// k_render.hip -- stage 3 of Alg. 1 (front-to-back compositing on the
// HEALPix grid, Eq. unified_rendering) and its per-pixel backward pass.
//
// One 256-thread workgroup per active tile, one pixel per lane; the four
// waves each own 64 consecutive active pixels of the tile.  The tile's
// depth-sorted list is walked in chunks of 64 entries: all 256 threads stage
// a chunk's 64-byte records into LDS (one 16-byte quarter each, the next
// chunk's records requested before the current one is evaluated), a barrier
// publishes it, and every wave reads the records as LDS broadcasts.  Per
// chunk, a wave first tests every entry against its 64 pixels as a whole and
// visits only the entries that can reach one of them.  The forward stops a
// wave once its pixels are saturated and the block once all four waves are
// (a vote taken with the chunk's barrier); the backward walks the chunks
// from the back, reduces each entry's gradients across the wave and the
// block, and adds them to per-Gaussian accumulators with global atomics.
#include "hp_common.h"
#include "hp_offset.h"

struct RenderArgs {
  int order;
  const int32_t* active_tiles;
  const int32_t* tile_start;
  const int32_t* tile_count;
  const int32_t* active_pix;
  const float4* rec;
  const float* depth;  // radial depth r of every Gaussian (inverse-depth channel)
  const uint32_t* vals;
  const uint32_t* ranges;
  float eps_T, alpha_max, q_cut;
  int64_t n_active;
};

__device__ __forceinline__ void pixel_of_lane(const RenderArgs& A, int ct, bool* valid, int64_t* slot, float* p) {
  const int t = A.active_tiles[ct];
  const int cnt = A.tile_count[t];
  const int local = threadIdx.x;
  *slot = (int64_t)A.tile_start[t] + local;
  // the output arrays hold n_active pixels: a pixel past them is never written
  *valid = local < cnt && *slot < A.n_active;
  p[0] = p[1] = p[2] = 0.f;
  if (*valid) {
    double v[3];
    hp_pix_dir(A.order, A.active_pix[*slot], v);
    p[0] = (float)v[0]; p[1] = (float)v[1]; p[2] = (float)v[2];
  }
}

static RenderArgs make_args(const HpGeom& g, const HpMaskView& mv, const HpProjView& pv, const uint32_t* vals,
                            const uint32_t* ranges, const hp_params* prm, int64_t n_active) {
  RenderArgs A;
  A.order = g.order;
  A.active_tiles = mv.active_tiles;
  A.tile_start = mv.tile_start;
  A.tile_count = mv.tile_count;
  A.active_pix = mv.active_pix;
  A.rec = pv.rec;
  A.depth = pv.depth;
  A.vals = vals;
  A.ranges = ranges;
  A.eps_T = prm->eps_T;
  A.alpha_max = prm->alpha_max;
  A.q_cut = prm->q_cut;
  A.n_active = n_active;
  return A;
}

struct RenderOut {
  float* rgb;
  float* T;
  int32_t* ncon;
  int32_t* nused;  // nullable: Gaussians composited per pixel
  float* invd;     // nullable: composited inverse radial depth (Sec. 3.2 depth supervision)
};

// A tile's list is walked in chunks of HP_CHUNK entries staged in LDS: each of
// the block's 256 threads fetches one 16-byte quarter of one record, so a
// chunk costs one round of loads for the whole block.  The records of chunk
// c + 1 (whose ids arrived a chunk earlier) and the ids of chunk c + 2 are
// requested before chunk c is evaluated, so their latency overlaps the
// evaluation; the waves then read each record as an LDS broadcast.
#define HP_CHUNK 64
#define HP_STAGE (4 * HP_CHUNK)  // float4 per chunk buffer = threads per block

__device__ __forceinline__ float4 stage_load(const float4* __restrict__ rec, uint32_t g, int q) {
  return rec[4 * (size_t)g + q];
}

// Bounding cap of the wave's pixels: centre = normalised sum of their
// directions, (sin, cos) of half the largest angle to them, rounded up.  A
// list entry whose r_s disc misses this cap has q > 9 at every pixel of the
// wave (the 3-sigma ellipse lies inside the disc), so the wave skips it.
struct WaveCap {
  float cx, cy, cz, sr, cr;
};
__device__ __forceinline__ WaveCap wave_cap(bool valid, const float p[3]) {
  WaveCap w;
  const float sx = hp_wave_sum(valid ? p[0] : 0.f), sy = hp_wave_sum(valid ? p[1] : 0.f),
              sz = hp_wave_sum(valid ? p[2] : 0.f);
  const float inv = rsqrtf(sx * sx + sy * sy + sz * sz);  // no valid pixel: NaN centre, no entry passes
  w.cx = sx * inv; w.cy = sy * inv; w.cz = sz * inv;
  const float dx = p[0] - w.cx, dy = p[1] - w.cy, dz = p[2] - w.cz;
  float c2 = valid ? dx * dx + dy * dy + dz * dz : 0.f;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c2 = fmaxf(c2, __shfl_xor(c2, off, 64));
  w.sr = fminf(1.f, 0.5f * sqrtf(c2) * 1.0001f + 1e-6f);  // sin(R/2) = chord / 2
  w.cr = sqrtf(fmaxf(0.f, 1.f - w.sr * w.sr));
  return w;
}
// entry with unit direction u and sg = sin((r_s + guard) / 2) (record word 15)
__device__ __forceinline__ bool wave_cap_hit(const WaveCap& w, float4 r0, float sg) {
  const float cg = sqrtf(fmaxf(0.f, 1.f - sg * sg));
  const float dx = w.cx - r0.x, dy = w.cy - r0.y, dz = w.cz - r0.z;
  const float sh = w.sr * cg + w.cr * sg;  // sin((R + theta) / 2)
  const float ch = w.cr * cg - w.sr * sg;  // cos((R + theta) / 2)
  return (ch <= 0.f) || (dx * dx + dy * dy + dz * dz <= 4.f * sh * sh);
}

// Second per-wave test, on the 3-sigma ellipse instead of the r_s disc:
// (a, b) = E p with E's rows orthonormal, so |(a, b)(p) - (a, b)(w)| <= |p - w|
// and sqrt(qt) = |L (a, b)| (conic = L^T L) changes by at most
// sqrt(lambda_max(conic)) |p - w|.  Every pixel of the wave lies within the
// chord 2 sr of the cap centre w, so if sqrt(qt(w)) exceeds sqrt(q_cut) +
// 2 sr sqrt(lambda_max) no pixel of the wave reaches qt <= q_cut.  The bound
// is widened by 1e-4 relative against float rounding.
__device__ __forceinline__ bool wave_ellipse_hit(const WaveCap& w, float4 r1, float4 r2, float rq_cut) {
  const float wp[3] = {w.cx, w.cy, w.cz};
  const HpOffset o = hp_offset(wp, r1, r2);
  const float h = 0.5f * (r2.y - r2.w);
  const float lmax = 0.5f * (r2.y + r2.w) + sqrtf(h * h + r2.z * r2.z);
  const float lim = rq_cut + 2.f * w.sr * sqrtf(fmaxf(lmax, 0.f));
  return o.qt <= lim * lim * 1.0001f + 1e-6f;
}

// DEPTH: also composite 1/r like a colour channel; the entries' 1/r ride
// along with their records through LDS.
template <bool DEPTH>
__device__ __forceinline__ void render_fwd_tile(const RenderArgs& A, const RenderOut& O, int ct, float4* s_rec,
                                                float* s_invd) {
  bool valid;
  int64_t slot;
  float p[3];
  pixel_of_lane(A, ct, &valid, &slot, p);
  const uint32_t j0 = hp_uniform(A.ranges[2 * ct]), j1 = hp_uniform(A.ranges[2 * ct + 1]);
  const uint32_t n = j1 - j0;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, Dinv = 0.f;
  bool done = !valid;
  uint32_t used = n;
  int nu = 0;
  const int tid = threadIdx.x;
  const uint32_t e = (uint32_t)tid >> 2;  // entry of a chunk this thread stages
  const int q = tid & 3;                  // and which quarter of its record
  const uint32_t* vals = A.vals + j0;
  const int lane = hp_lane();
  const WaveCap wc = wave_cap(valid, p);
  const float rq_cut = sqrtf(A.q_cut);
  // per wave: does any pixel still composite; two sets by chunk parity, so
  // that a wave already writing the next chunk's flag never overwrites one
  // that a slower wave has yet to read
  __shared__ int s_live[2][4];
  {
    const uint32_t g0 = e < n ? vals[e] : 0u;
    s_rec[tid] = e < n ? stage_load(A.rec, g0, q) : make_float4(0.f, 0.f, 0.f, 0.f);
    if (DEPTH && q == 0) s_invd[e] = e < n ? 1.f / A.depth[g0] : 0.f;
  }
  uint32_t gnext = HP_CHUNK + e < n ? vals[HP_CHUNK + e] : 0u;
  __syncthreads();
  const uint32_t nch = (n + HP_CHUNK - 1) / HP_CHUNK;
  for (uint32_t c = 0; c < nch; ++c) {
    const uint32_t base = c * HP_CHUNK;
    float4 stage = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t gstage = gnext;
    float dstage = 1.f;
    if (base + HP_CHUNK + e < n) {
      stage = stage_load(A.rec, gstage, q);
      if (DEPTH && q == 0) dstage = A.depth[gstage];
    }
    gnext = base + 2 * HP_CHUNK + e < n ? vals[base + 2 * HP_CHUNK + e] : 0u;
    const float4* cur = s_rec + (c & 1) * HP_STAGE;
    const float* curd = s_invd + (c & 1) * HP_CHUNK;
    const uint32_t cnt = n - base < HP_CHUNK ? n - base : HP_CHUNK;
    // entry i: Mahalanobis bound first (q >= qt), then the exact q and the
    // compositing step; entries go two at a time so that the second one's
    // loads and bound overlap the first one's work.  Entries the wave skips
    // have qt > q_cut at every pixel of the wave, so skipping them changes
    // nothing; n_contrib still counts list positions.
    auto step = [&](uint32_t i, const HpOffset& o) {
      if (done || !(o.qt <= A.q_cut)) return;
      const float4 r0 = cur[4 * i], r3 = cur[4 * i + 3];
      const float qq = o.qt * hp_k2(hp_offset_s2(o), hp_offset_c(p, r0));
      if (!(qq <= A.q_cut)) return;
      const float alpha = fminf(A.alpha_max, r0.w * hp_exp_neg_half(qq));
      const float w = alpha * T;
      C0 += w * r3.x;
      C1 += w * r3.y;
      C2 += w * r3.z;
      if (DEPTH) Dinv += w * curd[i];
      T -= w;
      ++nu;
      if (T < A.eps_T) {
        done = true;
        used = base + i + 1;
      }
    };
    // only entries that can reach a pixel of this wave (lane j tests entry j
    // against the wave's cap and ellipse bound), front to back
    uint64_t todo = __ballot((uint32_t)lane < cnt && wave_cap_hit(wc, cur[4 * lane], cur[4 * lane + 3].w) &&
                             wave_ellipse_hit(wc, cur[4 * lane + 1], cur[4 * lane + 2], rq_cut));
    while (todo != 0) {
      if (__ballot(!done) == 0) break;
      const uint32_t ia = (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      const HpOffset oa = hp_offset(p, cur[4 * ia + 1], cur[4 * ia + 2]);
      if (todo != 0) {
        const uint32_t ib = (uint32_t)__builtin_ctzll(todo);
        todo &= todo - 1;
        const HpOffset ob = hp_offset(p, cur[4 * ib + 1], cur[4 * ib + 2]);
        step(ia, oa);
        step(ib, ob);
      } else {
        step(ia, oa);
      }
    }
    // one barrier both publishes the next chunk and tells whether any pixel
    // of the block still composites
    s_rec[((c + 1) & 1) * HP_STAGE + tid] = stage;
    if (DEPTH && q == 0) s_invd[((c + 1) & 1) * HP_CHUNK + e] = 1.f / dstage;
    const int par = c & 1;
    const uint64_t live = __ballot(!done);  // all lanes vote, before one lane writes
    if (lane == 0) s_live[par][tid >> 6] = live != 0;
    __syncthreads();
    if (!(s_live[par][0] | s_live[par][1] | s_live[par][2] | s_live[par][3])) break;
  }
  if (valid) {
    O.rgb[slot] = C0;
    O.rgb[A.n_active + slot] = C1;
    O.rgb[2 * A.n_active + slot] = C2;
    O.T[slot] = T;
    O.ncon[slot] = (int32_t)used;
    if (O.nused) O.nused[slot] = nu;
    if (DEPTH) O.invd[slot] = Dinv;
  }
}

template <bool DEPTH>
__global__ __launch_bounds__(256) void k_render_fwd(RenderArgs A, RenderOut O) {
  __shared__ float4 s_rec[2 * HP_STAGE];
  __shared__ float s_invd[2 * HP_CHUNK];
  render_fwd_tile<DEPTH>(A, O, hp_xcd_tile(blockIdx.x, gridDim.x), s_rec, s_invd);
}

// Several requests in one launch: block b renders tile b - first[r] of
// request r, where first[] is the prefix of the requests' tile counts.
#define HP_MAX_BATCH 16
struct RenderBatch {
  int n;
  int first[HP_MAX_BATCH + 1];
  RenderArgs A[HP_MAX_BATCH];
  RenderOut O[HP_MAX_BATCH];
};

__global__ __launch_bounds__(256) void k_render_fwd_batch(RenderBatch B) {
  __shared__ float4 s_rec[2 * HP_STAGE];
  const int b = hp_xcd_tile(blockIdx.x, gridDim.x);
  int r = 0;
  while (r + 1 < B.n && b >= B.first[r + 1]) ++r;
  render_fwd_tile<false>(B.A[r], B.O[r], b - B.first[r], s_rec, nullptr);
}

// Per-Gaussian gradient accumulators written by the pixel pass:
// [0..2] colour, [3] opacity, [4..6] conic (A, B, C), [7] omega, [8] phi,
// [9] inverse radial depth 1/r (written only with a depth gradient).
#define HP_NACC 10
// constant factor of each value as the per-pixel terms leave it out
__constant__ float kFlushScale[HP_NACC] = {1.f, 1.f, 1.f, 1.f, -0.5f, -1.f, -0.5f, -1.f, -1.f, 1.f};
template <bool B>
struct HpBool {
  static constexpr bool value = B;
};

// DEPTH: the upstream gradient also holds dL/d(inverse depth) per pixel; the
// inverse depth enters the compositing like a colour channel, and the tenth
// accumulator receives dL/d(1/r) per Gaussian.
template <bool DEPTH>
__global__ __launch_bounds__(256) void k_render_bwd(RenderArgs A, int64_t P, const float* __restrict__ Tfin,
                                                    const int32_t* __restrict__ ncon, const float* __restrict__ gC,
                                                    const float* __restrict__ gTfin, const float* __restrict__ gDinv,
                                                    float* __restrict__ acc) {
  constexpr int NA = DEPTH ? 10 : 9;  // values reduced per (wave, entry)
  __shared__ float4 s_rec[2 * HP_STAGE];
  __shared__ int s_nc[4];
  // per chunk entry: the block's gradient totals (the 4 waves' sums), sent to
  // memory with one atomic per non-zero value once the chunk is done
  __shared__ float s_acc[HP_CHUNK * NA];
  __shared__ uint32_t s_gid[2][HP_CHUNK];  // Gaussian id of every staged entry
  __shared__ float s_invd[2][HP_CHUNK];    // 1/r of every staged entry (DEPTH)
  const int ct = hp_xcd_tile(blockIdx.x, gridDim.x);
  bool valid;
  int64_t slot;
  float p[3];
  pixel_of_lane(A, ct, &valid, &slot, p);
  const uint32_t j0 = hp_uniform(A.ranges[2 * ct]);
  int nc = 0;
  float Tf = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gT = 0.f, gD = 0.f;
  if (valid) {
    nc = ncon[slot];
    Tf = Tfin[slot];
    g0 = gC[slot];
    g1 = gC[A.n_active + slot];
    g2 = gC[2 * A.n_active + slot];
    gT = gTfin ? gTfin[slot] : 0.f;
    if (DEPTH) gD = gDinv[slot];
  }
  // trip counts: the largest n_contrib of the wave and of the block
  int ncmax = nc;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) ncmax = max(ncmax, __shfl_xor(ncmax, off, 64));
  ncmax = (int)hp_uniform((uint32_t)ncmax);
  const int tid = threadIdx.x, lane = hp_lane();
  const WaveCap wc = wave_cap(valid, p);
  const float rq_cut = sqrtf(A.q_cut);
  if (lane == 0) s_nc[tid >> 6] = ncmax;
  for (int t = tid; t < HP_CHUNK * NA; t += 256) s_acc[t] = 0.f;
  __syncthreads();
  const int nb = max(max(s_nc[0], s_nc[1]), max(s_nc[2], s_nc[3]));
  float Tcur = Tf;  // transmittance after the current entry
  // g . (colour composited behind the current entry) + dL/dT_final * T_final
  // (with DEPTH the inverse depth counts as a fourth colour channel)
  float SgT = gT * Tf;
  const float amax = A.alpha_max;
  // entries nb-1 .. 0 in chunks of HP_CHUNK aligned at j0, last chunk first;
  // the staging runs a chunk ahead as in the forward pass
  const uint32_t e = (uint32_t)tid >> 2;
  const int qs = tid & 3;
  const uint32_t* vals = A.vals + j0;
  const int ctop = nb > 0 ? (nb - 1) / HP_CHUNK : -1;
  uint32_t gnext = 0u;
  if (ctop >= 0) {
    const uint32_t k0 = (uint32_t)ctop * HP_CHUNK + e;
    const uint32_t g = k0 < (uint32_t)nb ? vals[k0] : 0u;
    s_rec[tid] = k0 < (uint32_t)nb ? stage_load(A.rec, g, qs) : make_float4(0.f, 0.f, 0.f, 0.f);
    if (qs == 3) s_gid[0][e] = g;
    if (DEPTH && qs == 2) s_invd[0][e] = k0 < (uint32_t)nb ? 1.f / A.depth[g] : 0.f;
    if (ctop >= 1) gnext = vals[(uint32_t)(ctop - 1) * HP_CHUNK + e];
  }
  __syncthreads();
  for (int ch = ctop; ch >= 0; --ch) {
    float4 stage = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t gstage = gnext;
    float dstage = 1.f;
    if (ch >= 1) {
      stage = stage_load(A.rec, gstage, qs);  // chunk ch - 1 is full
      if (DEPTH && qs == 2) dstage = A.depth[gstage];
    }
    if (ch >= 2) gnext = vals[(uint32_t)(ch - 2) * HP_CHUNK + e];
    const float4* cur = s_rec + ((ctop - ch) & 1) * HP_STAGE;
    const float* curd = s_invd[(ctop - ch) & 1];
    const int kbase = ch * HP_CHUNK;
    const int ktop = min(kbase + HP_CHUNK, ncmax) - 1;  // this wave's last entry in the chunk
    const int nrel = nc - kbase;                          // entries of the chunk this pixel composited
    // lane j tests entry kbase + j against the wave's cap and ellipse bound; walk the hits from the back
    uint64_t todo = 0;
    if (ktop >= kbase)
      todo = __ballot(lane <= ktop - kbase && wave_cap_hit(wc, cur[4 * lane], cur[4 * lane + 3].w) &&
                      wave_ellipse_hit(wc, cur[4 * lane + 1], cur[4 * lane + 2], rq_cut));
    while (todo != 0) {
      const int i = 63 - __builtin_clzll(todo);
      todo &= ~(1ull << i);
      const float4 r0 = cur[4 * i], r1 = cur[4 * i + 1], r2 = cur[4 * i + 2], r3 = cur[4 * i + 3];
      const HpOffset o = hp_offset(p, r1, r2);
      const float a = o.a, b = o.b, qt = o.qt;
      const bool pass1 = i < nrel && qt <= A.q_cut;  // entry k = kbase + i < nc, and q >= qt
      // lane predicates are combined as wave masks (scalar ANDs), which keeps
      // every test below a single compare
      const uint64_t m1 = __builtin_amdgcn_ballot_w64(i < nrel) & __builtin_amdgcn_ballot_w64(qt <= A.q_cut);
      if (m1 == 0) continue;
      const float c = hp_offset_c(p, r0);
      const float s2 = hp_offset_s2(o);
      // Wave-uniform skips only; inside, every lane computes and the lanes
      // without a hit carry zero weight (their inputs are made finite first),
      // which avoids masked branches.  FAR: some lane of the wave is outside
      // the series range of k2, so k2 depends on c as well.
      auto composite = [&](auto far_tag) {
        constexpr bool FAR = decltype(far_tag)::value;
        float k2, d1, d2 = 0.f;  // k2, dk2/ds2, dk2/dc
        if constexpr (FAR) {
          k2 = hp_k2_grad(s2, c, &d1, &d2);
        } else {
          k2 = hp_k2_series(s2);
          d1 = hp_k2_series_deriv(s2);
        }
        const bool inq = qt * k2 <= A.q_cut;
        if ((__builtin_amdgcn_ballot_w64(inq) & m1) == 0) return;
        const bool hit = pass1 && inq;
        // series k2 is finite everywhere; far from the centre it is not
        // (antipode), so there the lanes without a hit take neutral values
        float k2h = k2;
        if constexpr (FAR) {
          k2h = hit ? k2 : 1.f;
          d1 = hit ? d1 : 0.f;
          d2 = hit ? d2 : 0.f;
        }
        const float q = qt * k2h;  // finite on every lane
        const float G = hp_exp_neg_half(q);
        const float oG = r0.w * G;
        const bool lin = oG < amax;  // below the clamp alpha depends on q and opacity
        const float alpha = lin ? oG : amax;
        const float iom = __builtin_amdgcn_rcpf(1.f - alpha);
        const float Tb = Tcur * iom;  // transmittance before this entry
        const float wgt = hit ? alpha * Tb : 0.f;
        float v[NA];
        v[0] = g0 * wgt;
        v[1] = g1 * wgt;
        v[2] = g2 * wgt;
        // dL/dalpha = Tb (g . rgb) - (g . S + dL/dT_final T_final) / (1 - alpha)
        float gr = g0 * r3.x + g1 * r3.y + g2 * r3.z;
        if (DEPTH) gr += gD * curd[i];
        const float dLda = (hit && lin) ? Tb * gr - iom * SgT : 0.f;
        SgT += wgt * gr;
        Tcur = hit ? Tb : Tcur;
        v[3] = dLda * G;
        // m = -2 dL/dq; values 4..8 leave out their constant factors, which
        // the flush applies once per Gaussian (kFlushScale)
        const float m = alpha * dLda;
        const float mk = m * k2h;
        const float ma = mk * a, mb = mk * b;
        v[4] = ma * a;  // dL/dA = -v4 / 2
        v[5] = ma * b;  // dL/dB = -v5
        v[6] = mb * b;  // dL/dC = -v6 / 2
        // dq/da = 2 fa, dq/db = 2 fb, dq/dc = 2 hc, with k2 = k2(s2, c)
        const float e = qt * d1;
        const float fa = k2h * o.u1 + e * a;
        const float fb = k2h * o.u2 + e * b;
        // motion of (a, b, c) with the Gaussian's longitude / latitude:
        // da/dw = -cos(phi) c + sin(phi) b, db/dw = -sin(phi) a, dc/dw = cos(phi) a
        // da/dp = 0, db/dp = -c, dc/dp = b
        const float cph = r1.w, sph = r0.y;
        float t2, t3;
        if constexpr (FAR) {
          const float hc = 0.5f * qt * d2;
          t2 = hc * a - fa * c;
          t3 = hc * b - fb * c;
        } else {
          t2 = -(fa * c);
          t3 = -(fb * c);
        }
        v[7] = m * (sph * (fa * b - fb * a) + cph * t2);  // dL/domega = -v7
        v[8] = m * t3;                                     // dL/dphi = -v8
        if constexpr (DEPTH) v[9] = gD * wgt;              // dL/d(1/r)
        // values 0..7: lane 8m holds the wave's total of value m; value 8: every lane
        const float t8 = hp_wave_totals8_spread(v);
        const float t9 = hp_wave_total_all(v[8]);
        if constexpr (DEPTH) {
          const float t10 = hp_wave_total_all(v[9]);
          if ((lane & 7) == 0 || lane == 1 || lane == 2)
            atomicAdd(&s_acc[i * NA + (lane == 1 ? 8 : (lane == 2 ? 9 : lane >> 3))],
                      lane == 1 ? t9 : (lane == 2 ? t10 : t8));
        } else {
          if ((lane & 7) == 0 || lane == 1)
            atomicAdd(&s_acc[i * NA + (lane == 1 ? 8 : lane >> 3)], lane == 1 ? t9 : t8);
        }
      };
      if (((__builtin_amdgcn_ballot_w64(!(c > 0.f)) | __builtin_amdgcn_ballot_w64(!(s2 < HP_K2_S2MAX))) & m1) == 0)
        composite(HpBool<false>{});
      else
        composite(HpBool<true>{});
    }
    s_rec[((ctop - ch + 1) & 1) * HP_STAGE + tid] = stage;
    if (qs == 3) s_gid[(ctop - ch + 1) & 1][e] = gstage;
    if (DEPTH && qs == 2) s_invd[(ctop - ch + 1) & 1][e] = 1.f / dstage;
    __syncthreads();  // the chunk's totals are complete and the next chunk is staged
    for (int t = tid; t < HP_CHUNK * NA; t += 256) {
      const float x = s_acc[t];
      if (x != 0.f) {
        const int i = t / NA, m = t - i * NA;
        const uint32_t g = s_gid[(ctop - ch) & 1][i];
        unsafeAtomicAdd(&acc[(int64_t)m * P + g], x * kFlushScale[m]);
        s_acc[t] = 0.f;
      }
    }
    __syncthreads();  // totals sent and cleared before the next chunk adds to them
  }
}

extern "C" hp_status hp_render_fwd(const void* projected, int64_t P, const uint32_t* vals, const uint32_t* tile_ranges,
                                   int32_t n_tiles, const hp_view* view, const hp_params* prm, const void* mask,
                                   int64_t n_active, float* rgb, float* T, int32_t* n_contrib, int32_t* n_used,
                                   float* inv_depth, void* stream) {
  HP_TRY(hp_check_view(view, prm));
  if (P < 0 || n_tiles < 0 || n_active < 0) return HP_ERR_INVALID_ARG;
  if (!projected || !mask || (n_tiles > 0 && !tile_ranges)) return HP_ERR_INVALID_ARG;
  if (n_active > 0 && (!rgb || !T || !n_contrib)) return HP_ERR_INVALID_ARG;
  if (n_tiles == 0) return HP_OK;
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_tiles > g.ntile || n_active > g.npix) return HP_ERR_INVALID_ARG;
  RenderArgs A = make_args(g, hp_mask_view((const char*)mask, g), hp_proj_view((const char*)projected, P), vals,
                           tile_ranges, prm, n_active);
  RenderOut O{rgb, T, n_contrib, n_used, inv_depth};
  if (inv_depth)
    hipLaunchKernelGGL(k_render_fwd<true>, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, A, O);
  else
    hipLaunchKernelGGL(k_render_fwd<false>, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, A, O);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_render_fwd_batch(int32_t n_req, const hp_render_req* reqs, const hp_params* prm,
                                         void* stream) {
  if (n_req < 1 || n_req > HP_MAX_BATCH || !reqs) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_params(prm));
  RenderBatch B;
  B.n = n_req;
  int64_t total = 0;
  for (int r = 0; r < n_req; ++r) {
    const hp_render_req& q = reqs[r];
    if (q.order < 0 || q.order > HP_MAX_ORDER || q.P < 0 || q.n_tiles < 0 || q.n_active < 0 || !q.projected ||
        !q.mask)
      return HP_ERR_INVALID_ARG;
    if (q.n_tiles > 0 && (!q.tile_ranges || !q.vals || !q.rgb || !q.T || !q.n_contrib)) return HP_ERR_INVALID_ARG;
    const HpGeom g = hp_geom(q.order, prm->tile_log2);
    if (q.n_tiles > g.ntile || q.n_active > g.npix) return HP_ERR_INVALID_ARG;
    B.first[r] = (int)total;
    B.A[r] = make_args(g, hp_mask_view((const char*)q.mask, g), hp_proj_view((const char*)q.projected, q.P), q.vals,
                       q.tile_ranges, prm, q.n_active);
    B.O[r] = RenderOut{q.rgb, q.T, q.n_contrib, nullptr, nullptr};
    total += q.n_tiles;
  }
  B.first[n_req] = (int)total;
  if (total == 0) return HP_OK;
  if (total > 0x7fffffff) return HP_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_render_fwd_batch, dim3((unsigned)total), dim3(256), 0, (hipStream_t)stream, B);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

// ---------------------------------------------------------------------------
// Persistent serving render: a device queue of (request, tile) items that a
// long-running launch would drain while the requests' preparation
// (preprocess, binning) is still running on another stream.  Each request's
// push kernel (queued after its binning) stores the request's arguments,
// appends one item per active tile and publishes them by moving the tail; the
// last push of a batch also closes the queue.  The consumer's blocks take
// tickets from the head, wait for the ticket's item, render the tile and
// count it in the request's done counter; a request whose done count falls
// short of its tiles is rendered again by the caller.  The consumer launch is
// switched off (hp_render_fwd_persistent returns HP_ERR_UNSUPPORTED): its
// launches did not end on the hardware and the cause is not known.
// ---------------------------------------------------------------------------
// the counters that every block touches sit in cache lines of their own
struct QueueHead {
  uint32_t head, pad0[31];
  uint32_t tail, pad1[31];
  uint32_t closed, overflow, pad2[30];
  uint32_t done[HP_MAX_BATCH];
  uint32_t ntiles[HP_MAX_BATCH];
};
struct QueueReq {
  RenderArgs A;
  RenderOut O;
};
struct QueueView {
  QueueHead* h;
  QueueReq* reqs;
  uint32_t* items;
  int64_t cap;
};
static size_t queue_head_bytes() { return hp_align256(sizeof(QueueHead)) + hp_align256(sizeof(QueueReq) * HP_MAX_BATCH); }
static QueueView queue_view(void* q, size_t bytes) {
  QueueView v;
  v.h = (QueueHead*)q;
  v.reqs = (QueueReq*)((char*)q + hp_align256(sizeof(QueueHead)));
  v.items = (uint32_t*)((char*)q + queue_head_bytes());
  v.cap = bytes > queue_head_bytes() ? (int64_t)((bytes - queue_head_bytes()) / 4) : 0;
  return v;
}

__global__ void k_queue_reset(QueueHead* h) {
  uint32_t* w = (uint32_t*)h;
  for (int i = threadIdx.x; i < (int)(sizeof(QueueHead) / 4); i += blockDim.x) w[i] = 0u;
}

// one block: the request's arguments, its items, then the new tail
__global__ __launch_bounds__(256) void k_queue_push(QueueView Q, int slot, RenderArgs A, RenderOut O, int n_tiles,
                                                    int last) {
  const uint32_t t0 = __hip_atomic_fetch_add(&Q.h->tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const bool fits = (int64_t)t0 + n_tiles <= Q.cap;
  if (fits) {
    if (threadIdx.x == 0) {
      Q.reqs[slot].A = A;
      Q.reqs[slot].O = O;
      Q.h->ntiles[slot] = (uint32_t)n_tiles;
    }
    for (int i = threadIdx.x; i < n_tiles; i += blockDim.x) Q.items[t0 + i] = ((uint32_t)slot << 24) | (uint32_t)i;
  }
  // every thread's writes reach device scope before the tail moves
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (fits) __hip_atomic_store(&Q.h->tail, t0 + (uint32_t)n_tiles, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store(&Q.h->overflow, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (last) __hip_atomic_store(&Q.h->closed, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Claim the next item (thread 0 only): a ticket from one atomic add on the
// head, then a wait until the ticket's item is published.  Returns 1 and the
// item; 0 when the queue is closed and holds no item at the ticket, or when
// spin_limit polls (each sleeps about 2000 cycles) pass without it.  A
// ticket abandoned that way leaves its item unrendered, which the request's
// done counter shows to the caller.  The counters are read with atomic
// read-modify-writes (an add of 0), performed at the device's coherence
// point, so they see the other XCDs' latest values where a plain load could
// be served stale from this XCD's L2; and no fence is issued per poll (an
// acquire fence would invalidate the whole L2 of the polling block's XCD
// under the render and the binning running beside it).
__device__ __forceinline__ uint32_t q_peek(uint32_t* p) {
  return __hip_atomic_fetch_add(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int queue_claim(const QueueView& Q, int spin_limit, uint32_t* item) {
  const uint32_t idx = __hip_atomic_fetch_add(&Q.h->head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int spins = 0; spins <= spin_limit; ++spins) {
    if (idx < q_peek(&Q.h->tail)) {
      *item = q_peek(&Q.items[idx]);
      return 1;
    }
    // the tail is final once closed: the flag is read before a second look
    if (q_peek(&Q.h->closed) && idx >= q_peek(&Q.h->tail)) return 0;
    __builtin_amdgcn_s_sleep(32);
  }
  return 0;
}

__global__ __launch_bounds__(256) void k_render_fwd_persistent(QueueView Q, int spin_limit) {
  __shared__ float4 s_rec[2 * HP_STAGE];
  __shared__ uint32_t s_item;
  __shared__ int s_ok;
  __shared__ uint32_t s_req[(sizeof(QueueReq) + 3) / 4];
  constexpr int kReqWords = (int)((sizeof(QueueReq) + 3) / 4);
  while (true) {
    if (threadIdx.x == 0) {
      uint32_t it = 0;
      s_ok = queue_claim(Q, spin_limit, &it);
      s_item = it;
    }
    __syncthreads();
    if (!s_ok) break;
    const uint32_t it = s_item;
    const int slot = (int)(it >> 24);
    const int ct = (int)(it & 0xFFFFFFu);
    // the request's arguments, read coherently (written by its push kernel,
    // possibly on another XCD, after this launch began)
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&Q.reqs[slot]);
    for (int w = threadIdx.x; w < kReqWords; w += blockDim.x) s_req[w] = q_peek(const_cast<uint32_t*>(src + w));
    __syncthreads();
    const QueueReq* rq = reinterpret_cast<const QueueReq*>(s_req);
    const RenderArgs A = rq->A;
    const RenderOut O = rq->O;
    render_fwd_tile<false>(A, O, ct, s_rec, nullptr);
    __syncthreads();  // s_item and s_req may be reused
    // the outputs are read after the launch ends: the count needs no fence
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&Q.h->done[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

constexpr bool kPersistentEnabled = false;

extern "C" size_t hp_render_queue_bytes(int64_t max_items) {
  return max_items < 0 ? 0 : queue_head_bytes() + hp_align256((size_t)max_items * 4);
}

extern "C" hp_status hp_render_queue_reset(void* queue, size_t queue_bytes, void* stream) {
  if (!queue || queue_bytes < queue_head_bytes()) return HP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, (hipStream_t)stream, (QueueHead*)queue);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_render_queue_push(void* queue, size_t queue_bytes, int32_t slot, const hp_render_req* req,
                                          const hp_params* prm, int32_t last, void* stream) {
  if (!queue || !req || slot < 0 || slot >= HP_MAX_BATCH || queue_bytes < queue_head_bytes()) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_params(prm));
  const hp_render_req& q = *req;
  if (q.order < 0 || q.order > HP_MAX_ORDER || q.P < 0 || q.n_tiles < 0 || q.n_active < 0 || !q.projected || !q.mask)
    return HP_ERR_INVALID_ARG;
  if (q.n_tiles > 0 && (!q.tile_ranges || !q.vals || !q.rgb || !q.T || !q.n_contrib)) return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(q.order, prm->tile_log2);
  if (q.n_tiles > g.ntile || q.n_active > g.npix || q.n_tiles >= (1 << 24)) return HP_ERR_INVALID_ARG;
  const RenderArgs A = make_args(g, hp_mask_view((const char*)q.mask, g), hp_proj_view((const char*)q.projected, q.P),
                                 q.vals, q.tile_ranges, prm, q.n_active);
  const RenderOut O{q.rgb, q.T, q.n_contrib, nullptr, nullptr};
  hipLaunchKernelGGL(k_queue_push, dim3(1), dim3(256), 0, (hipStream_t)stream, queue_view(queue, queue_bytes), (int)slot,
                     A, O, (int)q.n_tiles, (int)(last != 0));
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_render_fwd_persistent(void* queue, size_t queue_bytes, int32_t n_blocks, int32_t spin_limit,
                                              void* stream) {
  if (!queue || queue_bytes < queue_head_bytes() || n_blocks < 1 || n_blocks > 65536 || spin_limit < 0)
    return HP_ERR_INVALID_ARG;
  // Switched off: launches of this consumer did not end on MI355X although
  // every item had been published before they started, and no defect that
  // explains it has been found.  Nothing is launched until one is.
  if (!kPersistentEnabled) return HP_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_render_fwd_persistent, dim3((unsigned)n_blocks), dim3(256), 0, (hipStream_t)stream,
                     queue_view(queue, queue_bytes), (int)spin_limit);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_render_queue_status(const void* queue, int32_t n_req, int32_t* done_tiles,
                                            int32_t* overflow, void* stream) {
  if (!queue || n_req < 0 || n_req > HP_MAX_BATCH || (n_req > 0 && !done_tiles)) return HP_ERR_INVALID_ARG;
  QueueHead h;
  HP_TRY(hp_read_small(&h, queue, sizeof(QueueHead), (hipStream_t)stream));
  for (int r = 0; r < n_req; ++r) done_tiles[r] = (int32_t)h.done[r];
  if (overflow) *overflow = (int32_t)h.overflow;
  return HP_OK;
}

// the backward of stage 1 lives with the forward in k_preprocess.hip
hp_status hp_preprocess_bwd_launch(const hp_gaussians* g, const hp_view* view, const hp_params* prm, const float* acc,
                                   hp_gaussians_grad* grad, hipStream_t s);

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

extern "C" size_t hp_render_bwd_workspace_bytes(int64_t P) { return P < 0 ? 0 : hp_align256((size_t)P * HP_NACC * 4); }

extern "C" hp_status hp_render_bwd(const hp_gaussians* gs, const void* projected, const uint32_t* vals,
                                   const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view,
                                   const hp_params* prm, const void* mask, int64_t n_active, const float* T,
                                   const int32_t* n_contrib, const float* dL_drgb, const float* dL_dT,
                                   const float* dL_dinv_depth, hp_gaussians_grad* grad, void* ws, size_t ws_bytes,
                                   void* stream) {
  HP_TRY(hp_check_gaussians(gs));
  HP_TRY(hp_check_view(view, prm));
  if (!projected || !mask || !grad || n_tiles < 0 || n_active < 0) return HP_ERR_INVALID_ARG;
  if (gs->P > 0 && (!grad->mean || !grad->scale || !grad->rot || !grad->opacity || !grad->sh || !ws))
    return HP_ERR_INVALID_ARG;
  if (n_active > 0 && n_tiles > 0 && (!T || !n_contrib || !dL_drgb || !tile_ranges || !vals)) return HP_ERR_INVALID_ARG;
  if (ws_bytes < hp_render_bwd_workspace_bytes(gs->P)) return HP_ERR_CAPACITY;
  return hp_render_bwd_acc(gs, projected, vals, tile_ranges, n_tiles, view, prm, mask, n_active, T, n_contrib,
                           dL_drgb, dL_dT, dL_dinv_depth, grad, (float*)ws, stream);
}

// hp_render_bwd after its argument checks, with the accumulators [HP_NACC][P]
// at `acc` (zeroed here by a kernel)
hp_status hp_render_bwd_acc(const hp_gaussians* gs, const void* projected, const uint32_t* vals,
                            const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view, const hp_params* prm,
                            const void* mask, int64_t n_active, const float* T, const int32_t* n_contrib,
                            const float* dL_drgb, const float* dL_dT, const float* dL_dinv_depth,
                            hp_gaussians_grad* grad, float* acc, void* stream) {
  if (gs->P == 0) return HP_OK;
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_tiles > g.ntile || n_active > g.npix) return HP_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f32, dim3(hp_blocks(gs->P * HP_NACC, 256)), dim3(256), 0, s, acc, gs->P * HP_NACC);
  HP_CHECK_LAUNCH();
  HP_TRY(hp_render_bwd_pixels(projected, gs->P, vals, tile_ranges, n_tiles, view, prm, mask, n_active, T, n_contrib,
                              dL_drgb, dL_dT, dL_dinv_depth, acc, stream));
  return hp_preprocess_bwd_launch(gs, view, prm, acc, grad, s);
}

extern "C" hp_status hp_render_bwd_pixels(const void* projected, int64_t P, const uint32_t* vals,
                                          const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view,
                                          const hp_params* prm, const void* mask, int64_t n_active, const float* T,
                                          const int32_t* n_contrib, const float* dL_drgb, const float* dL_dT,
                                          const float* dL_dinv_depth, float* acc, void* stream) {
  HP_TRY(hp_check_view(view, prm));
  if (P < 0 || !projected || !mask || n_tiles < 0 || n_active < 0) return HP_ERR_INVALID_ARG;
  if (P > 0 && !acc) return HP_ERR_INVALID_ARG;
  if (n_active > 0 && n_tiles > 0 && (!T || !n_contrib || !dL_drgb || !tile_ranges || !vals)) return HP_ERR_INVALID_ARG;
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_tiles > g.ntile || n_active > g.npix) return HP_ERR_INVALID_ARG;
  if (P == 0 || n_tiles == 0 || n_active == 0) return HP_OK;
  RenderArgs A = make_args(g, hp_mask_view((const char*)mask, g), hp_proj_view((const char*)projected, P), vals,
                           tile_ranges, prm, n_active);
  if (dL_dinv_depth)
    hipLaunchKernelGGL(k_render_bwd<true>, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, A, P, T,
                       n_contrib, dL_drgb, dL_dT, dL_dinv_depth, acc);
  else
    hipLaunchKernelGGL(k_render_bwd<false>, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, A, P, T,
                       n_contrib, dL_drgb, dL_dT, (const float*)nullptr, acc);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_preprocess_bwd(const hp_gaussians* gs, const hp_view* view, const hp_params* prm,
                                       const float* acc, hp_gaussians_grad* grad, void* stream) {
  HP_TRY(hp_check_gaussians(gs));
  HP_TRY(hp_check_view(view, prm));
  if (!grad) return HP_ERR_INVALID_ARG;
  if (gs->P == 0) return HP_OK;
  if (!acc || !grad->mean || !grad->scale || !grad->rot || !grad->opacity || !grad->sh) return HP_ERR_INVALID_ARG;
  return hp_preprocess_bwd_launch(gs, view, prm, acc, grad, (hipStream_t)stream);
}

// ---- radian-space statistics for adaptive density control -------------------
// one block per active tile: every Gaussian of the tile's list [start, end)
__global__ void k_mark_visible(const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges, int64_t P,
                               uint8_t* __restrict__ vis) {
  const uint32_t s = ranges[2 * (int64_t)blockIdx.x], e = ranges[2 * (int64_t)blockIdx.x + 1];
  for (uint32_t k = s + threadIdx.x; k < e; k += blockDim.x) {
    const uint32_t g = vals[k];
    if ((int64_t)g < P) vis[g] = 1;
  }
}

// r_s,max and the norm of the gradient with respect to the centre's
// displacement along the sphere: east = d omega cos(phi), north = d phi, so
// dL/d east = (dL/d omega) / cos(phi); cos(phi) is e_phi.y, record word 7
__global__ void k_density_stats(HpProjView pv, int64_t P, const float* __restrict__ acc,
                                const uint8_t* __restrict__ vis, float* __restrict__ rs_max,
                                float* __restrict__ gacc, int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P || !vis[i]) return;
  const float rs = pv.radius[i];
  if (!(rs > 0.f)) return;
  rs_max[i] = fmaxf(rs_max[i], rs);
  const float cph = pv.rec[4 * i + 1].w;
  const float ge = acc[7 * P + i] / cph, gn = acc[8 * P + i];
  gacc[i] += sqrtf(ge * ge + gn * gn);
  cnt[i] += 1;
}

extern "C" hp_status hp_mark_visible(const uint32_t* vals, const uint32_t* tile_ranges, int32_t n_tiles, int64_t P,
                                     uint8_t* visible, void* stream) {
  if (n_tiles < 0 || P < 0 || (n_tiles > 0 && (!vals || !tile_ranges)) || (P > 0 && !visible))
    return HP_ERR_INVALID_ARG;
  if (n_tiles == 0) return HP_OK;
  hipLaunchKernelGGL(k_mark_visible, dim3((unsigned)n_tiles), dim3(256), 0, (hipStream_t)stream, vals, tile_ranges, P,
                     visible);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_density_stats(const void* projected, int64_t P, const float* acc, const uint8_t* visible,
                                      float* rs_max, float* grad_accum, int32_t* count, void* stream) {
  if (P < 0) return HP_ERR_INVALID_ARG;
  if (P == 0) return HP_OK;
  if (!projected || !acc || !visible || !rs_max || !grad_accum || !count) return HP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_density_stats, dim3(hp_blocks(P, 256)), dim3(256), 0, (hipStream_t)stream,
                     hp_proj_view((const char*)projected, P), P, acc, visible, rs_max, grad_accum, count);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
