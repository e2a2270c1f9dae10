/*
 * hp.h -- C ABI of the HEALPix Gaussian rasterizer for AMD Instinct MI355X
 * (gfx950).  Every operation runs in hand-written HIP kernels; this header
 * only uses plain C types.
 *
 * Conventions (all calls):
 *  - Device pointers point to device (HBM) memory owned by the caller.  The
 *    library never allocates or frees memory; scratch space comes from a
 *    caller buffer whose size the matching _bytes / _workspace_bytes
 *    function returns.  Buffers must be 256-byte aligned (hipMalloc and
 *    torch allocations are).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call only enqueues work and returns without waiting, except the
 *    read-back helpers hp_mask_counts, hp_read_total and hp_check_count,
 *    which wait for the stream.  Counts that size later work (tasks, pairs)
 *    stay in device memory; a count that exceeds a caller's capacity makes
 *    the calls that depend on it write nothing (and leave every tile range
 *    empty), and the caller learns it from the device count itself.
 *  - Arrays are float32 structure-of-arrays [component][count].
 *  - Argument checks happen on the host before anything is enqueued and
 *    return HP_ERR_INVALID_ARG / HP_ERR_UNSUPPORTED without side effects.
 *    A failed launch returns HP_ERR_DEVICE.  Calls keep no global state and
 *    may run concurrently on different streams with different buffers.
 *
 * The method is the camera-agnostic 3D Gaussian rasterizer on the HEALPix
 * equal-area sphere grid of arXiv 2606.29794 ("UniTriSplat"): Sec. 3.1
 * (grid, NESTED (x, y, f) indexing, tiles of B x B samples, visibility
 * mask), Sec. 3.2 (projection Pi, Eq. lonlat_projection; latitude scaling,
 * Eq. arc_scaling; gradients, Eqs. backward_lat_scale and grad_via_J_S),
 * Sec. 3.3 (tile query), Sec. 3.4 (spherical offset, Eq.
 * unified_rendering), Sec. 4.1 (HEALPix-SSIM and the training loss) and
 * supplementary Alg. 1 (the three-stage pipeline).
 */
#ifndef HP_H
#define HP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hp_status;
#define HP_OK 0
#define HP_ERR_INVALID_ARG 1 /* null pointer, bad size, order/degree out of range */
#define HP_ERR_UNSUPPORTED 2 /* valid request this build does not handle */
#define HP_ERR_CAPACITY 3    /* caller buffer too small (see the call) */
#define HP_ERR_DEVICE 4      /* HIP launch/runtime error */

#define HP_CAM_FULL 0    /* full sphere (omnidirectional / equirectangular) */
#define HP_CAM_FISHEYE 1 /* anisotropic equidistant fisheye, FoV (fov_x, fov_y) */
#define HP_CAM_PINHOLE 2 /* perspective, half-FoVs fov_x/2, fov_y/2 */

#define HP_MAX_ORDER 12  /* Nside up to 4096 */
#define HP_MAX_SH_DEGREE 3

/* Constants of the method.  Defaults (hp_default_params):
 *   eps_T = 1e-4     early termination once T < eps_T (Alg. 1 rendering loop)
 *   alpha_max = 0.99 opacity clamp
 *   q_cut = 9        a Gaussian reaches a pixel only where d^T Sigma^-1 d <= 9
 *   r_min = 0.1      Gaussians with radial depth below r_min are culled
 *   rs_sigma = 3     bounding radius r_s = 3 sqrt(lambda_max(Sigma_arc)) (Sec. 3.2)
 *   bin_guard = 1e-6 radians added to the tile-overlap test
 *   sh_offset = 0.5  colour = max(0, sh_offset + sum_lm sh_lm Y_lm(view dir))
 *   tile_log2 = 4    tiles of B x B = 16 x 16 samples (Table tab:resolution);
 *                    below order 4 the tile is the whole face (B = Nside). */
typedef struct {
  float eps_T, alpha_max, q_cut, r_min, rs_sigma, bin_guard, sh_offset;
  int32_t tile_log2;
} hp_params;

/* One camera.  W: world->camera rotation, row-major; b = -W * center; the
 * HEALPix grid is fixed in the camera frame with its pole on camera +y and
 * longitude omega = atan2(t_x, t_z) (Eq. lonlat_projection).  order k gives
 * Nside = 2^k, Npix = 12 * 4^k.  fov_x/fov_y in radians (ignored for FULL). */
typedef struct {
  float W[9], b[3], center[3];
  int32_t cam_type;
  float fov_x, fov_y;
  int32_t order;
} hp_view;

/* Gaussians (Alg. 1 input {(mu, s, q, o, c)}), device pointers:
 *   mean [3][P], scale [3][P] (> 0, already exponentiated),
 *   rot [4][P] quaternion (w, x, y, z), normalised inside the library,
 *   opacity [P] in (0, 1) (already through the sigmoid),
 *   sh [(d+1)^2][3][P] real SH coefficients, d = sh_degree in 0..3. */
typedef struct {
  int64_t P;
  int32_t sh_degree;
  const float *mean, *scale, *rot, *opacity, *sh;
} hp_gaussians;

/* Gradients, same shapes as hp_gaussians; ACCUMULATED into (+=). */
typedef struct {
  float *mean, *scale, *rot, *opacity, *sh;
} hp_gaussians_grad;

/* HEALPix-SSIM constants (Sec. 4.1; window of Wang et al. 2004):
 * 11 x 11 window on face-local (x, y), Gaussian sigma, C1 = (0.01)^2,
 * C2 = (0.03)^2, loss weight lambda = 0.2.  zones = 1 selects the
 * zone-specific windows of Sec. 4.1: pixels of the equatorial belt (|z| <=
 * 2/3) keep the isotropic window exp(-(a^2 + b^2) / (2 sigma^2)) of chart
 * offsets (a, b); pixels of the polar caps weigh each chart neighbour by its
 * great-circle distance d, exp(-d^2 / (2 sigma^2 Omega)) with Omega = 4 pi /
 * Npix, i.e. the same Gaussian measured on the sphere (anisotropic in the
 * chart, where the rings compress the pixels).  zones = 0 (default): the
 * isotropic chart window everywhere. */
typedef struct {
  float sigma, C1, C2, lambda;
  int32_t zones;
} hp_ssim_params;

void hp_default_params(hp_params* p);
void hp_default_ssim_params(hp_ssim_params* p);
const char* hp_status_string(hp_status s);

/* ---- grid ------------------------------------------------------------
 * hp_grid_init: geometry tables of one HEALPix order, independent of any
 * camera (the grid is camera-fixed): for every node of the NESTED quadtree
 * from the 12 base faces (level 0) down to the tiles (level k_t = k - b,
 * b = min(tile_log2, k)), a bounding cap (unit centre, angular radius).  A
 * tile's cap is centred on the normalised sum of its B x B pixel-centre
 * directions with radius the largest angle to them; a parent's cap contains
 * its children's caps.  Computed in FP64 on the device, stored as float.
 * grid: device buffer of hp_grid_bytes(order, tile_log2) bytes. */
size_t hp_grid_bytes(int32_t order, int32_t tile_log2);
hp_status hp_grid_init(int32_t order, const hp_params* prm, void* grid, size_t grid_bytes, void* stream);

/* ---- visibility mask (Sec. 3.1: M_C(p) = 1[(omega_p, phi_p) in R_C]) ----
 * Marks the pixels whose centre lies in the camera's field of view, decided
 * in FP64 on pixel-centre directions:
 *   FULL: all;  FISHEYE: incident angle psi <= (pi/2) w_eff(gamma) with
 *   w_eff = sqrt((w_x cos gamma)^2 + (w_y sin gamma)^2), w = FoV/pi (supp.
 *   anisotropic equidistant model);  PINHOLE: t_z > 0, |t_x| <= tan(fov_x/2) t_z,
 *   |t_y| <= tan(fov_y/2) t_z.
 * The mask depends only on (order, cam_type, fov_x, fov_y), not on the pose.
 * mask: device buffer of hp_mask_bytes(order, tile_log2) bytes receiving:
 *   the sorted list of active NESTED pixels (int32), per tile the offset of
 *   its first active pixel in that list, its active count and 256-bit
 *   membership, the compact index of every active tile, and per quadtree node
 *   whether any active pixel lies below it.
 * hp_mask_counts waits for `stream` and returns n_active (active pixels) and
 * n_tiles (active tiles); outputs of the other calls are indexed by these.
 * hp_mask_active_pix returns the device pointer to the int32 active pixel
 * list inside `mask`. */
size_t hp_mask_bytes(int32_t order, int32_t tile_log2);
hp_status hp_mask(const hp_view* view, const hp_params* prm, const void* grid, void* mask, size_t mask_bytes,
                  void* stream);
hp_status hp_mask_counts(const void* mask, int32_t order, int32_t tile_log2, int64_t* n_active,
                         int32_t* n_tiles, void* stream);
const int32_t* hp_mask_active_pix(const void* mask, int32_t order, int32_t tile_log2);

/* ---- stage 1: preprocessing (Alg. 1; Eqs. lonlat_projection, arc_scaling) --
 * Per Gaussian: t = W mu + b, r = |t|, (omega, phi) = Pi(t);
 * Sigma_3D = R diag(s^2) R^T; Sigma_arc = S_phi J W Sigma_3D W^T J^T S_phi
 * with S_phi = diag(cos phi, 1), evaluated as (1/r^2) E W Sigma_3D W^T E^T where
 * E = [e_omega; e_phi] is the unit tangent frame (the same matrix: S_phi J =
 * E / r); conic = Sigma_arc^-1; r_s = min(pi, 3 sqrt(lambda_max)); colour
 * from SH at the world direction normalise(mu - center).  Culled (r < r_min
 * or det Sigma_arc <= 0) Gaussians get radius 0 and depth +inf.
 * projected: device buffer of hp_projected_bytes(P) bytes: a 64-byte record
 * per Gaussian (unit direction, opacity, tangent frame, conic, colour) plus
 * depth [P] and radius [P] float arrays and a disc [P] float4 array (unit
 * direction, sin((r_s + bin_guard) / 2): the part the binning reads). */
size_t hp_projected_bytes(int64_t P);
hp_status hp_preprocess(const hp_gaussians* g, const hp_view* view, const hp_params* prm, void* projected,
                        size_t projected_bytes, void* stream);
const float* hp_projected_depth(const void* projected, int64_t P);
/* Serving form of hp_preprocess: n_views (1..8) cameras in one launch that
 * reads every Gaussian once; projected[v] (host array of device pointers,
 * each of hp_projected_bytes(P) bytes) receives view v. */
hp_status hp_preprocess_batch(const hp_gaussians* g, int32_t n_views, const hp_view* views, const hp_params* prm,
                              void* const* projected, size_t projected_bytes, void* stream);
const float* hp_projected_radius(const void* projected, int64_t P);

/* ---- stage 2a: tile assignment (Alg. 1 QueryDisc + pair emission) --------
 * T_i = { active tiles t : angle(cap centre_t, dir_i) <= r_s,i + R_t + bin_guard }
 * (the tile's bounding cap against the Gaussian's r_s disc), found by a
 * pruned traversal of the NESTED quadtree: each Gaussian walks the tree down
 * to three levels above the tiles and every passing node there becomes a task
 * whose subtree (at most 64 tiles) is walked separately, so no walk is long.
 * Pairs (key = compact active tile index, val = Gaussian index) are emitted
 * in order of increasing radial depth (ties by index), so a stable sort on the
 * tile key alone yields the per-tile front-to-back order of Alg. 1.
 * phase: HP_BIN_COUNT counts pairs (writes *n_pairs, device int64),
 *        HP_BIN_EMIT writes them (needs a previous COUNT on the same ws),
 *        HP_BIN_ALL does both.  Nothing waits for the host: if *n_pairs >
 *        capacity when EMIT runs, EMIT writes nothing; the caller reads
 *        *n_pairs (hp_read_total / hp_check_count) and calls EMIT again with
 *        larger buffers.  If the tasks exceed the workspace (16 P + 2^20 of
 *        them), *n_pairs is set to INT64_MAX, which no capacity admits.
 * keys/vals: device uint32 [capacity]; ws: hp_bin_workspace_bytes(P). */
#define HP_BIN_COUNT 1
#define HP_BIN_EMIT 2
#define HP_BIN_ALL 3
size_t hp_bin_workspace_bytes(int64_t P);
hp_status hp_bin(int32_t phase, const void* projected, int64_t P, const hp_view* view, const hp_params* prm,
                 const void* grid, const void* mask, uint32_t* keys, uint32_t* vals, int64_t capacity,
                 int64_t* n_pairs, void* ws, size_t ws_bytes, void* stream);
/* hp_bin_sorted: the same tile sets, emitted directly in the per-tile
 * front-to-back order that hp_bin + hp_sort produce (Alg. 1 stage 2 as one
 * step), without a sort of the pairs.  The tasks are sorted by their node
 * (stable, so each node keeps depth order); every node's tasks are cut into
 * chunks of 64; per chunk and tile the hits are counted, the counts are
 * scanned in (tile, chunk) order and each hit is written at its slot.
 * phase as for hp_bin (COUNT writes *n_pairs; EMIT fills vals [capacity] with
 * Gaussian ids grouped by tile and tile_ranges [n_tiles][2] with each active
 * tile's (start, end) in vals, n_tiles from hp_mask_counts).  No phase waits
 * for the host: the task and chunk counts that size the steps are read on
 * the device.  If *n_pairs > capacity (or is INT64_MAX: the tasks exceeded
 * the workspace, or the COUNT before did not complete), EMIT writes no pair
 * and sets every tile range to (0, 0), so a render over the result reads no
 * list entry.  A typical caller passes HP_BIN_ALL with a capacity from an
 * earlier view and checks *n_pairs afterwards (hp_check_count).
 * ws: hp_bin_sorted_workspace_bytes(P, order, tile_log2) bytes. */
size_t hp_bin_sorted_workspace_bytes(int64_t P, int32_t order, int32_t tile_log2);
hp_status hp_bin_sorted(int32_t phase, const void* projected, int64_t P, const hp_view* view, const hp_params* prm,
                        const void* grid, const void* mask, uint32_t* vals, uint32_t* tile_ranges, int32_t n_tiles,
                        int64_t capacity, int64_t* n_pairs, void* ws, size_t ws_bytes, void* stream);
/* hp_bin_query: tile lists from the paper's own queries (Sec. 3.3 and its
 * supplementary stage-2 description), which decide on centres at the query
 * order kq = kt + log2 f ("x f" search depth of the ablation, f = 1 .. B):
 *  HP_QUERY_RING   (Alg. 3): tile t holds Gaussian i when a pixel of order kq
 *    in t lies on a ring whose centre latitude is within r_s of the disc's
 *    and at a position between floor and ceil of the ring's window of
 *    Eq. ring_phi_range (all of the ring when the ring lies inside the disc);
 *  HP_QUERY_NESTED (Alg. 2): tile t holds i when a node of order kt .. kq in
 *    t has its centre within r_s (the DFS from the 12 base pixels with
 *    PixRad bounding the distance from a node centre to its descendants'
 *    centres at order kq).
 * These sets can leave out tiles that the Gaussian reaches (unlike
 * hp_bin_sorted's), so the image can differ from the exact one.  Lists are in
 * the same per-tile front-to-back order as hp_bin_sorted's.
 * Arguments as for hp_bin_sorted, plus mode, f (a power of two, at most the
 * tile side B) and n_kept (device int64, nullable).  COUNT writes *n_pairs,
 * the number of candidates (the capacity EMIT needs: hp_bin_sorted's pairs
 * with the test angle widened to contain the query's set).  EMIT writes the
 * candidates and filters every tile's list in place: tile_ranges[k] =
 * (start, start + kept), entries past a tile's end are stale, *n_kept = the
 * total kept.  HP_ERR_INVALID_ARG for an unknown mode or f.
 * ws: hp_bin_query_workspace_bytes(P, order, tile_log2) bytes. */
#define HP_QUERY_RING 1
#define HP_QUERY_NESTED 2
size_t hp_bin_query_workspace_bytes(int64_t P, int32_t order, int32_t tile_log2);
hp_status hp_bin_query(int32_t phase, int32_t mode, int32_t f, const void* projected, int64_t P, const hp_view* view,
                       const hp_params* prm, const void* grid, const void* mask, uint32_t* vals, uint32_t* tile_ranges,
                       int32_t n_tiles, int64_t capacity, int64_t* n_pairs, int64_t* n_kept, void* ws,
                       size_t ws_bytes, void* stream);
/* Waits for `stream` and copies one device int64 to the host. */
hp_status hp_read_total(const int64_t* dev_value, int64_t* host_value, void* stream);
/* Synchronous form of the capacity check of an asynchronous count (the
 * pairs of hp_bin / hp_bin_sorted / hp_bin_query): waits for `stream`,
 * copies *dev_count to *host_count (nullable) and returns HP_ERR_CAPACITY
 * when it is negative or exceeds `capacity` (the emission then wrote
 * nothing), HP_OK otherwise. */
hp_status hp_check_count(const int64_t* dev_count, int64_t capacity, int64_t* host_count, void* stream);

/* ---- stage 2b: sort + tile ranges (Alg. 1: sort by tile then depth,
 * identify [start_t, end_t)) -------------------------------------------------
 * Stable LSD radix sort of the first *n_pairs (keys, vals) pairs on the tile
 * key; n_pairs is a device int64 (as hp_bin writes it), read on the device,
 * so the call does not wait for the binning.  The sorted values are written
 * back to vals (keys too).  tile_ranges [n_tiles][2] receives (start, end)
 * of each active tile's list in vals.  If *n_pairs exceeds capacity (the
 * size of keys and vals) nothing is sorted and every range is (0, 0).
 * ws: hp_sort_workspace_bytes(capacity, n_tiles). */
size_t hp_sort_workspace_bytes(int64_t capacity, int32_t n_tiles);
hp_status hp_sort(uint32_t* keys, uint32_t* vals, const int64_t* n_pairs, int64_t capacity, int32_t n_tiles,
                  uint32_t* tile_ranges, void* ws, size_t ws_bytes, void* stream);

/* ---- stage 3: rendering (Eq. unified_rendering; Alg. 1 rendering loop) ----
 * For each active pixel p, in its tile's list order: d = spherical offset of
 * p from the Gaussian centre (great-circle distance along the bearing, Sec.
 * 3.4), q = d^T conic d; where q <= q_cut: alpha = min(alpha_max, o e^{-q/2}),
 * C += T alpha c, T *= 1 - alpha, stop once T < eps_T.
 * Outputs over the n_active active pixels (mask order): rgb [3][n_active],
 * T [n_active] (final transmittance; background is left to the caller),
 * n_contrib [n_active] (list entries consumed, skipped ones included),
 * n_used [n_active] (nullable: Gaussians actually composited), and
 * inv_depth [n_active] (nullable: the inverse radial depth 1/r composited
 * like a colour, sum_i T_i alpha_i / r_i, for depth supervision, Sec. 3.2). */
hp_status hp_render_fwd(const void* projected, int64_t P, const uint32_t* vals, const uint32_t* tile_ranges,
                        int32_t n_tiles, const hp_view* view, const hp_params* prm, const void* mask, int64_t n_active,
                        float* rgb, float* T, int32_t* n_contrib, int32_t* n_used, float* inv_depth, void* stream);

/* Serving form of hp_render_fwd: up to 16 independent renders (different
 * cameras, orders and scenes) in ONE launch whose workgroups cover the union
 * of their active tiles; every output equals that of hp_render_fwd on the same
 * request alone (bit for bit: no atomics in the forward). */
typedef struct {
  const void* projected;
  int64_t P;
  const uint32_t* vals;
  const uint32_t* tile_ranges;
  int32_t n_tiles;
  int32_t order;
  const void* mask;
  int64_t n_active;
  float* rgb;
  float* T;
  int32_t* n_contrib;
} hp_render_req;
hp_status hp_render_fwd_batch(int32_t n_req, const hp_render_req* reqs, const hp_params* prm, void* stream);

/* Persistent form of the serving render: a device queue of (request, tile)
 * items that one long-running launch drains while the requests' preparation
 * (preprocess, binning) still runs on another stream.
 *  hp_render_queue_bytes: size of a queue holding max_items items (and the
 *    arguments of up to 16 requests); the buffer is device memory owned by
 *    the caller.
 *  hp_render_queue_reset: empties the queue (a kernel; no host wait).
 *  hp_render_queue_push: queues a kernel that stores request `slot`'s
 *    arguments (0 <= slot < 16, distinct within one batch), appends one item
 *    per active tile of it and publishes them; with last != 0 it also closes
 *    the queue (no further pushes until the next reset).  Queue it on the
 *    stream of the request's binning, after it.  Items beyond the queue's
 *    capacity are not appended and set an overflow flag.
 *  hp_render_fwd_persistent: the consumer, n_blocks workgroups that claim
 *    published items, render each tile as hp_render_fwd does and count it
 *    in its request's done counter; a workgroup leaves when the queue is
 *    closed and drained, or after spin_limit empty polls.  DISABLED: it
 *    checks its arguments and returns HP_ERR_UNSUPPORTED without launching
 *    anything.  Launches of this consumer did not complete on MI355X (the
 *    host wait after them never returned, with every item already
 *    published before the launch), and no defect that explains it has been
 *    found in the code; until one is, the kernel is built but not run.
 *    Callers render a batch with hp_render_fwd_batch instead.
 *  hp_render_queue_status: waits for `stream` and reads the done counters of
 *    the first n_req requests and the overflow flag; a request whose count
 *    is below its tile count was not finished (the launch ran out of polls
 *    before its items appeared) and must be rendered again. */
size_t hp_render_queue_bytes(int64_t max_items);
hp_status hp_render_queue_reset(void* queue, size_t queue_bytes, void* stream);
hp_status hp_render_queue_push(void* queue, size_t queue_bytes, int32_t slot, const hp_render_req* req,
                               const hp_params* prm, int32_t last, void* stream);
hp_status hp_render_fwd_persistent(void* queue, size_t queue_bytes, int32_t n_blocks, int32_t spin_limit,
                                   void* stream);
hp_status hp_render_queue_status(const void* queue, int32_t n_req, int32_t* done_tiles, int32_t* overflow,
                                 void* stream);

/* ---- backward (Sec. 3.2 Eqs. backward_lat_scale, grad_via_J_S) ------------
 * Reverse traversal per pixel from n_contrib with T recomputed as
 * T_j = T_{j+1} / (1 - alpha_j) (no per-Gaussian forward state), gradients
 * of alpha through q to the conic and the Gaussian direction, then per
 * Gaussian through Sigma_arc, S_phi, J, W to scale and rotation and through
 * t = W mu + b and the SH view direction to the mean; SH coefficients and
 * opacities directly.  dL_drgb [3][n_active], dL_dT [n_active] (nullable),
 * dL_dinv_depth [n_active] (nullable: upstream gradient of hp_render_fwd's
 * inv_depth; it reaches the means also through d(1/r)/dt = -t / r^3).
 * Gradients are accumulated into `grad`.  ws: hp_render_bwd_workspace_bytes(P). */
size_t hp_render_bwd_workspace_bytes(int64_t P);
hp_status hp_render_bwd(const hp_gaussians* g, const void* projected, const uint32_t* vals,
                        const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view, const hp_params* prm,
                        const void* mask, int64_t n_active, const float* T, const int32_t* n_contrib,
                        const float* dL_drgb, const float* dL_dT, const float* dL_dinv_depth, hp_gaussians_grad* grad,
                        void* ws, size_t ws_bytes, void* stream);
/* The two halves of hp_render_bwd (which zeroes its workspace, then runs
 * both).  hp_render_bwd_pixels is the pixel pass: per Gaussian, dL with
 * respect to its colour (3), opacity (1), conic (A, B, C) and the longitude
 * and latitude of its centre (omega, phi), and (only when dL_dinv_depth is
 * given) its inverse radial depth 1/r, ACCUMULATED into acc [10][P] (float,
 * device, laid out value-major: acc[m * P + i]; row 9 is left untouched
 * without a depth gradient, so the caller zeroes it).  It needs no Gaussian
 * parameters, only the projected records.  hp_preprocess_bwd
 * carries such accumulators back through Sec. 3.2's chain (conic -> Sigma_arc
 * -> scale, rotation and centre; colour -> SH and view direction) into
 * `grad` (accumulated).  Errors as hp_render_bwd. */
hp_status hp_render_bwd_pixels(const void* projected, int64_t P, const uint32_t* vals, const uint32_t* tile_ranges,
                               int32_t n_tiles, const hp_view* view, const hp_params* prm, const void* mask,
                               int64_t n_active, const float* T, const int32_t* n_contrib, const float* dL_drgb,
                               const float* dL_dT, const float* dL_dinv_depth, float* acc, void* stream);
hp_status hp_preprocess_bwd(const hp_gaussians* g, const hp_view* view, const hp_params* prm, const float* acc,
                            hp_gaussians_grad* grad, void* stream);

/* hp_render_bwd_noalloc: hp_render_bwd for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same arguments without ws / ws_bytes and the
 * same kernels; the per-Gaussian accumulators live in a fixed array of the
 * library on each device (10 * HP_NOALLOC_MAX_P floats = 40 MiB, held until
 * the process ends).  No memory is allocated by the call.  P above
 * HP_NOALLOC_MAX_P returns HP_ERR_CAPACITY.  Every call on a device shares
 * that device's array and leaves it holding its accumulators (the next call
 * clears what it uses first): calls that overlap on one device, on different
 * streams or from different threads, race and must be ordered by the caller.
 * `stream` must belong to the current device. */
#define HP_NOALLOC_MAX_P (1 << 20)
hp_status hp_render_bwd_noalloc(const hp_gaussians* g, const void* projected, const uint32_t* vals,
                                const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view,
                                const hp_params* prm, const void* mask, int64_t n_active, const float* T,
                                const int32_t* n_contrib, const float* dL_drgb, const float* dL_dT,
                                const float* dL_dinv_depth, hp_gaussians_grad* grad, void* stream);

/* ---- radian-space statistics for adaptive density control -----------------
 * (Sec. 4.2: r_s,max tracked across iterations, thresholds in radians.)
 * hp_mark_visible sets visible[i] = 1 for every Gaussian id in the view's
 * tile lists (vals[start, end) of every tile_ranges entry, n_tiles of them;
 * visible [P] uint8 is zeroed by the caller).  hp_density_stats then, for every Gaussian with visible[i],
 * sets rs_max[i] = max(rs_max[i], r_s,i), adds to grad_accum[i] the norm of
 * the loss gradient with respect to a displacement of its centre along the
 * sphere, |(dL/domega / cos phi, dL/dphi)| (rows 7 and 8 of the pixel pass's
 * acc [10][P], cos phi from the projected record), and increments count[i].
 * rs_max, grad_accum [P] float and count [P] int32 are device arrays owned by
 * the caller and updated in place. */
hp_status hp_mark_visible(const uint32_t* vals, const uint32_t* tile_ranges, int32_t n_tiles, int64_t P,
                          uint8_t* visible, void* stream);
hp_status hp_density_stats(const void* projected, int64_t P, const float* acc, const uint8_t* visible, float* rs_max,
                           float* grad_accum, int32_t* count, void* stream);

/* ---- HEALPix-SSIM and the training loss (Sec. 4.1) ------------------------
 * Per active pixel and channel, Gaussian-weighted 11x11 statistics over
 * face-local (x, y) offsets, neighbours across face edges taken in the
 * neighbouring face with its axes rotated to line up; the missing quadrant at
 * the eight three-face vertices and inactive pixels get weight 0 and the rest
 * is renormalised.  SSIM = ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)
 * (sx^2 + sy^2 + C2)).  out[0] = mean SSIM over active pixels and channels
 * (the masked average of the supplementary HSSIM metric), out[1] = mean L1,
 * out[2] = L = (1 - lambda) L1 + lambda (1 - mean SSIM).
 * img, ref: [3][n_active] in mask order; ssim_map [3][n_active] nullable.
 * If dL_dloss (device scalar) is non-null, dL_dimg [3][n_active] receives
 * dL_dloss * dL/dimg.  tables: from hp_ssim_tables for this mask (required).
 * Orders 0-12, tiles of 1 to 16 pixels a side; tiles narrower than 8
 * pixels (orders 0-2), where the window is wider than a face, sum the 121
 * taps directly instead of in two separable passes.
 * ws: hp_ssim_workspace_bytes. */
size_t hp_ssim_workspace_bytes(int32_t order, int32_t tile_log2, int64_t n_active);
hp_status hp_ssim(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                  const hp_params* prm, const hp_ssim_params* sp, const void* mask, const int32_t* tables, float* out,
                  float* ssim_map, const float* dL_dloss, float* dL_dimg, void* ws, size_t ws_bytes, void* stream);

/* hp_ssim_tables: the image-independent part of the HSSIM gathers, built
 * once per mask and passed to every hp_ssim call on that mask: for each
 * active tile and each cell of its (B + 10)^2 patch (the tile and a 5-pixel
 * halo on the face-extended chart), the compact slot of the neighbour pixel
 * (-1 where it is missing or inactive) with bit 30 set when the neighbour
 * lies in a polar cap.  tables: device int32 buffer of
 * hp_ssim_tables_bytes(order, tile_log2, n_tiles) bytes (2,704 per active
 * tile with 16 x 16 tiles). */
size_t hp_ssim_tables_bytes(int32_t order, int32_t tile_log2, int32_t n_tiles);
hp_status hp_ssim_tables(const hp_params* prm, const void* mask, int32_t order, int64_t n_active, int32_t n_tiles,
                         int32_t* tables, size_t tables_bytes, void* stream);

/* The same loss split at the point where the upstream gradient becomes known
 * (an autograd forward and its later backward).  hp_ssim_forward_saved does
 * what hp_ssim does without dL_dloss and also leaves the per-pixel SSIM
 * partials of the backward (12 floats per active pixel) in ws;
 * hp_ssim_backward_saved then computes dL_dimg = dL_dloss * dL/dimg from them
 * with the gather pass alone.  Between the two calls the caller keeps ws, img
 * and ref unchanged; both calls take the same sizes, mask, tables and
 * parameters.  Errors as hp_ssim; the backward's dL_dloss and dL_dimg are
 * required. */
hp_status hp_ssim_forward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                                const hp_params* prm, const hp_ssim_params* sp, const void* mask,
                                const int32_t* tables, float* out, float* ssim_map, void* ws, size_t ws_bytes,
                                void* stream);
hp_status hp_ssim_backward_saved(const float* img, const float* ref, int64_t n_active, int32_t n_tiles, int32_t order,
                                 const hp_params* prm, const hp_ssim_params* sp, const void* mask,
                                 const int32_t* tables, const void* ws, size_t ws_bytes, const float* dL_dloss,
                                 float* dL_dimg, void* stream);

/* ---- image synthesis (Eq. camera_synthesis; supp. camera models) ----------
 * Camera images are planar float [3][H][W] (channel, row, column), row 0 at
 * the top; pixel (i, j) is centred at (u, v) = (i + 1/2, j + 1/2).  The camera
 * model is view->cam_type with view->fov_x / fov_y (radians): HP_CAM_PINHOLE
 * (focal lengths W / (2 tan(fov_x / 2)), H / (2 tan(fov_y / 2))),
 * HP_CAM_FISHEYE (anisotropic equidistant, Eq. fish_weff, f = W / pi, H / pi,
 * valid inside the inscribed ellipse), HP_CAM_FULL (equirectangular
 * panorama, longitude 2 pi u / W - pi, latitude pi / 2 - pi v / H).  All
 * models share one camera frame: +z optical axis, +x right, +y up.
 *
 * hp_sphere_to_image: I_C(u, v) = Interp_H(I_H, P_C(u, v)).  img holds the
 * HEALPix image [3][n_active] in the order of `mask` (hp_mask for the same
 * view and order; n_active from hp_mask_counts).  Interp_H is bilinear over
 * the ring structure (two enclosing rings, two enclosing pixels per ring,
 * linear in longitude and in colatitude; the pole value is the mean of the
 * nearest ring's four pixels); neighbours outside the mask get weight 0 and
 * the rest are renormalised.  out [3][H][W] receives the image; valid
 * [H][W] (nullable) 1 where the pixel lies in the camera's domain and has an
 * active neighbour, else 0 and out = 0.
 *
 * hp_image_to_sphere: samples of the camera image img [3][H][W] at the
 * centres of the mask's active pixels (supp. Eq. supp_image_to_healpix):
 * bilinear over image pixel centres, clamped at the border (wrapped in
 * longitude for the panorama).  out [3][n_active]; valid [n_active]
 * (nullable) 1 where the centre projects into the camera's domain.
 *
 * Both: asynchronous on `stream`; HP_ERR_INVALID_ARG for null pointers,
 * W or H <= 0, W * H > 2^31, n_active outside [0, 12 * 4^order], or an
 * invalid view.  All buffers are device memory owned by the caller. */
hp_status hp_sphere_to_image(const void* mask, const hp_view* view, const hp_params* prm, int64_t n_active,
                             const float* img, int32_t W, int32_t H, float* out, uint8_t* valid, void* stream);
hp_status hp_image_to_sphere(const void* mask, const hp_view* view, const hp_params* prm, int64_t n_active,
                             const float* img, int32_t W, int32_t H, float* out, uint8_t* valid, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HP_H */
