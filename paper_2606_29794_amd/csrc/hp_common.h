// hp_common.h -- host-side helpers shared by the C-ABI entry points.
#pragma once

#include <math.h>
#include <string.h>

#include "hp_device.h"

#define HP_CHECK_LAUNCH()                                   \
  do {                                                      \
    if (hipGetLastError() != hipSuccess) return HP_ERR_DEVICE; \
  } while (0)

#define HP_TRY(expr)                 \
  do {                               \
    hp_status _s = (expr);           \
    if (_s != HP_OK) return _s;      \
  } while (0)

// float not below the double value (keeps cap radii conservative)
HP_HD float hp_round_up_f(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

static inline hp_status hp_check_params(const hp_params* p) {
  if (!p) return HP_ERR_INVALID_ARG;
  if (p->tile_log2 < 0 || p->tile_log2 > 4) return HP_ERR_INVALID_ARG;
  if (!(p->eps_T > 0 && p->eps_T < 1) || !(p->alpha_max > 0 && p->alpha_max < 1) || !(p->q_cut > 0) ||
      !(p->r_min >= 0) || !(p->rs_sigma > 0) || !(p->bin_guard >= 0))
    return HP_ERR_INVALID_ARG;
  return HP_OK;
}

static inline hp_status hp_check_view(const hp_view* v, const hp_params* p) {
  if (!v) return HP_ERR_INVALID_ARG;
  HP_TRY(hp_check_params(p));
  if (v->order < 0 || v->order > HP_MAX_ORDER) return HP_ERR_INVALID_ARG;
  if (v->cam_type < HP_CAM_FULL || v->cam_type > HP_CAM_PINHOLE) return HP_ERR_INVALID_ARG;
  for (int k = 0; k < 9; ++k)
    if (!isfinite(v->W[k])) return HP_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(v->b[k]) || !isfinite(v->center[k])) return HP_ERR_INVALID_ARG;
  if (v->cam_type == HP_CAM_FISHEYE && !(v->fov_x > 0 && v->fov_y > 0 && v->fov_x <= 2 * M_PI && v->fov_y <= 2 * M_PI))
    return HP_ERR_INVALID_ARG;
  if (v->cam_type == HP_CAM_PINHOLE && !(v->fov_x > 0 && v->fov_y > 0 && v->fov_x < M_PI && v->fov_y < M_PI))
    return HP_ERR_INVALID_ARG;
  return HP_OK;
}

static inline hp_status hp_check_gaussians(const hp_gaussians* g) {
  if (!g) return HP_ERR_INVALID_ARG;
  if (g->P < 0 || g->P > ((int64_t)1 << 31) - 1) return HP_ERR_INVALID_ARG;
  if (g->sh_degree < 0 || g->sh_degree > HP_MAX_SH_DEGREE) return HP_ERR_INVALID_ARG;
  if (g->P > 0 && (!g->mean || !g->scale || !g->rot || !g->opacity || !g->sh)) return HP_ERR_INVALID_ARG;
  return HP_OK;
}

// view constants passed to kernels by value
struct HpViewK {
  float W[9], b[3], c[3];
};
static inline HpViewK hp_viewk(const hp_view* v) {
  HpViewK k;
  memcpy(k.W, v->W, sizeof(k.W));
  memcpy(k.b, v->b, sizeof(k.b));
  memcpy(k.c, v->center, sizeof(k.c));
  return k;
}

static inline unsigned hp_blocks(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// Small device-to-host read that waits for `s`, straight into the caller's
// host memory (no staging buffer is allocated).
static inline hp_status hp_read_small(void* dst, const void* src, size_t n, hipStream_t s) {
  if (hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s) != hipSuccess) return HP_ERR_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return HP_ERR_DEVICE;
  return HP_OK;
}

// hp_bin_sorted with every Gaussian's test angle widened by `widen` radians
// (0: identical to hp_bin_sorted); the candidate stage of hp_bin_query.
hp_status hp_bin_sorted_widened(int32_t phase, const void* projected, int64_t P, const hp_view* view,
                                const hp_params* prm, const void* grid, const void* mask, uint32_t* vals,
                                uint32_t* tile_ranges, int32_t n_tiles, int64_t capacity, int64_t* n_pairs, void* ws,
                                size_t ws_bytes, void* stream, double widen);

// hp_render_bwd after its argument checks, accumulators [HP_NACC][P] at acc
hp_status hp_render_bwd_acc(const hp_gaussians* gs, const void* projected, const uint32_t* vals,
                            const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view, const hp_params* prm,
                            const void* mask, int64_t n_active, const float* T, const int32_t* n_contrib,
                            const float* dL_drgb, const float* dL_dT, const float* dL_dinv_depth,
                            hp_gaussians_grad* grad, float* acc, void* stream);
