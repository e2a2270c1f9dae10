// k_render_noalloc.hip -- hp_render_bwd_noalloc: the render backward of
// hp_render_bwd with its per-Gaussian accumulators in a fixed device array
// of this library instead of a caller workspace, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).
#include <mutex>

#include "hp_common.h"

// accumulators of the pixel pass: [10][P] floats for P <= HP_NOALLOC_MAX_P
// (40 MiB, held on every device the library runs on until the process ends)
static __device__ __align__(256) float scratch[10 * (size_t)HP_NOALLOC_MAX_P];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_scratch[kMaxDevices];
hipError_t g_err[kMaxDevices];

// device address of `scratch` on the current device, looked up once per
// device (the array's name in host code is only a host-side stand-in)
hp_status scratch_on_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HP_ERR_DEVICE;
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess || !g_scratch[dev]) return HP_ERR_DEVICE;
  *out = (float*)g_scratch[dev];
  return HP_OK;
}

}  // namespace

extern "C" hp_status hp_render_bwd_noalloc(const hp_gaussians* gs, const void* projected, const uint32_t* vals,
                                           const uint32_t* tile_ranges, int32_t n_tiles, const hp_view* view,
                                           const hp_params* prm, const void* mask, int64_t n_active, const float* T,
                                           const int32_t* n_contrib, const float* dL_drgb, const float* dL_dT,
                                           const float* dL_dinv_depth, hp_gaussians_grad* grad, void* stream) {
  HP_TRY(hp_check_gaussians(gs));
  HP_TRY(hp_check_view(view, prm));
  if (!projected || !mask || !grad || n_tiles < 0 || n_active < 0) return HP_ERR_INVALID_ARG;
  if (gs->P > 0 && (!grad->mean || !grad->scale || !grad->rot || !grad->opacity || !grad->sh))
    return HP_ERR_INVALID_ARG;
  if (n_active > 0 && n_tiles > 0 && (!T || !n_contrib || !dL_drgb || !tile_ranges || !vals)) return HP_ERR_INVALID_ARG;
  if (gs->P > HP_NOALLOC_MAX_P) return HP_ERR_CAPACITY;
  if (gs->P == 0) return HP_OK;
  float* acc = nullptr;
  HP_TRY(scratch_on_current_device(&acc));
  return hp_render_bwd_acc(gs, projected, vals, tile_ranges, n_tiles, view, prm, mask, n_active, T, n_contrib, dL_drgb,
                           dL_dT, dL_dinv_depth, grad, acc, stream);
}
