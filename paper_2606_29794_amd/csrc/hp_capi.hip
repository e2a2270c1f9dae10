// hp_capi.hip -- parameter defaults, status strings and small read-back
// helpers of the C ABI (include/hp.h).
#include "hp_common.h"

extern "C" void hp_default_params(hp_params* p) {
  if (!p) return;
  p->eps_T = 1e-4f;
  p->alpha_max = 0.99f;
  p->q_cut = 9.0f;
  p->r_min = 0.1f;
  p->rs_sigma = 3.0f;
  p->bin_guard = 1e-6f;
  p->sh_offset = 0.5f;
  p->tile_log2 = 4;
}

extern "C" void hp_default_ssim_params(hp_ssim_params* p) {
  if (!p) return;
  p->sigma = 1.5f;
  p->C1 = 0.01f * 0.01f;
  p->C2 = 0.03f * 0.03f;
  p->lambda = 0.2f;
  p->zones = 0;
}

extern "C" const char* hp_status_string(hp_status s) {
  switch (s) {
    case HP_OK: return "ok";
    case HP_ERR_INVALID_ARG: return "invalid argument";
    case HP_ERR_UNSUPPORTED: return "unsupported";
    case HP_ERR_CAPACITY: return "buffer too small";
    case HP_ERR_DEVICE: return "device error";
    default: return "unknown status";
  }
}

extern "C" hp_status hp_read_total(const int64_t* dev_value, int64_t* host_value, void* stream) {
  if (!dev_value || !host_value) return HP_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  int64_t v = 0;
  HP_TRY(hp_read_small(&v, dev_value, sizeof(v), s));
  *host_value = v;
  return HP_OK;
}

extern "C" hp_status hp_check_count(const int64_t* dev_count, int64_t capacity, int64_t* host_count, void* stream) {
  if (!dev_count || capacity < 0) return HP_ERR_INVALID_ARG;
  int64_t v = 0;
  HP_TRY(hp_read_small(&v, dev_count, sizeof(v), (hipStream_t)stream));
  if (host_count) *host_count = v;
  return (v < 0 || v > capacity) ? HP_ERR_CAPACITY : HP_OK;
}
