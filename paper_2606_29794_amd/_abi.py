"""ctypes mirror of include/hp.h.  Argument marshalling only: every step of
the rasterizer runs in libhp.so's HIP kernels.  Loading fails loudly when the
library is missing -- there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HP_SANITIZED=1 selects the host-sanitized build (build.py, sanitize=True),
# for host-only checks in a process that preloads the ASan runtime
LIB_PATH = os.path.join(HERE, "libhp_san.so" if os.environ.get("HP_SANITIZED") == "1" else "libhp.so")

HP_OK, HP_ERR_INVALID_ARG, HP_ERR_UNSUPPORTED, HP_ERR_CAPACITY, HP_ERR_DEVICE = 0, 1, 2, 3, 4
HP_CAM_FULL, HP_CAM_FISHEYE, HP_CAM_PINHOLE = 0, 1, 2
HP_BIN_COUNT, HP_BIN_EMIT, HP_BIN_ALL = 1, 2, 3
HP_QUERY_RING, HP_QUERY_NESTED = 1, 2
HP_NOALLOC_MAX_P = 1 << 20   # largest scene of hp_render_bwd_noalloc


class HPError(RuntimeError):
    def __init__(self, name: str, status: int, msg: str):
        super().__init__(f"{name} failed: {msg} (status {status})")
        self.status = status


class hp_params(C.Structure):
    _fields_ = [("eps_T", C.c_float), ("alpha_max", C.c_float), ("q_cut", C.c_float), ("r_min", C.c_float),
                ("rs_sigma", C.c_float), ("bin_guard", C.c_float), ("sh_offset", C.c_float),
                ("tile_log2", C.c_int32)]


class hp_view(C.Structure):
    _fields_ = [("W", C.c_float * 9), ("b", C.c_float * 3), ("center", C.c_float * 3), ("cam_type", C.c_int32),
                ("fov_x", C.c_float), ("fov_y", C.c_float), ("order", C.c_int32)]


class hp_gaussians(C.Structure):
    _fields_ = [("P", C.c_int64), ("sh_degree", C.c_int32), ("mean", C.c_void_p), ("scale", C.c_void_p),
                ("rot", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class hp_gaussians_grad(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("rot", C.c_void_p), ("opacity", C.c_void_p),
                ("sh", C.c_void_p)]


class hp_render_req(C.Structure):
    _fields_ = [("projected", C.c_void_p), ("P", C.c_int64), ("vals", C.c_void_p), ("tile_ranges", C.c_void_p),
                ("n_tiles", C.c_int32), ("order", C.c_int32), ("mask", C.c_void_p), ("n_active", C.c_int64),
                ("rgb", C.c_void_p), ("T", C.c_void_p), ("n_contrib", C.c_void_p)]


class hp_ssim_params(C.Structure):
    _fields_ = [("sigma", C.c_float), ("C1", C.c_float), ("C2", C.c_float), ("lam", C.c_float), ("zones", C.c_int32)]


P_ = C.c_void_p
I32, I64, SZ = C.c_int32, C.c_int64, C.c_size_t
_PROTOS = {
    "hp_default_params": (None, [C.POINTER(hp_params)]),
    "hp_default_ssim_params": (None, [C.POINTER(hp_ssim_params)]),
    "hp_status_string": (C.c_char_p, [I32]),
    "hp_grid_bytes": (SZ, [I32, I32]),
    "hp_grid_init": (I32, [I32, C.POINTER(hp_params), P_, SZ, P_]),
    "hp_mask_bytes": (SZ, [I32, I32]),
    "hp_mask": (I32, [C.POINTER(hp_view), C.POINTER(hp_params), P_, P_, SZ, P_]),
    "hp_mask_counts": (I32, [P_, I32, I32, C.POINTER(I64), C.POINTER(I32), P_]),
    "hp_mask_active_pix": (P_, [P_, I32, I32]),
    "hp_projected_bytes": (SZ, [I64]),
    "hp_preprocess": (I32, [C.POINTER(hp_gaussians), C.POINTER(hp_view), C.POINTER(hp_params), P_, SZ, P_]),
    "hp_projected_depth": (P_, [P_, I64]),
    "hp_preprocess_batch": (I32, [C.POINTER(hp_gaussians), I32, C.POINTER(hp_view), C.POINTER(hp_params),
                                  C.POINTER(P_), SZ, P_]),
    "hp_render_fwd_batch": (I32, [I32, C.POINTER(hp_render_req), C.POINTER(hp_params), P_]),
    "hp_render_queue_bytes": (SZ, [I64]),
    "hp_render_queue_reset": (I32, [P_, SZ, P_]),
    "hp_render_queue_push": (I32, [P_, SZ, I32, C.POINTER(hp_render_req), C.POINTER(hp_params), I32, P_]),
    "hp_render_fwd_persistent": (I32, [P_, SZ, I32, I32, P_]),
    "hp_render_queue_status": (I32, [P_, I32, C.POINTER(I32), C.POINTER(I32), P_]),
    "hp_projected_radius": (P_, [P_, I64]),
    "hp_bin_workspace_bytes": (SZ, [I64]),
    "hp_bin": (I32, [I32, P_, I64, C.POINTER(hp_view), C.POINTER(hp_params), P_, P_, P_, P_, I64, P_, P_, SZ, P_]),
    "hp_bin_sorted_workspace_bytes": (SZ, [I64, I32, I32]),
    "hp_bin_sorted": (I32, [I32, P_, I64, C.POINTER(hp_view), C.POINTER(hp_params), P_, P_, P_, P_, I32, I64, P_, P_,
                            SZ, P_]),
    "hp_bin_query_workspace_bytes": (SZ, [I64, I32, I32]),
    "hp_bin_query": (I32, [I32, I32, I32, P_, I64, C.POINTER(hp_view), C.POINTER(hp_params), P_, P_, P_, P_, I32, I64,
                           P_, P_, P_, SZ, P_]),
    "hp_read_total": (I32, [P_, C.POINTER(I64), P_]),
    "hp_sort_workspace_bytes": (SZ, [I64, I32]),
    "hp_sort": (I32, [P_, P_, P_, I64, I32, P_, P_, SZ, P_]),
    "hp_check_count": (I32, [P_, I64, C.POINTER(I64), P_]),
    "hp_render_fwd": (I32, [P_, I64, P_, P_, I32, C.POINTER(hp_view), C.POINTER(hp_params), P_, I64, P_, P_, P_,
                            P_, P_, P_]),
    "hp_render_bwd_workspace_bytes": (SZ, [I64]),
    "hp_render_bwd": (I32, [C.POINTER(hp_gaussians), P_, P_, P_, I32, C.POINTER(hp_view), C.POINTER(hp_params), P_,
                            I64, P_, P_, P_, P_, P_, C.POINTER(hp_gaussians_grad), P_, SZ, P_]),
    "hp_render_bwd_pixels": (I32, [P_, I64, P_, P_, I32, C.POINTER(hp_view), C.POINTER(hp_params), P_, I64, P_, P_, P_,
                                   P_, P_, P_, P_]),
    "hp_mark_visible": (I32, [P_, P_, I32, I64, P_, P_]),
    "hp_density_stats": (I32, [P_, I64, P_, P_, P_, P_, P_, P_]),
    "hp_preprocess_bwd": (I32, [C.POINTER(hp_gaussians), C.POINTER(hp_view), C.POINTER(hp_params), P_,
                                C.POINTER(hp_gaussians_grad), P_]),
    "hp_render_bwd_noalloc": (I32, [C.POINTER(hp_gaussians), P_, P_, P_, I32, C.POINTER(hp_view), C.POINTER(hp_params),
                                    P_, I64, P_, P_, P_, P_, P_, C.POINTER(hp_gaussians_grad), P_]),
    "hp_ssim_workspace_bytes": (SZ, [I32, I32, I64]),
    "hp_ssim": (I32, [P_, P_, I64, I32, I32, C.POINTER(hp_params), C.POINTER(hp_ssim_params), P_, P_, P_, P_, P_, P_,
                      P_, SZ, P_]),
    "hp_ssim_tables_bytes": (SZ, [I32, I32, I32]),
    "hp_ssim_tables": (I32, [C.POINTER(hp_params), P_, I32, I64, I32, P_, SZ, P_]),
    "hp_ssim_forward_saved": (I32, [P_, P_, I64, I32, I32, C.POINTER(hp_params), C.POINTER(hp_ssim_params), P_, P_,
                                    P_, P_, P_, SZ, P_]),
    "hp_ssim_backward_saved": (I32, [P_, P_, I64, I32, I32, C.POINTER(hp_params), C.POINTER(hp_ssim_params), P_,
                                     P_, P_, SZ, P_, P_, P_]),
    "hp_sphere_to_image": (I32, [P_, C.POINTER(hp_view), C.POINTER(hp_params), I64, P_, I32, I32, P_, P_, P_]),
    "hp_image_to_sphere": (I32, [P_, C.POINTER(hp_view), C.POINTER(hp_params), I64, P_, I32, I32, P_, P_, P_]),
}

# every symbol the header declares
EXPORTS = tuple(_PROTOS)

_lib = None


def lib() -> C.CDLL:
    """The loaded libhp.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2606_29794_amd/build.py "
                               "(there is no non-HIP implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(name: str, status: int) -> None:
    if status != HP_OK:
        msg = lib().hp_status_string(status).decode()
        raise HPError(name, status, msg)


def call(name: str, *args) -> None:
    check(name, getattr(lib(), name)(*args))


def default_params(**kw) -> hp_params:
    p = hp_params()
    lib().hp_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def default_ssim_params(**kw) -> hp_ssim_params:
    p = hp_ssim_params()
    lib().hp_default_ssim_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def make_view(W, b, center, cam_type: int, fov_x: float, fov_y: float, order: int) -> hp_view:
    v = hp_view()
    Wl = [float(x) for x in list(_flat(W))]
    for k in range(9):
        v.W[k] = Wl[k]
    for k, x in enumerate(_flat(b)):
        v.b[k] = float(x)
    for k, x in enumerate(_flat(center)):
        v.center[k] = float(x)
    v.cam_type = int(cam_type)
    v.fov_x = float(fov_x)
    v.fov_y = float(fov_y)
    v.order = int(order)
    return v


def _flat(a):
    try:
        import numpy as np
        return np.asarray(a, dtype=np.float64).reshape(-1).tolist()
    except Exception:  # pragma: no cover
        return list(a)
