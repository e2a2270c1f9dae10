"""FP64 CPU oracle of the HEALPix Gaussian rasterizer -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2606_29794_amd``); the two meet only through the seeded inputs of
``paper_2606_29794_amd.scenes``.

The arithmetic lives in ``hp_oracle.cpp`` (plain C++17, double precision,
OpenMP loops); this module builds it with g++ and wraps it with ctypes.
Each wrapper names the paper passage the underlying routine follows.

Parity status of each function is stated in tests/test_oracle_*.py; all of
them are pinned there (closed forms, invariants, finite differences).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hp_oracle.cpp")
_LIB = os.path.join(_HERE, "libhp_oracle.so")

# constants of the method (readings of the paper; identical values are used
# by the HIP path, which defines its own copy)
EPS_T = 1e-4          # early-termination transmittance (Alg. 1)
ALPHA_MAX = 0.99      # opacity clamp
Q_CUT = 9.0           # 3-sigma Mahalanobis support
R_MIN = 0.1           # near cull on radial depth
RS_SIGMA = 3.0        # r_s = 3 sqrt(lambda_max)  (Sec. 3.2)
BIN_GUARD = 1e-6      # radians added to the tile-overlap test
SH_OFFSET = 0.5
TILE_LOG2 = 4         # B = 16 (Table tab:resolution)
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
LAMBDA = 0.2


_LIB_SAN = os.path.join(_HERE, "libhp_oracle_san.so")
# checking build: AddressSanitizer + UBSan (g++); a process that loads it
# must preload g++'s ASan runtime (asan_runtime) and set HP_ORACLE_SANITIZED=1
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile hp_oracle.cpp into libhp_oracle.so (g++, -O2, OpenMP), or
    with sanitize into libhp_oracle_san.so."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        opt = _SAN_FLAGS if sanitize else ["-O2"]
        cmd = ["g++", *opt, "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return lib


def asan_runtime() -> str:
    """g++'s ASan runtime, which a process loading libhp_oracle_san.so preloads."""
    path = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("g++'s ASan runtime was not found")
    return path


class _Scene(C.Structure):
    _fields_ = [("P", C.c_int64), ("sh_degree", C.c_int),
                ("mean", C.c_void_p), ("scale", C.c_void_p), ("rot", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class _View(C.Structure):
    _fields_ = [("W", C.c_double * 9), ("b", C.c_double * 3), ("center", C.c_double * 3),
                ("cam_type", C.c_int), ("fov_x", C.c_double), ("fov_y", C.c_double), ("order", C.c_int)]


class _Params(C.Structure):
    _fields_ = [("eps_T", C.c_double), ("alpha_max", C.c_double), ("q_cut", C.c_double),
                ("r_min", C.c_double), ("rs_sigma", C.c_double), ("bin_guard", C.c_double),
                ("sh_offset", C.c_double), ("tile_log2", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build(sanitize=os.environ.get("HP_ORACLE_SANITIZED") == "1"))
        _lib.or_mask.restype = C.c_int64
        _lib.or_tile_sets.restype = C.c_int64
        _lib.or_chart_pixel.restype = C.c_int64
        _lib.or_hssim.restype = C.c_double
        _lib.or_num_threads.restype = C.c_int
        _lib.or_query_tiles.restype = C.c_int64
    return _lib


def _p(a):
    """Pointer argument for a call; the returned object keeps `a` alive, so a
    temporary (np.ascontiguousarray of a strided view) lives until the call
    that receives it returns."""
    if a is None:
        return None
    v = C.c_void_p(a.ctypes.data)
    v._keep = a
    return v


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def params(**kw) -> _Params:
    d = dict(eps_T=EPS_T, alpha_max=ALPHA_MAX, q_cut=Q_CUT, r_min=R_MIN, rs_sigma=RS_SIGMA,
             bin_guard=BIN_GUARD, sh_offset=SH_OFFSET, tile_log2=TILE_LOG2)
    d.update(kw)
    return _Params(**d)


def view_struct(cam: dict) -> _View:
    v = _View()
    W = np.asarray(cam["W"], np.float32).astype(np.float64).reshape(-1)
    for k in range(9):
        v.W[k] = W[k]
    for k in range(3):
        v.b[k] = float(np.float32(cam["b"][k]))
        v.center[k] = float(np.float32(cam["center"][k]))
    v.cam_type = int(cam["cam_type"])
    # the C ABI carries the field of view as float32: use the same input value
    v.fov_x = float(np.float32(cam["fov_x"]))
    v.fov_y = float(np.float32(cam["fov_y"]))
    v.order = int(cam["order"])
    return v


class SceneRef:
    """Keeps the float32 arrays alive while the C struct points at them."""

    def __init__(self, scene):
        self.arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in
                     (scene.mean, scene.scale, scene.rot, scene.opacity, scene.sh)]
        self.s = _Scene(scene.P, scene.sh_degree, *[a.ctypes.data for a in self.arrs])
        self.P = scene.P
        self.K = (scene.sh_degree + 1) ** 2


# ---------------------------------------------------------------------------
# HEALPix geometry (Gorski et al. 2005; the grid of Sec. 3.1)
# ---------------------------------------------------------------------------

def npix(order: int) -> int:
    return 12 * (1 << (2 * order))


def nest2xyf(order, p):
    p = np.ascontiguousarray(p, np.int64)
    x = np.empty_like(p); y = np.empty_like(p); f = np.empty(p.shape, np.int32)
    lib().or_nest2xyf(order, C.c_int64(p.size), _p(p), _p(x), _p(y), _p(f))
    return x, y, f


def xyf2nest(order, x, y, f):
    x = np.ascontiguousarray(x, np.int64); y = np.ascontiguousarray(y, np.int64)
    f = np.ascontiguousarray(f, np.int32); p = np.empty_like(x)
    lib().or_xyf2nest(order, C.c_int64(x.size), _p(x), _p(y), _p(f), _p(p))
    return p


def nest2ring(order, p):
    p = np.ascontiguousarray(p, np.int64); r = np.empty_like(p)
    lib().or_nest2ring(order, C.c_int64(p.size), _p(p), _p(r))
    return r


def ring2nest_table(order):
    """Inverse of nest2ring by inverting the full table (plain and exact)."""
    p = np.arange(npix(order), dtype=np.int64)
    r = nest2ring(order, p)
    inv = np.full(p.size, -1, np.int64)
    inv[r] = p
    return inv


def pix_ringinfo(order, p):
    p = np.ascontiguousarray(p, np.int64)
    jr = np.empty_like(p); jp = np.empty_like(p)
    z = np.empty(p.shape, np.float64); phi = np.empty(p.shape, np.float64)
    lib().or_pix_ringinfo(order, C.c_int64(p.size), _p(p), _p(jr), _p(jp), _p(z), _p(phi))
    return jr, jp, z, phi


def pix_vec(order, p):
    """Camera-frame unit vectors [n][3] of nested pixel centres."""
    p = np.ascontiguousarray(p, np.int64)
    v = np.empty((p.size, 3), np.float64)
    lib().or_pix_vec(order, C.c_int64(p.size), _p(p), _p(v))
    return v


def chart_pixel(order, f, x, y) -> int:
    return int(lib().or_chart_pixel(order, int(f), C.c_int64(int(x)), C.c_int64(int(y))))


def tile_order(order: int, tile_log2: int = TILE_LOG2) -> int:
    return order - min(tile_log2, order)


# ---------------------------------------------------------------------------
# Camera mask (Sec. 3.1 M_C; supp. camera models)
# ---------------------------------------------------------------------------

def mask(cam: dict) -> np.ndarray:
    v = view_struct(cam)
    n = lib().or_mask(C.byref(v), None)
    out = np.empty(n, np.int64)
    lib().or_mask(C.byref(v), _p(out))
    return out


def nside_star(W: float, H: float, omega_in: float) -> float:
    """Continuous matched resolution N* = sqrt(4 pi W H / (12 Omega_in)) (Sec. 3.1)."""
    return math.sqrt(4 * math.pi * W * H / (12.0 * omega_in))


def omega_in(kind: str, theta: float = 0.0, theta_x: float = 0.0, theta_y: float = 0.0) -> float:
    """Visible solid angle: 4 pi (equirectangular), 2 pi (1 - cos theta)
    (fisheye, half-FoV theta), 4 asin(sin theta_x sin theta_y) (perspective)."""
    if kind == "erp":
        return 4 * math.pi
    if kind == "fisheye":
        return 2 * math.pi * (1 - math.cos(theta))
    if kind == "pinhole":
        return 4 * math.asin(math.sin(theta_x) * math.sin(theta_y))
    raise ValueError(kind)


def orders_for(W, H, om):
    """(k, k_L, k_H) = (round, floor, ceil) of log2 N* (Table tab:resolution)."""
    l2 = math.log2(nside_star(W, H, om))
    return int(round(l2)), int(math.floor(l2)), int(math.ceil(l2))


# ---------------------------------------------------------------------------
# SH, preprocessing, tiles, compositing, gradients, HSSIM
# ---------------------------------------------------------------------------

def sh_basis(deg: int, v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    Y = np.zeros((v.shape[0], 16), np.float64)
    lib().or_sh_basis(deg, C.c_int64(v.shape[0]), _p(v), _p(Y))
    return Y[:, : (deg + 1) ** 2]


@dataclass
class Projected:
    valid: np.ndarray
    omega: np.ndarray
    phi: np.ndarray
    rho: np.ndarray
    conic: np.ndarray   # [3][P]  (A, B, C)
    sarc: np.ndarray    # [3][P]  Sigma_arc (omega-omega, omega-phi, phi-phi)
    rs: np.ndarray
    rgb: np.ndarray     # [3][P]

    def dirs(self) -> np.ndarray:
        """Camera-frame unit directions [3][P]."""
        c = np.cos(self.phi)
        return np.stack([c * np.sin(self.omega), np.sin(self.phi), c * np.cos(self.omega)])


def preprocess(scene, cam, prm=None) -> Projected:
    prm = prm or params()
    S = SceneRef(scene)
    v = view_struct(cam)
    P = scene.P
    valid = np.zeros(P, np.int32)
    om = np.zeros(P); ph = np.zeros(P); rho = np.zeros(P); rs = np.zeros(P)
    conic = np.zeros((3, P)); sarc = np.zeros((3, P)); rgb = np.zeros((3, P))
    lib().or_preprocess(C.byref(S.s), C.byref(v), C.byref(prm), _p(valid), _p(om), _p(ph), _p(rho),
                        _p(conic), _p(sarc), _p(rs), _p(rgb))
    return Projected(valid, om, ph, rho, conic, sarc, rs, rgb)


def tile_caps(order: int, tile_log2: int = TILE_LOG2):
    kt = tile_order(order, tile_log2)
    nt = 12 * (1 << (2 * kt))
    c = np.zeros((nt, 3)); r = np.zeros(nt)
    lib().or_tile_caps(order, tile_log2, _p(c), _p(r))
    return c, r


def tile_active(order: int, active: np.ndarray, tile_log2: int = TILE_LOG2) -> np.ndarray:
    kt = tile_order(order, tile_log2)
    nt = 12 * (1 << (2 * kt))
    t = np.zeros(nt, np.uint8)
    t[np.asarray(active) >> (2 * (order - kt))] = 1
    return t


def tile_sets(order, proj: Projected, active, gids=None, prm=None, caps=None, report_band=0.0):
    """Binning definition: (gid, tile, margin, in) for every valid Gaussian in
    gids and every active tile with distance(cap centre, Gaussian) within
    r_s + R_t + guard (in = 1), plus near misses within report_band (in = 0)."""
    prm = prm or params()
    tc, tr = caps if caps is not None else tile_caps(order, prm.tile_log2)
    ta = tile_active(order, active, prm.tile_log2)
    P = proj.valid.size
    gids = np.arange(P, dtype=np.int64) if gids is None else np.ascontiguousarray(gids, np.int64)
    args = (order, C.byref(prm), _p(np.ascontiguousarray(tc)), _p(np.ascontiguousarray(tr)), _p(ta),
            C.c_int64(gids.size), _p(gids), _p(proj.valid), _p(proj.omega), _p(proj.phi), _p(proj.rs),
            C.c_double(report_band))
    n = lib().or_tile_sets(*args, C.c_int64(0), None, None, None, None)
    g = np.empty(n, np.int64); t = np.empty(n, np.int64); m = np.empty(n); i = np.empty(n, np.int32)
    lib().or_tile_sets(*args, C.c_int64(n), _p(g), _p(t), _p(m), _p(i))
    return g, t, m, i


def sorted_tile_lists(order, proj: Projected, g, t, inn, prm=None):
    """Per-tile lists ordered by (rho, gid) (Alg. 1 sort; ties by index).
    Returns (list, ranges[ntile][2]) over the pairs with inn == 1."""
    prm = prm or params()
    kt = tile_order(order, prm.tile_log2)
    nt = 12 * (1 << (2 * kt))
    sel = inn.astype(bool)
    g = g[sel]; t = t[sel]
    order_idx = np.lexsort((g, proj.rho[g], t))
    lst = g[order_idx]
    ts = t[order_idx]
    starts = np.searchsorted(ts, np.arange(nt), side="left")
    ends = np.searchsorted(ts, np.arange(nt), side="right")
    return lst, np.stack([starts, ends], axis=1).astype(np.int64)


def render(scene, cam, proj: Projected, pix, prm=None, qtol=0.0, ttol=0.0, want_depth=False, qtol_rel=0.0,
           qtol_dir=0.0):
    """Brute-force compositing at nested pixels `pix` (Eq. unified_rendering).
    Returns rgb [3][n], T [n], n_used [n], frag [n]; with want_depth also the
    composited inverse radial depth [n] (sum of alpha T / rho, Sec. 3.2).
    frag is the allowance of the pixel's fragile decisions (0: none): q within
    qtol + qtol_rel (|A| dx^2 + 2 |B dx dy| + |C| dy^2) + 2 qtol_dir
    sqrt(q_cut lambda_max(conic)) of q_cut (the magnitudes of q's terms, and
    the change of q an offset error of qtol_dir radians causes), T within
    ttol (relative) of eps_T."""
    prm = prm or params()
    S = SceneRef(scene)
    v = view_struct(cam)
    pix = np.ascontiguousarray(pix, np.int64)
    n = pix.size
    rgb = np.zeros((3, n)); T = np.zeros(n); nu = np.zeros(n, np.int64); fr = np.zeros(n)
    D = np.zeros(n) if want_depth else None
    qb = np.array([qtol, qtol_rel, qtol_dir])   # held until the call returns
    lib().or_render(C.byref(S.s), C.byref(v), C.byref(prm), _p(proj.valid), _p(proj.omega), _p(proj.phi),
                    _p(proj.rho), _p(np.ascontiguousarray(proj.conic)), _p(proj.rs),
                    _p(np.ascontiguousarray(proj.rgb)), C.c_int64(n), _p(pix), _p(qb),
                    C.c_double(ttol), _p(rgb), _p(T), _p(nu), _p(fr), _p(D))
    return (rgb, T, nu, fr, D) if want_depth else (rgb, T, nu, fr)


def n_contrib(scene, cam, proj: Projected, lst, ranges, pix, prm=None):
    prm = prm or params()
    S = SceneRef(scene)
    v = view_struct(cam)
    pix = np.ascontiguousarray(pix, np.int64)
    out = np.zeros(pix.size, np.int64)
    lst = np.ascontiguousarray(lst, np.int64)
    ranges = np.ascontiguousarray(ranges, np.int64)
    lib().or_n_contrib(C.byref(S.s), C.byref(v), C.byref(prm), _p(proj.omega), _p(proj.phi),
                       _p(np.ascontiguousarray(proj.conic)), _p(lst), _p(ranges), C.c_int64(pix.size), _p(pix),
                       _p(out))
    return out


def render_lists(scene, cam, proj: Projected, lst, ranges, pix, prm=None, qtol=0.0, ttol=0.0, qtol_rel=0.0,
                 qtol_dir=0.0):
    """Compositing at nested pixels `pix` where each pixel sees only its
    tile's list (lst / ranges as from sorted_tile_lists): the approximate
    tile sets of the paper's queries can leave a Gaussian out of a tile it
    reaches.  Returns rgb [3][n], T [n], n_used [n], frag [n] as render()."""
    prm = prm or params()
    S = SceneRef(scene)
    v = view_struct(cam)
    pix = np.ascontiguousarray(pix, np.int64)
    n = pix.size
    rgb = np.zeros((3, n)); T = np.zeros(n); nu = np.zeros(n, np.int64); fr = np.zeros(n)
    qb = np.array([qtol, qtol_rel, qtol_dir])   # held until the call returns
    lib().or_render_lists(C.byref(S.s), C.byref(v), C.byref(prm), _p(proj.omega), _p(proj.phi), _p(proj.rho),
                          _p(np.ascontiguousarray(proj.conic)), _p(np.ascontiguousarray(proj.rgb)),
                          _p(np.ascontiguousarray(lst, np.int64)), _p(np.ascontiguousarray(ranges, np.int64)),
                          C.c_int64(n), _p(pix), _p(qb), C.c_double(ttol),
                          _p(rgb), _p(T), _p(nu), _p(fr))
    return rgb, T, nu, fr


# ---------------------------------------------------------------------------
# The paper's tile queries (Sec. 3.3; Alg. 2 NESTED traversal, Alg. 3 RING scan)
# ---------------------------------------------------------------------------
QUERY_RING = 1
QUERY_NESTED = 2


def pixrad(kq: int) -> np.ndarray:
    """PixRad(o), o = 0 .. kq: the largest angle from a node centre at order o
    to the centre of one of its descendants at order kq (0 at o = kq)."""
    out = np.zeros(kq + 1)
    lib().or_pixrad(int(kq), _p(out))
    return out


def query_tiles(mode: int, order: int, proj: Projected, active, f: int, gids=None, drs_rel=0.0, drs_abs=0.0,
                prm=None, tile_active_mask=None):
    """(gid, tile) pairs of the paper's query `mode` (QUERY_RING / QUERY_NESTED)
    at search depth f (query order kt + log2 f), restricted to active tiles.
    The radius used is max(0, r_s (1 + drs_rel) + drs_abs)."""
    prm = prm or params()
    kt = tile_order(order, prm.tile_log2)
    fl = int(round(math.log2(f)))
    assert 1 << fl == f and kt + fl <= order
    ta = tile_active(order, active, prm.tile_log2) if tile_active_mask is None else \
        np.ascontiguousarray(tile_active_mask, np.uint8)
    P = proj.valid.size
    gids = np.arange(P, dtype=np.int64) if gids is None else np.ascontiguousarray(gids, np.int64)
    r2n = _ring2nest(kt + fl) if mode == QUERY_RING else None
    args = (int(mode), kt, fl, _p(r2n), _p(ta), C.c_int64(gids.size), _p(gids), _p(proj.valid),
            _p(proj.omega), _p(proj.phi), _p(proj.rs), C.c_double(drs_rel), C.c_double(drs_abs))
    n = lib().or_query_tiles(*args, C.c_int64(0), None, None)
    g = np.empty(n, np.int64); t = np.empty(n, np.int64)
    lib().or_query_tiles(*args, C.c_int64(n), _p(g), _p(t))
    return g, t


@dataclass
class Grads:
    mean: np.ndarray
    scale: np.ndarray
    rot: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray


def render_bwd(scene, cam, proj: Projected, pix, dLdC, dLdT=None, prm=None, dLdD=None, want_angles=False):
    """Exact gradients of L at pixels `pix` given dL/dC [3][n], dL/dT [n] and
    (optionally) dL/d(inverse depth) [n].  With want_angles also returns the
    per-Gaussian gradient with respect to the centre's (omega, phi) [2][P]."""
    prm = prm or params()
    S = SceneRef(scene)
    v = view_struct(cam)
    pix = np.ascontiguousarray(pix, np.int64)
    n = pix.size
    P = scene.P
    g = Grads(np.zeros((3, P)), np.zeros((3, P)), np.zeros((4, P)), np.zeros(P), np.zeros((S.K, 3, P)))
    dLdC = np.ascontiguousarray(dLdC, np.float64)
    dLdT = None if dLdT is None else np.ascontiguousarray(dLdT, np.float64)
    dLdD = None if dLdD is None else np.ascontiguousarray(dLdD, np.float64)
    ang = np.zeros((2, P)) if want_angles else None
    lib().or_render_bwd(C.byref(S.s), C.byref(v), C.byref(prm), _p(proj.valid), _p(proj.omega), _p(proj.phi),
                        _p(proj.rho), _p(np.ascontiguousarray(proj.conic)), _p(proj.rs),
                        _p(np.ascontiguousarray(proj.rgb)), C.c_int64(n), _p(pix), _p(dLdC), _p(dLdT),
                        _p(g.mean), _p(g.scale), _p(g.rot), _p(g.opacity), _p(g.sh), _p(dLdD), _p(ang))
    return (g, ang) if want_angles else g


def hssim(order, active, img, ref, sigma=SSIM_SIGMA, c1=SSIM_C1, c2=SSIM_C2, want_map=False, want_grad=False,
          zones=False):
    """Mean HEALPix-SSIM over active pixels and channels (Sec. 4.1, supp. eq.
    for the masked average); optional map [3][n] and d mean / d img [3][n].
    zones: the zone-specific windows (isotropic chart window in the
    equatorial belt, great-circle Gaussian of sigma pitches in the polar
    caps); otherwise the isotropic chart window everywhere."""
    active = np.ascontiguousarray(active, np.int64)
    img = np.ascontiguousarray(img, np.float64)
    ref = np.ascontiguousarray(ref, np.float64)
    n = active.size
    m = np.zeros((3, n)) if want_map else None
    g = np.zeros((3, n)) if want_grad else None
    mean = lib().or_hssim(order, C.c_int64(n), _p(active), _p(img), _p(ref), C.c_double(sigma), C.c_double(c1),
                          C.c_double(c2), int(bool(zones)), _p(m), _p(g))
    return mean, m, g


def hssim_window(order, p, sigma=SSIM_SIGMA, zones=False):
    """Raw window of nested pixel p: (neighbour ids [11, 11] with -1 in a
    missing quadrant, weights [11, 11]), indexed by the chart offsets
    (a + 5, b + 5)."""
    q = np.zeros(121, np.int64)
    w = np.zeros(121)
    lib().or_hssim_window(int(order), C.c_int64(int(p)), C.c_double(sigma), int(bool(zones)), _p(q), _p(w))
    return q.reshape(11, 11), w.reshape(11, 11)


def loss(order, active, img, ref, lam=LAMBDA, want_grad=False, zones=False):
    """L = (1 - lambda) L1 + lambda (1 - HSSIM) (Sec. 4.1); L1 = mean |img - ref|.
    Returns (L, dL/dimg or None)."""
    img = np.asarray(img, np.float64); ref = np.asarray(ref, np.float64)
    l1 = float(np.mean(np.abs(img - ref)))
    s, _, gs = hssim(order, active, img, ref, want_grad=want_grad, zones=zones)
    L = (1 - lam) * l1 + lam * (1 - s)
    if not want_grad:
        return L, None
    g = (1 - lam) * np.sign(img - ref) / img.size - lam * gs
    return L, g


# ---------------------------------------------------------------------------
# Image synthesis between the sphere and camera images (Eq. camera_synthesis,
# Interp_H; supp. camera models; supp. Eq. supp_image_to_healpix).  Readings:
# one y-up camera frame for every model, pixel centres at half-integers,
# ring-bilinear Interp_H with the pole as the mean of the nearest ring and
# renormalisation over active neighbours (see hp_oracle.cpp).
# ---------------------------------------------------------------------------

def _cam_args(cam):
    return int(cam["cam_type"]), float(np.float32(cam["fov_x"])), float(np.float32(cam["fov_y"]))


def cam_rays(cam: dict, W: int, H: int, uv) -> tuple:
    """Camera-frame unit rays [n][3] through image positions uv [n][2], and
    whether each lies in the camera's valid domain."""
    uv = np.ascontiguousarray(uv, np.float64).reshape(-1, 2)
    d = np.empty((uv.shape[0], 3), np.float64)
    ok = np.empty(uv.shape[0], np.int32)
    t, fx, fy = _cam_args(cam)
    lib().or_cam_rays(t, int(W), int(H), C.c_double(fx), C.c_double(fy), C.c_int64(uv.shape[0]), _p(uv), _p(d), _p(ok))
    return d, ok.astype(bool)


def cam_project(cam: dict, W: int, H: int, d) -> tuple:
    """Image positions [n][2] of camera-frame directions d [n][3] and validity."""
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    uv = np.empty((d.shape[0], 2), np.float64)
    ok = np.empty(d.shape[0], np.int32)
    t, fx, fy = _cam_args(cam)
    lib().or_cam_project(t, int(W), int(H), C.c_double(fx), C.c_double(fy), C.c_int64(d.shape[0]), _p(d), _p(uv), _p(ok))
    return uv, ok.astype(bool)


_r2n_cache = {}


def _ring2nest(order):
    if order not in _r2n_cache:
        _r2n_cache[order] = np.ascontiguousarray(ring2nest_table(order))
    return _r2n_cache[order]


def interp_weights(order: int, d) -> tuple:
    """Interp_H at directions d [n][3]: NESTED pixels [n][4] and weights [n][4]."""
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    pix = np.empty((d.shape[0], 4), np.int64)
    w = np.empty((d.shape[0], 4), np.float64)
    lib().or_interp_weights(order, _p(_ring2nest(order)), C.c_int64(d.shape[0]), _p(d), _p(pix), _p(w))
    return pix, w


def sphere_to_image(cam: dict, active, img, W: int, H: int) -> tuple:
    """Camera image [3][H][W] (and valid flags [H][W]) from the HEALPix image
    img [3][n_active] on the sorted active pixels (Eq. camera_synthesis)."""
    active = np.ascontiguousarray(active, np.int64)
    img = np.ascontiguousarray(img, np.float64).reshape(3, active.size)
    out = np.empty((3, H, W), np.float64)
    ok = np.empty((H, W), np.int32)
    t, fx, fy = _cam_args(cam)
    lib().or_sphere_to_image(int(cam["order"]), _p(_ring2nest(cam["order"])), C.c_int64(active.size), _p(active),
                             _p(img), t, int(W), int(H), C.c_double(fx), C.c_double(fy), _p(out), _p(ok))
    return out, ok.astype(bool)


def image_to_sphere(cam: dict, active, img, W: int, H: int) -> tuple:
    """Samples [3][n_active] of the camera image img [3][H][W] at the active
    HEALPix pixel centres (supp. Eq. supp_image_to_healpix) and validity."""
    active = np.ascontiguousarray(active, np.int64)
    img = np.ascontiguousarray(img, np.float64).reshape(3, H, W)
    out = np.empty((3, active.size), np.float64)
    ok = np.empty(active.size, np.int32)
    t, fx, fy = _cam_args(cam)
    lib().or_image_to_sphere(int(cam["order"]), C.c_int64(active.size), _p(active), _p(img), t, int(W), int(H),
                             C.c_double(fx), C.c_double(fy), _p(out), _p(ok))
    return out, ok.astype(bool)


def density_stats(rs, visible, g_ang, phi, rs_max, grad_accum, count):
    """Radian-space statistics for adaptive density control (Sec. 4.2): for
    every Gaussian visible in the view (in at least one tile), r_s,max <-
    max(r_s,max, r_s), the norm of the gradient with respect to the centre's
    displacement along the sphere (east = d omega cos phi, north = d phi),
    |(dL/domega / cos phi, dL/dphi)|, is added to grad_accum and count is
    incremented.  Returns new arrays."""
    rs = np.asarray(rs, np.float64); vis = np.asarray(visible, bool)
    g = np.asarray(g_ang, np.float64); phi = np.asarray(phi, np.float64)
    rs_max = np.where(vis, np.maximum(rs_max, rs), rs_max)
    norm = np.hypot(g[0] / np.cos(phi), g[1])
    grad_accum = np.where(vis, grad_accum + norm, grad_accum)
    count = np.where(vis, count + 1, count)
    return rs_max, grad_accum, count
