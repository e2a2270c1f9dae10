"""Host-side driver of the HEALPix rasterizer: device buffers come from
PyTorch's caching allocator, every computation is a call into libhp.so on the
current HIP stream (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import math
import threading
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A


def _p(t):
    """Pointer argument for a call into the library.  The returned object keeps
    `t` alive, so a temporary (x.contiguous() of a strided tensor) is not
    returned to the caching allocator, and handed to the next temporary of the
    same call, before the call has enqueued its kernels."""
    if t is None:
        return None
    v = C.c_void_p(t.data_ptr())
    v._keep = t
    return v


def _dense(t):
    """A float32 contiguous device tensor for a kernel argument (a copy if t is
    strided); anything else is refused rather than reinterpreted."""
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float32:
        raise ValueError("expected a float32 device tensor")
    return t.contiguous()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _bytes(n, device):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


@dataclass
class Camera:
    """World->camera rotation W (row-major 3x3), translation b = -W center,
    camera type (A.HP_CAM_*), field of view (radians) and HEALPix order."""
    W: np.ndarray
    b: np.ndarray
    center: np.ndarray
    cam_type: int = A.HP_CAM_FULL
    fov_x: float = 2 * math.pi
    fov_y: float = math.pi
    order: int = 9

    @staticmethod
    def from_dict(d: dict) -> "Camera":
        return Camera(np.asarray(d["W"], np.float32), np.asarray(d["b"], np.float32),
                      np.asarray(d["center"], np.float32), int(d["cam_type"]), float(d["fov_x"]),
                      float(d["fov_y"]), int(d["order"]))

    def view(self) -> A.hp_view:
        return A.make_view(self.W, self.b, self.center, self.cam_type, self.fov_x, self.fov_y, self.order)

    def mask_key(self, tile_log2: int):
        if self.cam_type == A.HP_CAM_FULL:
            return (self.order, 0, 0.0, 0.0, tile_log2)
        return (self.order, self.cam_type, float(np.float32(self.fov_x)), float(np.float32(self.fov_y)), tile_log2)


@dataclass
class Gaussians:
    """Device tensors, float32, contiguous: mean [3,P], scale [3,P] (>0),
    rot [4,P] (w,x,y,z), opacity [P] in (0,1), sh [K,3,P]."""
    mean: torch.Tensor
    scale: torch.Tensor
    rot: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor

    @property
    def P(self) -> int:
        return int(self.mean.shape[1])

    @property
    def sh_degree(self) -> int:
        return int(round(math.sqrt(self.sh.shape[0]))) - 1

    @staticmethod
    def from_scene(scene, device="cuda") -> "Gaussians":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)
        return Gaussians(t(scene.mean), t(scene.scale), t(scene.rot), t(scene.opacity), t(scene.sh))

    def struct(self) -> A.hp_gaussians:
        for x in (self.mean, self.scale, self.rot, self.opacity, self.sh):
            if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
                raise ValueError("Gaussian tensors must be contiguous float32 device tensors")
        return A.hp_gaussians(self.P, self.sh_degree, self.mean.data_ptr(), self.scale.data_ptr(),
                              self.rot.data_ptr(), self.opacity.data_ptr(), self.sh.data_ptr())


def check_mask_counts(order: int, tile_log2: int, n_active: int, n_tiles: int) -> None:
    """The header a mask computation left behind must describe a subset of
    the grid: 0 <= n_active <= Npix, 0 <= n_tiles <= the tile count, every
    active tile holding at least one and at most B^2 active pixels.  Buffers
    are sized from these numbers, so anything else (a mask read before its
    computation completed, a corrupted buffer) is refused here."""
    b = min(tile_log2, order)
    npix = 12 << (2 * order)
    ntile = 12 << (2 * (order - b))
    if not (0 <= n_active <= npix and 0 <= n_tiles <= ntile):
        raise RuntimeError(f"inconsistent mask header: n_active {n_active}, n_tiles {n_tiles} at order {order}")
    if not (n_tiles <= n_active <= n_tiles << (2 * b)):
        raise RuntimeError(f"inconsistent mask header: {n_active} active pixels in {n_tiles} tiles of {1 << (2 * b)}")


@dataclass
class MaskInfo:
    buf: torch.Tensor
    n_active: int
    n_tiles: int
    active_pix: torch.Tensor   # int32 [n_active], sorted nested ids


class PairCapacityError(RuntimeError):
    """A binning wanted more list entries than the buffer it was given held:
    its lists were left empty.  The capacity hints have been raised, so the
    same work run again fits."""


class PairCount:
    """The pair count of one binning as the device wrote it (int64 [2]: the
    entries the lists need, and the entries kept by a paper query, defined
    for a query only), with the
    capacity of the list buffer it was emitted into.  Reading it waits for
    the binning; nothing on the render path reads it."""

    def __init__(self, dev: torch.Tensor, capacity: int):
        self.dev = dev
        self.capacity = int(capacity)
        self._host = None

    def value(self, which: int = 0) -> int:
        if self._host is None:
            self._host = self.dev.cpu().tolist()
        return int(self._host[which])

    @property
    def overflowed(self) -> bool:
        return self.value(0) > self.capacity


@dataclass
class FwdState:
    """What the backward pass needs from a forward render: no per-Gaussian
    forward state beyond the projected records."""
    camera: Camera
    mask: MaskInfo
    projected: torch.Tensor
    vals: torch.Tensor
    ranges: torch.Tensor
    count: PairCount
    rgb: torch.Tensor
    T: torch.Tensor
    n_contrib: torch.Tensor
    P: int
    inv_depth: torch.Tensor | None = None

    @property
    def n_pairs(self) -> int:
        """List entries (waits for the binning)."""
        return self.count.value(0)


@dataclass
class Prepared:
    """Stages 1-2 of one view (projected records and tile lists), made on
    the stream `stream_id`; `event` marks their completion there."""
    camera: Camera
    projected: torch.Tensor
    vals: torch.Tensor
    ranges: torch.Tensor
    count: PairCount
    event: torch.cuda.Event
    stream_id: int


class Prefetch:
    """Stages 1-2 of a sequence of views, enqueued at once on side streams
    (view i on stream i mod n), so that they overlap the caller's rendering
    of the views before them.  Nothing in them waits for the host.  get(i)
    returns view i."""

    def __init__(self, R: "Rasterizer", g: "Gaussians", cams, query=None, streams: int = 2):
        n = max(1, min(streams, len(cams)))
        side = R.side_streams(n)
        # the side streams first wait for the work the caller queued so far
        # (e.g. an update of the Gaussians)
        start = torch.cuda.Event()
        start.record(torch.cuda.current_stream(R.device))
        for st in side:
            st.wait_event(start)
        self._views = []
        for i, cam in enumerate(cams):
            with torch.cuda.stream(side[i % n]):
                self._views.append(R.prepare(g, cam, query))

    def get(self, i: int) -> Prepared:
        return self._views[i]


class Rasterizer:
    """Grid tables per HEALPix order and masks per camera model are built once
    and cached; everything else is per call."""

    def __init__(self, device="cuda", **params):
        self.device = torch.device(device)
        self.prm = A.default_params(**params)
        self._grids = {}
        self._masks = {}
        # cached tables are written on the stream current at creation; a
        # later user on another stream waits for this event first
        self._ready = {}
        # the caches may be used from several host threads (serving workers)
        self._lock = threading.RLock()
        self._sides = []
        # list capacities per (P, camera model, order, query) from earlier
        # counts; per (P, order, camera type, query) the largest count per
        # active tile seen, which sizes the lists of a camera model not seen
        # before (a new field of view) without a count read-back; and the
        # counts not yet compared with their capacity
        self._cap_hint = {}
        self._tile_ratio = {}
        self._pending = []
        self._overflows = []
        # one binning workspace per stream (work on a stream is ordered, so
        # the next binning there may reuse it)
        self._ws = {}
        # HSSIM patch tables per camera model (hp_ssim_tables)
        self._ssim_tables = {}

    def side_streams(self, n: int) -> list:
        """The first n streams of prefetch() (default priority), created once."""
        with self._lock:
            while len(self._sides) < n:
                self._sides.append(torch.cuda.Stream(device=self.device))
            return self._sides[:n]

    def prefetch(self, g: "Gaussians", cams, query=None, streams: int = 2) -> Prefetch:
        """Enqueue stages 1-2 of every camera in `cams` on up to `streams` side
        streams (with the caller's stream, 4: the hardware queues a process
        gets by default); pass prefetch.get(i) as forward(..., prepared=) /
        render(..., prepared=)."""
        return Prefetch(self, g, cams, query, streams)

    # camera models kept (masks and HSSIM tables): a serving trace with a
    # field of view per request would otherwise grow the caches without end
    CACHE_MODELS = 256

    def _evict(self, cache: dict, ready_prefix) -> None:
        """Drops the oldest entries of a per-camera-model cache beyond
        CACHE_MODELS (and their ready events).  Work in flight keeps its own
        references to the tensors.  Lock held."""
        while len(cache) > self.CACHE_MODELS:
            old = next(iter(cache))
            del cache[old]
            if ready_prefix is not None:
                self._ready.pop(ready_prefix + old, None)

    def _created(self, key):
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        self._ready[key] = (ev, torch.cuda.current_stream(self.device).cuda_stream)

    def _await(self, key):
        ev, sid = self._ready[key]
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != sid:
            cur.wait_event(ev)

    # ---- camera-independent tables ------------------------------------
    def grid(self, order: int) -> torch.Tensor:
        with self._lock:
            return self._grid(order)

    def _grid(self, order: int) -> torch.Tensor:
        key = (order, self.prm.tile_log2)
        g = self._grids.get(key)
        if g is None:
            n = A.lib().hp_grid_bytes(order, self.prm.tile_log2)
            if n == 0:
                raise ValueError(f"unsupported order {order}")
            g = _bytes(n, self.device)
            A.call("hp_grid_init", order, C.byref(self.prm), _p(g), n, _stream())
            self._grids[key] = g
            self._created(("grid",) + key)
        else:
            self._await(("grid",) + key)
        return g

    def mask(self, cam: Camera) -> MaskInfo:
        with self._lock:
            return self._mask(cam)

    def _mask(self, cam: Camera) -> MaskInfo:
        key = cam.mask_key(self.prm.tile_log2)
        m = self._masks.get(key)
        if m is None:
            n = A.lib().hp_mask_bytes(cam.order, self.prm.tile_log2)
            buf = _bytes(n, self.device)
            v = cam.view()
            A.call("hp_mask", C.byref(v), C.byref(self.prm), _p(self.grid(cam.order)), _p(buf), n, _stream())
            na, nt = C.c_int64(0), C.c_int32(0)
            A.call("hp_mask_counts", _p(buf), cam.order, self.prm.tile_log2, C.byref(na), C.byref(nt), _stream())
            check_mask_counts(cam.order, self.prm.tile_log2, int(na.value), int(nt.value))
            ptr = A.lib().hp_mask_active_pix(_p(buf), cam.order, self.prm.tile_log2)
            off = ptr - buf.data_ptr()
            ap = buf[off: off + 4 * na.value].view(torch.int32)
            m = MaskInfo(buf, int(na.value), int(nt.value), ap)
            self._masks[key] = m
            self._evict(self._masks, ("mask",))
            self._created(("mask",) + key)
        else:
            self._await(("mask",) + key)
        return m

    # ---- stage 1 ---------------------------------------------------------
    def preprocess(self, g: Gaussians, cam: Camera) -> torch.Tensor:
        n = A.lib().hp_projected_bytes(g.P)
        proj = _bytes(n, self.device)
        gs = g.struct()
        v = cam.view()
        A.call("hp_preprocess", C.byref(gs), C.byref(v), C.byref(self.prm), _p(proj), n, _stream())
        return proj

    def projected_arrays(self, proj: torch.Tensor, P: int):
        """Views of a projected buffer: rec [P,16], depth [P], radius [P]."""
        rec = proj[: P * 64].view(torch.float32).view(P, 16)
        dptr = A.lib().hp_projected_depth(_p(proj), P) - proj.data_ptr()
        rptr = A.lib().hp_projected_radius(_p(proj), P) - proj.data_ptr()
        depth = proj[dptr: dptr + 4 * P].view(torch.float32)
        radius = proj[rptr: rptr + 4 * P].view(torch.float32)
        return rec, depth, radius

    # ---- stage 2 ---------------------------------------------------------
    def workspace(self, nbytes: int) -> torch.Tensor:
        """A scratch buffer of at least nbytes for work on the current stream
        (kept per stream and reused by the next call there)."""
        sid = torch.cuda.current_stream(self.device).cuda_stream
        with self._lock:
            ws = self._ws.get(sid)
            if ws is None or ws.numel() < nbytes:
                ws = _bytes(nbytes, self.device)
                self._ws[sid] = ws
            return ws

    def _bin_key(self, P: int, cam: Camera, query):
        return (P, cam.mask_key(self.prm.tile_log2), query)

    @staticmethod
    def _ratio_key(P: int, cam: Camera, query):
        return (P, cam.order, cam.cam_type, query)

    @staticmethod
    def _grow(n: int) -> int:
        return int(n * 1.25) + 65536

    def capacity_hint(self, P: int, cam: Camera, query, n_tiles: int):
        """List capacity for a binning of this view: the hint of its camera
        model, else the largest count per active tile seen for its order and
        camera type times its n_tiles (grown like a hint), else None (the
        count has to be read back).  Called with the lock held or not."""
        with self._lock:
            cap = self._cap_hint.get(self._bin_key(P, cam, query))
            if cap is not None:
                return cap
            r = self._tile_ratio.get(self._ratio_key(P, cam, query))
        return None if r is None else self._grow(int(math.ceil(r * max(n_tiles, 1))))

    def _note(self, key, rkey, n: int, n_tiles: int) -> None:
        """A count seen: the hints grow to cover it.  Lock held."""
        self._cap_hint[key] = max(self._cap_hint.get(key, 0), self._grow(n))
        self._tile_ratio[rkey] = max(self._tile_ratio.get(rkey, 0.0), n / max(n_tiles, 1))

    def _bin_call(self, phase, proj, P, cam, query, vals, ranges, cap, cnt, ws):
        m = self.mask(cam)
        v = cam.view()
        grid = self.grid(cam.order)
        if query is None:
            A.call("hp_bin_sorted", phase, _p(proj), P, C.byref(v), C.byref(self.prm), _p(grid), _p(m.buf), _p(vals),
                   _p(ranges), m.n_tiles, cap, _p(cnt), _p(ws), ws.numel(), _stream())
        else:
            code = {"ring": A.HP_QUERY_RING, "nested": A.HP_QUERY_NESTED}[query[0]]
            A.call("hp_bin_query", phase, code, int(query[1]), _p(proj), P, C.byref(v), C.byref(self.prm), _p(grid),
                   _p(m.buf), _p(vals), _p(ranges), m.n_tiles, cap, _p(cnt), C.c_void_p(cnt.data_ptr() + 8), _p(ws),
                   ws.numel(), _stream())

    def note_count(self, P: int, cam: Camera, query, n: int) -> None:
        """Raise the list capacity hints of (P, camera model, query) and of its
        order and camera type to cover a count of n entries."""
        n_tiles = self.mask(cam).n_tiles
        with self._lock:
            self._note(self._bin_key(P, cam, query), self._ratio_key(P, cam, query), n, n_tiles)

    def bin_lists(self, proj: torch.Tensor, P: int, cam: Camera, query=None, track: bool = True):
        """Tile lists of one view, in per-tile depth order: (vals, ranges,
        PairCount).  query None: hp_bin_sorted's exact tile sets; (mode, f):
        the paper's own query (mode "ring": Alg. 3 RING scan, "nested": Alg. 2
        quadtree traversal) at search depth f, whose lists hold stale entries
        past each tile's end.  The list buffer's capacity comes from earlier
        counts of the same scene size, camera model and query; without one,
        the count is read back once (the only wait).  A count beyond the
        capacity leaves the lists empty and is reported by verify() (track
        False: the caller checks the returned PairCount itself)."""
        m = self.mask(cam)
        key, rkey = self._bin_key(P, cam, query), self._ratio_key(P, cam, query)
        nbytes = (A.lib().hp_bin_sorted_workspace_bytes(P, cam.order, self.prm.tile_log2) if query is None else
                  A.lib().hp_bin_query_workspace_bytes(P, cam.order, self.prm.tile_log2))
        ws = self.workspace(nbytes)
        # the list count (written by every binning) and, for a paper query,
        # the entries kept (zero until its emission writes it)
        cnt = (torch.empty if query is None else torch.zeros)(2, dtype=torch.int64, device=self.device)
        ranges = torch.empty((max(m.n_tiles, 1), 2), dtype=torch.int32, device=self.device)
        cap = self.capacity_hint(P, cam, query, m.n_tiles)
        if cap is None:
            self._bin_call(A.HP_BIN_COUNT, proj, P, cam, query, None, None, 0, cnt, ws)
            n = C.c_int64(0)
            A.call("hp_read_total", _p(cnt), C.byref(n), _stream())
            cap = max(int(n.value), 1)
            with self._lock:
                self._note(key, rkey, cap, m.n_tiles)
            vals = torch.empty(cap, dtype=torch.int32, device=self.device)
            self._bin_call(A.HP_BIN_EMIT, proj, P, cam, query, vals, ranges, cap, cnt, ws)
            return vals, ranges, PairCount(cnt, cap)
        vals = torch.empty(cap, dtype=torch.int32, device=self.device)
        self._bin_call(A.HP_BIN_ALL, proj, P, cam, query, vals, ranges, cap, cnt, ws)
        if not track:
            return vals, ranges, PairCount(cnt, cap)
        # compared with the capacity later, without waiting now
        host = torch.empty(2, dtype=torch.int64, pin_memory=True)
        host.copy_(cnt, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        with self._lock:
            self._pending.append((key, rkey, m.n_tiles, host, ev, cap))
            if len(self._pending) > 64:
                self._settle(block=False)
        return vals, ranges, PairCount(cnt, cap)

    def _settle(self, block: bool) -> None:
        """Compares the counts of finished binnings with their capacities
        (all of them, waiting, when block): hints grow, overflows are kept
        for verify().  Called with the lock held."""
        keep = []
        for item in self._pending:
            key, rkey, n_tiles, host, ev, cap = item
            if block:
                ev.synchronize()
            elif not ev.query():
                keep.append(item)
                continue
            n = int(host[0])
            self._note(key, rkey, n, n_tiles)
            if n > cap:
                self._overflows.append((key, n, cap))
        self._pending = keep

    def verify(self, block: bool = True) -> None:
        """Waits for the binnings since the last verify() (block False: takes
        only those already finished) and compares their counts with the
        capacities they ran with; raises PairCapacityError if any list buffer
        was too small (its lists were left empty).  The capacity hints grow
        from every count seen, so a repeat fits."""
        with self._lock:
            self._settle(block=block)
            over, self._overflows = self._overflows, []
        if over:
            raise PairCapacityError(f"{len(over)} binning(s) needed more list entries than their buffers held "
                                    f"(needed, capacity): {[(n, c) for _, n, c in over]}")

    def bin(self, proj: torch.Tensor, P: int, cam: Camera):
        """Unsorted pairs of hp_bin (synchronous convenience: the count is
        read back): (keys, vals, n)."""
        m = self.mask(cam)
        v = cam.view()
        ws_n = A.lib().hp_bin_workspace_bytes(P)
        ws = _bytes(ws_n, self.device)
        npairs = torch.zeros(1, dtype=torch.int64, device=self.device)
        A.call("hp_bin", A.HP_BIN_COUNT, _p(proj), P, C.byref(v), C.byref(self.prm), _p(self.grid(cam.order)),
               _p(m.buf), None, None, 0, _p(npairs), _p(ws), ws_n, _stream())
        total = C.c_int64(0)
        A.call("hp_check_count", _p(npairs), 1 << 40, C.byref(total), _stream())
        n = int(total.value)
        keys = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        vals = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        A.call("hp_bin", A.HP_BIN_EMIT, _p(proj), P, C.byref(v), C.byref(self.prm), _p(self.grid(cam.order)),
               _p(m.buf), _p(keys), _p(vals), n, _p(npairs), _p(ws), ws_n, _stream())
        return keys, vals, n

    def bin_sorted(self, proj: torch.Tensor, P: int, cam: Camera):
        """Pairs emitted directly in per-tile depth order (synchronous
        convenience: waits for the count): (vals, ranges, n)."""
        vals, ranges, cnt = self.bin_lists(proj, P, cam)
        return vals, ranges, cnt.value(0)

    def bin_query(self, proj: torch.Tensor, P: int, cam: Camera, mode: str, f: int):
        """Tile lists of the paper's own queries (mode "ring": Alg. 3 RING scan,
        "nested": Alg. 2 quadtree traversal) at search depth f, in per-tile
        depth order (synchronous convenience): (vals, ranges, n_candidates,
        n_kept).  A tile's list is vals[ranges[k, 0]:ranges[k, 1]]; entries
        past a tile's end are stale."""
        vals, ranges, cnt = self.bin_lists(proj, P, cam, (mode, int(f)))
        return vals, ranges, cnt.value(0), cnt.value(1)

    def sort(self, keys, vals, n, n_tiles: int):
        """Stable tile sort of hp_bin's pairs; n: host count or device int64."""
        ranges = torch.zeros((max(n_tiles, 1), 2), dtype=torch.int32, device=self.device)
        cap = int(keys.numel())
        n_dev = n if isinstance(n, torch.Tensor) else torch.tensor([int(n)], dtype=torch.int64, device=self.device)
        ws_n = A.lib().hp_sort_workspace_bytes(cap, n_tiles)
        ws = _bytes(ws_n, self.device)
        A.call("hp_sort", _p(keys), _p(vals), _p(n_dev), cap, n_tiles, _p(ranges), _p(ws), ws_n, _stream())
        return ranges

    # ---- stage 3 ---------------------------------------------------------
    def render_fwd(self, proj, P, vals, ranges, cam: Camera, want_used: bool = False, want_depth: bool = False):
        """rgb [3, n], T [n], n_contrib [n] (and n_used [n] if want_used, and
        the composited inverse radial depth [n] last if want_depth)."""
        m = self.mask(cam)
        v = cam.view()
        rgb = torch.empty((3, max(m.n_active, 1)), dtype=torch.float32, device=self.device)
        T = torch.empty(max(m.n_active, 1), dtype=torch.float32, device=self.device)
        nc = torch.empty(max(m.n_active, 1), dtype=torch.int32, device=self.device)
        nu = torch.empty(max(m.n_active, 1), dtype=torch.int32, device=self.device) if want_used else None
        dinv = torch.empty(max(m.n_active, 1), dtype=torch.float32, device=self.device) if want_depth else None
        A.call("hp_render_fwd", _p(proj), P, _p(vals), _p(ranges), m.n_tiles, C.byref(v), C.byref(self.prm),
               _p(m.buf), m.n_active, _p(rgb), _p(T), _p(nc), _p(nu), _p(dinv), _stream())
        out = (rgb, T, nc) + ((nu,) if want_used else ()) + ((dinv,) if want_depth else ())
        return out

    def prepare(self, g: Gaussians, cam: Camera, query=None) -> Prepared:
        """Stages 1-2 for one view on the current stream.  query: None for the
        binning of hp_bin_sorted, or (mode, f) for the paper's own tile query
        (bin_query)."""
        self.mask(cam)
        proj = self.preprocess(g, cam)
        vals, ranges, cnt = self.bin_lists(proj, g.P, cam, None if query is None else (query[0], int(query[1])))
        cur = torch.cuda.current_stream(self.device)
        ev = torch.cuda.Event()
        ev.record(cur)
        return Prepared(cam, proj, vals, ranges, cnt, ev, cur.cuda_stream)

    def forward(self, g: Gaussians, cam: Camera, want_depth: bool = False, query=None,
                prepared: Prepared | None = None) -> FwdState:
        """Stages 1-3 for one view (query as for prepare()).  With `prepared`
        (from prepare() or prefetch() for the same Gaussians and camera),
        stages 1-2 are taken from it: the current stream waits for them."""
        m = self.mask(cam)
        if prepared is None:
            prepared = self.prepare(g, cam, query)
        else:
            cur = torch.cuda.current_stream(self.device)
            if cur.cuda_stream != prepared.stream_id:
                cur.wait_event(prepared.event)
                # made on another stream, used (and freed) on this one
                for t in (prepared.projected, prepared.vals, prepared.ranges, prepared.count.dev):
                    t.record_stream(cur)
        proj, vals, ranges, cnt = prepared.projected, prepared.vals, prepared.ranges, prepared.count
        out = self.render_fwd(proj, g.P, vals, ranges, cam, want_depth=want_depth)
        rgb, T, nc = out[:3]
        return FwdState(cam, m, proj, vals, ranges, cnt, rgb, T, nc, g.P, out[3] if want_depth else None)

    def backward(self, g: Gaussians, st: FwdState, dL_drgb, dL_dT, grads: Gaussians, dL_dinv_depth=None) -> None:
        """Accumulates gradients into the tensors of `grads`."""
        v = st.camera.view()
        gs = g.struct()
        gg = A.hp_gaussians_grad(grads.mean.data_ptr(), grads.scale.data_ptr(), grads.rot.data_ptr(),
                                 grads.opacity.data_ptr(), grads.sh.data_ptr())
        ws_n = A.lib().hp_render_bwd_workspace_bytes(g.P)
        ws = _bytes(ws_n, self.device)
        A.call("hp_render_bwd", C.byref(gs), _p(st.projected), _p(st.vals), _p(st.ranges), st.mask.n_tiles,
               C.byref(v), C.byref(self.prm), _p(st.mask.buf), st.mask.n_active, _p(st.T), _p(st.n_contrib),
               _p(dL_drgb.contiguous()), _p(None if dL_dT is None else dL_dT.contiguous()),
               _p(None if dL_dinv_depth is None else dL_dinv_depth.contiguous()), C.byref(gg), _p(ws), ws_n, _stream())

    def backward_pixels(self, st: FwdState, dL_drgb, dL_dT, acc: torch.Tensor, dL_dinv_depth=None) -> None:
        """Pixel pass of the backward alone: per-Gaussian dL/d(colour,
        opacity, conic, omega, phi[, 1/r]) accumulated into acc [10, P]."""
        v = st.camera.view()
        A.call("hp_render_bwd_pixels", _p(st.projected), st.P, _p(st.vals), _p(st.ranges), st.mask.n_tiles,
               C.byref(v), C.byref(self.prm), _p(st.mask.buf), st.mask.n_active, _p(st.T), _p(st.n_contrib),
               _p(dL_drgb.contiguous()), _p(None if dL_dT is None else dL_dT.contiguous()),
               _p(None if dL_dinv_depth is None else dL_dinv_depth.contiguous()), _p(acc), _stream())

    def backward_preprocess(self, g: Gaussians, cam: Camera, acc: torch.Tensor, grads: Gaussians) -> None:
        """Second half of the backward: acc [10, P] -> parameter gradients (accumulated)."""
        v = cam.view()
        gs = g.struct()
        gg = A.hp_gaussians_grad(grads.mean.data_ptr(), grads.scale.data_ptr(), grads.rot.data_ptr(),
                                 grads.opacity.data_ptr(), grads.sh.data_ptr())
        A.call("hp_preprocess_bwd", C.byref(gs), C.byref(v), C.byref(self.prm), _p(acc), C.byref(gg), _stream())

    # ---- radian-space density-control statistics -----------------------------
    def density_stats(self, st: FwdState, acc: torch.Tensor, rs_max: torch.Tensor, grad_accum: torch.Tensor,
                      count: torch.Tensor) -> None:
        """Updates rs_max / grad_accum [P] float and count [P] int32 in place for
        the Gaussians visible in this view (in any tile list), from the pixel
        pass's accumulators acc [10, P]."""
        vis = torch.zeros(max(st.P, 1), dtype=torch.uint8, device=self.device)
        A.call("hp_mark_visible", _p(st.vals), _p(st.ranges), st.mask.n_tiles, st.P, _p(vis), _stream())
        A.call("hp_density_stats", _p(st.projected), st.P, _p(acc), _p(vis), _p(rs_max), _p(grad_accum), _p(count),
               _stream())

    # ---- image synthesis (Eq. camera_synthesis; supp. camera models) ----------
    def sphere_to_image(self, img: torch.Tensor, cam: Camera, W: int, H: int, want_valid: bool = False):
        """Camera image [3][H][W] from the HEALPix image img [3][n_active] of
        `cam` (Interp_H over ring neighbours, renormalised over the active
        set); with want_valid also the uint8 validity map [H][W]."""
        img = _dense(img)
        m = self.mask(cam)
        out = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        valid = torch.empty((H, W), dtype=torch.uint8, device=self.device) if want_valid else None
        v = cam.view()
        A.call("hp_sphere_to_image", _p(m.buf), C.byref(v), C.byref(self.prm), m.n_active,
               _p(img), int(W), int(H), _p(out), _p(valid), _stream())
        return (out, valid) if want_valid else out

    def image_to_sphere(self, img: torch.Tensor, cam: Camera, want_valid: bool = False):
        """Samples [3][n_active] of the camera image img [3][H][W] at the
        centres of cam's active HEALPix pixels (bilinear in the image)."""
        img = _dense(img)
        m = self.mask(cam)
        H, W = int(img.shape[1]), int(img.shape[2])
        out = torch.empty((3, max(m.n_active, 1)), dtype=torch.float32, device=self.device)[:, :m.n_active]
        valid = torch.empty(max(m.n_active, 1), dtype=torch.uint8, device=self.device)[:m.n_active] if want_valid else None
        v = cam.view()
        A.call("hp_image_to_sphere", _p(m.buf), C.byref(v), C.byref(self.prm), m.n_active,
               _p(img), W, H, _p(out), _p(valid), _stream())
        return (out, valid) if want_valid else out

    # ---- loss ----------------------------------------------------------------
    def ssim_tables(self, cam: Camera) -> torch.Tensor:
        """HSSIM patch tables of the camera model (built once, cached)."""
        with self._lock:
            key = cam.mask_key(self.prm.tile_log2)
            t = self._ssim_tables.get(key)
            if t is None:
                m = self._mask(cam)
                n = A.lib().hp_ssim_tables_bytes(cam.order, self.prm.tile_log2, m.n_tiles)
                t = _bytes(n, self.device)
                A.call("hp_ssim_tables", C.byref(self.prm), _p(m.buf), cam.order, m.n_active, m.n_tiles, _p(t), n,
                       _stream())
                self._ssim_tables[key] = t
                self._evict(self._ssim_tables, ("ssim_tables",))
                self._created(("ssim_tables",) + key)
            else:
                self._await(("ssim_tables",) + key)
            return t

    def ssim_loss(self, img, ref, cam: Camera, sp: A.hp_ssim_params | None = None, dL_dloss=None, want_map=False):
        """Returns (out[3] = (mean SSIM, L1, loss), ssim_map or None, dL/dimg or None)."""
        img, ref = _dense(img), _dense(ref)
        m = self.mask(cam)
        sp = sp or A.default_ssim_params()
        out = torch.empty(3, dtype=torch.float32, device=self.device)  # written whole by the call
        smap = torch.empty_like(img) if want_map else None
        dimg = torch.empty_like(img) if dL_dloss is not None else None
        ws_n = A.lib().hp_ssim_workspace_bytes(cam.order, self.prm.tile_log2, m.n_active)
        ws = _bytes(ws_n, self.device)
        tab = self.ssim_tables(cam)
        A.call("hp_ssim", _p(img), _p(ref), m.n_active, m.n_tiles, cam.order,
               C.byref(self.prm), C.byref(sp), _p(m.buf), _p(tab), _p(out), _p(smap), _p(dL_dloss), _p(dimg), _p(ws),
               ws_n, _stream())
        return out, smap, dimg

    def ssim_forward_saved(self, img, ref, cam: Camera, sp: A.hp_ssim_params | None = None, want_map=False):
        """Loss forward that keeps the backward's per-pixel partials: returns
        (out[3], ssim_map or None, saved workspace for ssim_backward_saved)."""
        img, ref = _dense(img), _dense(ref)
        m = self.mask(cam)
        sp = sp or A.default_ssim_params()
        out = torch.empty(3, dtype=torch.float32, device=self.device)  # written whole by the call
        smap = torch.empty_like(img) if want_map else None
        ws_n = A.lib().hp_ssim_workspace_bytes(cam.order, self.prm.tile_log2, m.n_active)
        ws = _bytes(ws_n, self.device)
        A.call("hp_ssim_forward_saved", _p(img), _p(ref), m.n_active, m.n_tiles, cam.order, C.byref(self.prm),
               C.byref(sp), _p(m.buf), _p(self.ssim_tables(cam)), _p(out), _p(smap), _p(ws), ws_n, _stream())
        return out, smap, ws

    def ssim_backward_saved(self, img, ref, cam: Camera, sp: A.hp_ssim_params, ws, dL_dloss):
        """dL/dimg from the partials a previous ssim_forward_saved left in ws."""
        img, ref, dL_dloss = _dense(img), _dense(ref), _dense(dL_dloss)
        m = self.mask(cam)
        dimg = torch.empty_like(img)
        A.call("hp_ssim_backward_saved", _p(img), _p(ref), m.n_active, m.n_tiles, cam.order, C.byref(self.prm),
               C.byref(sp), _p(m.buf), _p(self.ssim_tables(cam)), _p(ws), ws.numel(), _p(dL_dloss), _p(dimg),
               _stream())
        return dimg
