"""Binning and sorting with counts that stay on the device (Alg. 1 stage 2:
QueryDisc, sort, ranges): the stable tile sort against numpy's stable sort at
sizes around the 4096-element tiles; a list buffer too small for the pairs
(nothing emitted, every range empty, the synchronous check reports
HP_ERR_CAPACITY, a rerun with the reported count matches the reference);
the Python layer's capacity hints; and a scene whose tasks exceed the
workspace, including a task total beyond 2^32."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_29794_amd import _abi as A
from paper_2606_29794_amd import scenes as SC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_2606_29794_amd import raster
    assert torch.cuda.is_available()
    return raster.Rasterizer()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("n,cap,n_tiles", [(0, 10, 5), (1, 1, 3), (4095, 5000, 300), (4096, 4096, 300),
                                           (4097, 9000, 300), (300_001, 400_000, 70_000), (250_000, 250_000, 12),
                                           # 1024 workgroups of several 1024-key tiles each, 3 passes
                                           (2_500_000, 3_000_000, 70_000)])
def test_sort_matches_stable_numpy_sort(R, n, cap, n_tiles):
    """hp_sort with the count in device memory and a buffer of `cap` pairs:
    keys, values (stable order) and ranges equal numpy's stable argsort."""
    import torch
    print("hp_sort n", n, "cap", cap, "tiles", n_tiles, flush=True)
    rng = np.random.default_rng(n + cap)
    keys = rng.integers(0, n_tiles, size=cap).astype(np.uint32)
    vals = rng.integers(0, 1 << 31, size=cap).astype(np.uint32)
    kd = torch.as_tensor(keys.view(np.int32), device="cuda")
    vd = torch.as_tensor(vals.view(np.int32), device="cuda")
    ranges = R.sort(kd, vd, torch.tensor([n], dtype=torch.int64, device="cuda"), n_tiles)
    torch.cuda.synchronize()
    o = np.argsort(keys[:n], kind="stable")
    assert np.array_equal(kd.cpu().numpy().view(np.uint32)[:n], keys[:n][o])
    assert np.array_equal(vd.cpu().numpy().view(np.uint32)[:n], vals[:n][o])
    # entries past the count are untouched
    assert np.array_equal(vd.cpu().numpy().view(np.uint32)[n:], vals[n:])
    r = ranges.cpu().numpy().astype(np.int64)[:n_tiles]
    cnt = np.bincount(keys[:n], minlength=n_tiles)
    assert np.array_equal(r[:, 1] - r[:, 0], cnt)
    nz = cnt > 0
    assert np.array_equal(r[nz, 0], np.searchsorted(keys[:n][o], np.arange(n_tiles)[nz]))


def test_sort_count_beyond_capacity_sorts_nothing(R):
    import torch
    keys = torch.arange(100, 0, -1, dtype=torch.int32, device="cuda")
    vals = torch.arange(100, dtype=torch.int32, device="cuda")
    k0, v0 = keys.clone(), vals.clone()
    ranges = R.sort(keys, vals, torch.tensor([101], dtype=torch.int64, device="cuda"), 128)
    torch.cuda.synchronize()
    assert torch.equal(keys, k0) and torch.equal(vals, v0)
    assert int(ranges.abs().sum()) == 0


def _cfg(P=20000, order=7):
    from paper_2606_29794_amd.raster import Camera, Gaussians
    wl = SC.config1(P=P, order=order)
    return Gaussians.from_scene(wl.scene), Camera.from_dict(wl.cameras[0])


def test_small_list_buffer_emits_nothing_then_rerun_matches(R):
    """HP_BIN_ALL with a capacity below the pair count: no pair is written,
    every tile range is (0, 0), hp_check_count returns HP_ERR_CAPACITY with
    the needed count, and a second call with that capacity reproduces the
    lists of the synchronous path."""
    import torch
    from paper_2606_29794_amd.raster import _p
    g, cam = _cfg()
    proj = R.preprocess(g, cam)
    vals_ref, ranges_ref, n = R.bin_sorted(proj, g.P, cam)
    assert n > 100
    m = R.mask(cam)
    ws_n = A.lib().hp_bin_sorted_workspace_bytes(g.P, cam.order, R.prm.tile_log2)
    ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = n // 2
    vals = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    ranges = torch.full((m.n_tiles, 2), 123, dtype=torch.int32, device="cuda")
    v = cam.view()
    args = lambda vv, rr, c: (A.HP_BIN_ALL, _p(proj), g.P, C.byref(v), C.byref(R.prm), _p(R.grid(cam.order)),
                              _p(m.buf), _p(vv), _p(rr), m.n_tiles, c, _p(cnt), _p(ws), ws_n, _stream())
    A.call("hp_bin_sorted", *args(vals, ranges, cap))
    got = C.c_int64(0)
    st = A.lib().hp_check_count(_p(cnt), cap, C.byref(got), _stream())
    assert st == A.HP_ERR_CAPACITY and got.value == n
    assert int((vals != -7).sum()) == 0
    assert int(ranges.abs().sum()) == 0
    vals2 = torch.empty(got.value, dtype=torch.int32, device="cuda")
    A.call("hp_bin_sorted", *args(vals2, ranges, got.value))
    assert A.lib().hp_check_count(_p(cnt), got.value, None, _stream()) == A.HP_OK
    torch.cuda.synchronize()
    assert torch.equal(vals2[:n], vals_ref[:n]) and torch.equal(ranges, ranges_ref)


def test_capacity_hints_and_verify(R):
    """The Python layer: a binning whose hint is too small leaves its lists
    empty and verify() raises; the hint then covers the count and the repeat
    equals the reference."""
    import torch
    from paper_2606_29794_amd.raster import PairCapacityError
    g, cam = _cfg(P=15000, order=6)
    proj = R.preprocess(g, cam)
    vals_ref, ranges_ref, n = R.bin_sorted(proj, g.P, cam)
    key = R._bin_key(g.P, cam, None)
    R._cap_hint[key] = n // 3
    vals, ranges, cnt = R.bin_lists(proj, g.P, cam)
    with pytest.raises(PairCapacityError):
        R.verify()
    assert cnt.overflowed and int(ranges.abs().sum()) == 0
    assert R._cap_hint[key] >= n
    vals, ranges, cnt = R.bin_lists(proj, g.P, cam)
    R.verify()
    assert cnt.value(0) == n
    assert torch.equal(vals[:n], vals_ref[:n]) and torch.equal(ranges, ranges_ref)
    # without waiting: an overflow is reported once its binning has finished
    R._cap_hint[key] = n // 3
    R.bin_lists(proj, g.P, cam)
    torch.cuda.synchronize()
    with pytest.raises(PairCapacityError):
        R.verify(block=False)
    R.verify()


def _whole_sphere_scene(P):
    """P Gaussians much larger than their distance to the camera: every one
    covers the whole sphere (r_s = pi)."""
    rng = np.random.default_rng(5)
    d = rng.normal(size=(3, P))
    d /= np.linalg.norm(d, axis=0)
    mean = (2.0 * d).astype(np.float32)
    scale = np.full((3, P), 50.0, np.float32)
    rot = np.zeros((4, P), np.float32)
    rot[0] = 1
    opac = np.full(P, 0.5, np.float32)
    sh = np.zeros((1, 3, P), np.float32)
    return mean, scale, rot, opac, sh


@pytest.mark.parametrize("P", [100, 360_000])
def test_task_overflow_reports_capacity(R, P):
    """At order 12 a whole-sphere Gaussian makes one task per quadtree node
    of level 5 (12,288).  100 of them exceed the task capacity 16 P + 2^20;
    360,000 of them make 4.4e9 tasks, past 2^32 (the task offsets are 64-bit,
    so the total cannot wrap below the capacity).  The count reports
    INT64_MAX, hp_check_count HP_ERR_CAPACITY, nothing is emitted and every
    range is empty."""
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, _p
    print("task overflow P", P, flush=True)
    mean, scale, rot, opac, sh = _whole_sphere_scene(P)
    t = lambda a: torch.as_tensor(a, device="cuda")
    g = Gaussians(t(mean), t(scale), t(rot), t(opac), t(sh))
    cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), np.zeros(3, np.float32), A.HP_CAM_FULL,
                 2 * np.pi, np.pi, 12)
    proj = R.preprocess(g, cam)
    rad = R.projected_arrays(proj, P)[2]
    assert float(rad.min()) >= 3.14
    m = R.mask(cam)
    ws_n = A.lib().hp_bin_sorted_workspace_bytes(P, 12, R.prm.tile_log2)
    ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = 1 << 20
    vals = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    ranges = torch.full((m.n_tiles, 2), 9, dtype=torch.int32, device="cuda")
    v = cam.view()
    A.call("hp_bin_sorted", A.HP_BIN_ALL, _p(proj), P, C.byref(v), C.byref(R.prm), _p(R.grid(12)), _p(m.buf),
           _p(vals), _p(ranges), m.n_tiles, cap, _p(cnt), _p(ws), ws_n, _stream())
    got = C.c_int64(0)
    assert A.lib().hp_check_count(_p(cnt), cap, C.byref(got), _stream()) == A.HP_ERR_CAPACITY
    assert got.value == np.iinfo(np.int64).max
    assert int((vals != -7).sum()) == 0 and int(ranges.abs().sum()) == 0
