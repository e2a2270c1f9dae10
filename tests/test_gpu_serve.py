"""Continuous-batching server on the GPU: every request renders exactly the
same alone and inside a batch (the forward pass has no atomics), and a
sample is checked against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _trace(n, seed=77, orders=(6, 7, 8)):
    rng = np.random.default_rng(seed)
    cams = []
    for k in range(n):
        kind = k % 3
        order = int(orders[rng.integers(0, len(orders))])
        if kind == 0:
            fx = math.radians(rng.uniform(60, 90))
            cams.append(SC.make_camera(rng, order, SC.CAM_PINHOLE, fov_x=fx, fov_y=SC.pinhole_fov_y(fx), center_radius=0.5))
        elif kind == 1:
            f = math.radians(rng.uniform(180, 220))
            cams.append(SC.make_camera(rng, order, SC.CAM_FISHEYE, fov_x=f, fov_y=f, center_radius=0.5))
        else:
            cams.append(SC.make_camera(rng, order, SC.CAM_FULL, center_radius=0.5))
    arrivals = np.cumsum(rng.exponential(0.002, size=n))
    return cams, arrivals


def test_batched_preprocess_equals_single():
    import torch
    from paper_2606_29794_amd import _abi as A
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    import ctypes as C
    sc = SC.make_scene(50_000, 3, "log", 1.0, 20.0, seed=5)
    g = Gaussians.from_scene(sc)
    R = Rasterizer()
    cams, _ = _trace(5)
    singles = [R.preprocess(g, Camera.from_dict(c)) for c in cams]
    n = A.lib().hp_projected_bytes(g.P)
    outs = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in cams]
    views = (A.hp_view * len(cams))(*[Camera.from_dict(c).view() for c in cams])
    ptrs = (C.c_void_p * len(cams))(*[o.data_ptr() for o in outs])
    gs = g.struct()
    A.call("hp_preprocess_batch", C.byref(gs), len(cams), views, C.byref(R.prm), ptrs, n,
           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    for a, b in zip(singles, outs):
        # compare the records, depths and radii (not the alignment padding)
        for x, y in zip(R.projected_arrays(a, g.P), R.projected_arrays(b, g.P)):
            assert torch.equal(x, y)


def test_served_results_equal_solo_renders():
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    from paper_2606_29794_amd.serve import Request, Server
    sc = SC.make_scene(200_000, 3, "log", 1.0, 20.0, seed=9)
    g = Gaussians.from_scene(sc)
    R = Rasterizer()
    cams, arrivals = _trace(24)
    reqs = [Request(k, float(arrivals[k]), Camera.from_dict(c)) for k, c in enumerate(cams)]
    srv = Server(g, R, max_batch=8, n_streams=3, hbm_budget_bytes=8 << 30)
    stats = srv.serve(reqs, realtime=True, keep_outputs=True)
    torch.cuda.synchronize()
    assert stats.n == len(reqs)
    print("served", stats.summary())
    for res in stats.results:
        st = R.forward(g, reqs[res.rid].camera)
        torch.cuda.synchronize()
        assert torch.equal(res.rgb, st.rgb), res.rid
        assert torch.equal(res.T, st.T), res.rid
    # oracle spot check of one fisheye request
    k = 1
    act = st_act = None
    st = R.forward(g, reqs[k].camera)
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(act.size, size=min(400, act.size), replace=False))
    pr = O.preprocess(sc, cams[k])
    rgb_o, T_o, _, frag = O.render(sc, cams[k], pr, act[idx], **PT.BANDS)
    res = stats.results[k]
    PT.compare_render(res.rgb.cpu().numpy()[:, idx].astype(np.float64), res.T.cpu().numpy()[idx].astype(np.float64),
                      rgb_o, T_o, frag)


def test_sequential_baseline_runs():
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    from paper_2606_29794_amd.serve import Request, Server
    sc = SC.make_scene(50_000, 3, "log", 1.0, 20.0, seed=3)
    g = Gaussians.from_scene(sc)
    srv = Server(g, Rasterizer())
    cams, arrivals = _trace(6, seed=3)
    reqs = [Request(k, float(arrivals[k]), Camera.from_dict(c)) for k, c in enumerate(cams)]
    s1 = srv.serve_sequential(reqs, realtime=False, keep_outputs=True)
    s2 = srv.serve(reqs, realtime=False, keep_outputs=True)
    for a, b in zip(s1.results, sorted(s2.results, key=lambda r: r.rid)):
        assert torch.equal(a.rgb, b.rgb)


PERSISTENT_OFF = pytest.mark.skip(
    reason="hp_render_fwd_persistent is switched off (returns HP_ERR_UNSUPPORTED): its launches did not end on "
           "MI355X, in this test too, and no defect in the code that explains it has been found")


@PERSISTENT_OFF
def test_persistent_queue_equals_single_renders():
    """Through the C ABI: three requests pushed into a queue, then one
    persistent launch (same stream, so every item is there when it starts)
    renders every tile exactly as hp_render_fwd does alone."""
    import ctypes as C
    import torch
    from paper_2606_29794_amd import _abi as A
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer, _p
    sc = SC.make_scene(60_000, 3, "log", 1.0, 20.0, seed=4)
    g = Gaussians.from_scene(sc)
    R = Rasterizer()
    cams, _ = _trace(3, seed=8)
    qn = A.lib().hp_render_queue_bytes(1 << 16)
    queue = torch.empty(qn, dtype=torch.uint8, device="cuda")
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    A.call("hp_render_queue_reset", _p(queue), qn, sp)
    keep, outs, refs = [], [], []
    for k, cd in enumerate(cams):
        cam = Camera.from_dict(cd)
        st = R.forward(g, cam)
        m = st.mask
        rgb = torch.full((3, m.n_active), -1.0, device="cuda")
        T = torch.full((m.n_active,), -1.0, device="cuda")
        nc = torch.full((m.n_active,), -1, dtype=torch.int32, device="cuda")
        rq = A.hp_render_req(st.projected.data_ptr(), g.P, st.vals.data_ptr(), st.ranges.data_ptr(), m.n_tiles,
                             cam.order, m.buf.data_ptr(), m.n_active, rgb.data_ptr(), T.data_ptr(), nc.data_ptr())
        A.call("hp_render_queue_push", _p(queue), qn, k, C.byref(rq), C.byref(R.prm), int(k == 2), sp)
        keep.append(st)
        outs.append((rgb, T, nc, m.n_tiles))
        refs.append((st.rgb, st.T, st.n_contrib))
    A.call("hp_render_fwd_persistent", _p(queue), qn, 512, 1000, sp)
    done = (C.c_int32 * 3)()
    over = C.c_int32(0)
    A.call("hp_render_queue_status", _p(queue), 3, done, C.byref(over), sp)
    assert over.value == 0
    for k in range(3):
        rgb, T, nc, nt = outs[k]
        assert done[k] == nt
        assert torch.equal(rgb, refs[k][0]) and torch.equal(T, refs[k][1]) and torch.equal(nc, refs[k][2])


@PERSISTENT_OFF
@pytest.mark.parametrize("spin", [0, None])
def test_persistent_server_equals_batched_launches(spin):
    """The server with the persistent render (items drained while later
    requests are still being binned) gives the same images as with one
    ordinary launch per batch.  With a spin limit of 0 the launch gives up at
    the first empty poll (forced from the host): the requests it left
    unfinished are found by their done counters and rendered again."""
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    from paper_2606_29794_amd.serve import Request, Server
    sc = SC.make_scene(150_000, 3, "log", 1.0, 20.0, seed=10)
    g = Gaussians.from_scene(sc)
    R = Rasterizer()
    cams, arrivals = _trace(18, seed=12)
    reqs = [Request(k, float(arrivals[k]), Camera.from_dict(c)) for k, c in enumerate(cams)]
    kw = {} if spin is None else {"spin_limit": spin}
    s1 = Server(g, R, max_batch=6, n_streams=3, persistent=True, **kw).serve(reqs, realtime=False, keep_outputs=True)
    srv0 = Server(g, R, max_batch=6, n_streams=3, persistent=False)
    s2 = srv0.serve(reqs, realtime=False, keep_outputs=True)
    a = sorted(s1.results, key=lambda r: r.rid)
    b = sorted(s2.results, key=lambda r: r.rid)
    for x, y in zip(a, b):
        assert torch.equal(x.rgb, y.rgb) and torch.equal(x.T, y.T), x.rid


def test_admission_keeps_memory_within_budget():
    """With a budget that admits only a few requests at a time, the device
    memory the serving loop allocates beyond what it held before (the
    per-slot workspaces, the grids and masks of the camera models, all made
    during a warm-up) stays within the budget minus the reserve, and the
    served images still equal solo renders."""
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    from paper_2606_29794_amd.serve import Request, Server
    sc = SC.make_scene(100_000, 3, "log", 1.0, 20.0, seed=6)
    g = Gaussians.from_scene(sc)
    R = Rasterizer()
    cams, arrivals = _trace(24, seed=14)
    reqs = [Request(k, float(arrivals[k]), Camera.from_dict(c)) for k, c in enumerate(cams)]
    probe = Server(g, R, max_batch=8, n_streams=3)
    probe.serve(reqs, realtime=False)      # warm: hints, masks, tables, workspaces
    torch.cuda.synchronize()
    est = max(probe._estimate(r.camera) for r in reqs)
    reserve = probe.workspace_reserve()
    budget = reserve + int(2.5 * est)       # about two requests in flight
    srv = Server(g, R, max_batch=8, n_streams=3, hbm_budget_bytes=budget)
    srv.streams = probe.streams             # the warm-up's streams (their workspaces exist)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    stats = srv.serve(reqs, realtime=False, keep_outputs=False)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    print("budget in flight", budget - reserve, "peak", peak, "largest request estimate", est)
    assert stats.n == len(reqs)
    assert peak <= budget - reserve
    # the images of a run under the same budget, kept this time
    kept = Server(g, R, max_batch=8, n_streams=3, hbm_budget_bytes=budget).serve(reqs, realtime=False,
                                                                                keep_outputs=True)
    for res in kept.results[:6]:
        st = R.forward(g, reqs[res.rid].camera)
        torch.cuda.synchronize()
        assert torch.equal(res.rgb, st.rgb) and torch.equal(res.T, st.T), res.rid
