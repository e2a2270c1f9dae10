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
