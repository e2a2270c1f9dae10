"""hp_render_bwd_noalloc (accumulators in the library's fixed device array)
against hp_render_bwd (accumulators in a caller workspace), both called
through the C ABI on the same forward state: two calls in a row, the second
on a smaller scene, so a stale array from the first call would show."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_29794_amd import _abi as A
from paper_2606_29794_amd import scenes as SC
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _grads_both(R, P, order, seed):
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, _p
    wl = SC.config1(P=P, order=order)
    g = Gaussians.from_scene(wl.scene)
    cam = Camera.from_dict(wl.cameras[0])
    st = R.forward(g, cam)
    rng = np.random.default_rng(seed)
    n = st.mask.n_active
    dC = torch.as_tensor(rng.normal(size=(3, n)).astype(np.float32), device="cuda")
    dT = torch.as_tensor(rng.normal(size=n).astype(np.float32), device="cuda")
    v = cam.view()
    gs = g.struct()
    out = []
    for noalloc in (False, True):
        z = torch.zeros_like
        gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
        gg = A.hp_gaussians_grad(gr.mean.data_ptr(), gr.scale.data_ptr(), gr.rot.data_ptr(), gr.opacity.data_ptr(),
                                 gr.sh.data_ptr())
        common = (C.byref(gs), _p(st.projected), _p(st.vals), _p(st.ranges), st.mask.n_tiles, C.byref(v),
                  C.byref(R.prm), _p(st.mask.buf), n, _p(st.T), _p(st.n_contrib), _p(dC), _p(dT), None, C.byref(gg))
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if noalloc:
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            A.call("hp_render_bwd_noalloc", *common, stream)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
        else:
            ws_n = A.lib().hp_render_bwd_workspace_bytes(g.P)
            ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
            A.call("hp_render_bwd", *common, _p(ws), ws_n, stream)
            torch.cuda.synchronize()
        out.append({k: getattr(gr, k).cpu().numpy() for k in ("mean", "scale", "rot", "opacity", "sh")})
    return out


def test_noalloc_backward_equals_workspace_backward():
    import torch
    from paper_2606_29794_amd import raster
    assert torch.cuda.is_available()
    R = raster.Rasterizer()
    for P, order, seed in ((30_000, 7, 1), (6_000, 6, 2)):
        ref, got = _grads_both(R, P, order, seed)
        for k in ref:
            e = PT.grad_compare(f"noalloc P={P}:{k}", got[k], ref[k])
            print("P", P, k, "rel diff", e)
