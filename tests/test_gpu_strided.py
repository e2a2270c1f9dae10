"""Arguments that are strided views: the Python layer hands the library a
contiguous copy of each and keeps every copy alive until the call has
enqueued its kernels, so no copy's memory is handed to the next one of the
same call.  Results equal those of the contiguous tensors."""
import numpy as np
import pytest

from paper_2606_29794_amd import scenes as SC

pytestmark = pytest.mark.gpu


def _strided(x):
    """The same values as x [C, n], in a [C, n] view of an [n, C] tensor."""
    return x.t().contiguous().t()


def test_strided_images_and_gradients_equal_contiguous():
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    R = Rasterizer()
    rng = np.random.default_rng(21)
    sc = SC.make_scene(20_000, 3, "log", 1.0, 20.0, seed=21)
    g = Gaussians.from_scene(sc)
    cam = Camera.from_dict(SC.make_camera(rng, 6, SC.CAM_FULL, center_radius=0.5))
    st = R.forward(g, cam)
    n = st.mask.n_active
    ref = torch.rand((3, n), device="cuda")
    up = torch.ones(1, device="cuda")
    img_s, ref_s = _strided(st.rgb), _strided(ref)
    assert not img_s.is_contiguous() and not ref_s.is_contiguous()
    out_c, map_c, d_c = R.ssim_loss(st.rgb, ref, cam, dL_dloss=up, want_map=True)
    out_s, map_s, d_s = R.ssim_loss(img_s, ref_s, cam, dL_dloss=up, want_map=True)
    torch.cuda.synchronize()
    assert torch.equal(out_c, out_s) and torch.equal(map_c, map_s) and torch.equal(d_c, d_s)
    # two copies sharing memory would compare an image with itself (L1 0)
    assert float(out_s[1]) > 0.0 and float(out_s[0]) < 1.0
    # upstream gradients as strided views: the per-Gaussian accumulators agree
    # (float atomics: equal up to the order of the additions)
    gC = torch.randn((3, n), device="cuda")
    gT = torch.randn(n, device="cuda")
    gT_s = torch.stack([gT, gT], 1)[:, 0]
    assert not gT_s.is_contiguous()
    acc_c = torch.zeros((10, g.P), device="cuda")
    acc_s = torch.zeros((10, g.P), device="cuda")
    R.backward_pixels(st, gC, gT, acc_c)
    R.backward_pixels(st, _strided(gC), gT_s, acc_s)
    torch.cuda.synchronize()
    scale = float(acc_c.abs().max())
    assert scale > 0
    assert torch.allclose(acc_c, acc_s, rtol=1e-5, atol=1e-6 * scale)
