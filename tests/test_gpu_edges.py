"""GPU parity at the edges of the grid and of the input: the coarsest orders
(a tile is a whole face or less), the finest supported order (Nside 4096,
201M pixels, through a narrow pinhole), and an empty scene."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_2606_29794_amd import raster
    assert torch.cuda.is_available()
    return raster.Rasterizer()


@pytest.mark.parametrize("order", [0, 1, 2])
def test_coarsest_orders_forward_and_backward(R, order):
    """Nside 1, 2, 4: one tile per face (B = Nside), every pixel checked."""
    rng = np.random.default_rng(60 + order)
    wl = SC.config1_fd("overlap")
    sc = wl.scene
    cam = SC.make_camera(rng, order, SC.CAM_FULL)
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = O.mask(cam)
    assert np.array_equal(st.mask.active_pix.cpu().numpy().astype(np.int64), act)
    pr = O.preprocess(sc, cam)
    rgb_o, T_o, nu_o, frag = O.render(sc, cam, pr, act, **PT.BANDS)
    worst, nfrag = PT.compare_render(st.rgb.cpu().numpy().astype(np.float64), st.T.cpu().numpy().astype(np.float64),
                                     rgb_o, T_o, frag)
    # backward over the robust pixels
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    dC = rng.normal(size=(3, act.size))
    dC[:, frag > 0] = 0
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.as_tensor(dC, dtype=torch.float32, device="cuda"), None, gr)
    torch.cuda.synchronize()
    go = O.render_bwd(sc, cam, pr, act, dC, None)
    for k in ("mean", "scale", "rot", "opacity", "sh"):
        PT.grad_compare(f"order{order}:{k}", getattr(gr, k).cpu().numpy(), getattr(go, k))
    print("order", order, "pixels", act.size, "max err", worst, "fragile", nfrag)


def test_finest_order_narrow_pinhole(R):
    """Order 12 (Nside 4096) through a 10 x 6 degree pinhole: the active pixel
    list equals the oracle's, and sampled pixels match its render."""
    rng = np.random.default_rng(71)
    wl = SC.config1(P=20000, order=8)
    cam = SC.make_camera(rng, 12, SC.CAM_PINHOLE, fov_x=math.radians(10), fov_y=math.radians(6))
    g, c, st = PT.gpu_forward(R, wl.scene, cam)
    act = O.mask(cam)
    assert act.size > 0
    assert np.array_equal(st.mask.active_pix.cpu().numpy().astype(np.int64), act)
    idx = np.sort(rng.choice(act.size, size=min(400, act.size), replace=False))
    pr = O.preprocess(wl.scene, cam)
    rgb_o, T_o, nu_o, frag = O.render(wl.scene, cam, pr, act[idx], **PT.BANDS)
    worst, nfrag = PT.compare_render(st.rgb.cpu().numpy().astype(np.float64)[:, idx],
                                     st.T.cpu().numpy().astype(np.float64)[idx], rgb_o, T_o, frag)
    print("order 12 pinhole: active", act.size, "tiles", st.mask.n_tiles, "pairs", st.n_pairs, "max err", worst)
    assert float(T_o.min()) < 0.99   # something is in view


def test_empty_scene(R):
    """No Gaussian at all: every pixel keeps T = 1 and colour 0, no pairs."""
    import copy
    wl = SC.config0(P=1)
    sc = copy.deepcopy(wl.scene)
    sc.mean[:] = 0.01   # the one Gaussian sits inside r_min and is culled
    g, c, st = PT.gpu_forward(R, sc, wl.cameras[0])
    assert st.n_pairs == 0
    assert float(st.T.min()) == 1.0 and float(st.rgb.abs().max()) == 0.0


def test_single_visible_gaussian(R):
    """One Gaussian in view (the depth sort of a single element takes its own
    path: the key copied, the order written, no pass): image equal to the
    oracle's."""
    wl = SC.config0(P=1)
    cam = wl.cameras[0]
    g, c, st = PT.gpu_forward(R, wl.scene, cam)
    assert st.n_pairs > 0
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    pr = O.preprocess(wl.scene, cam)
    rgb_o, T_o, nu_o, frag = O.render(wl.scene, cam, pr, act, **PT.BANDS)
    PT.compare_render(st.rgb.cpu().numpy().astype(np.float64), st.T.cpu().numpy().astype(np.float64), rgb_o, T_o,
                      frag)
    assert float(T_o.min()) < 0.99   # the Gaussian covers some pixels


def test_wide_footprints_every_k2_range(R):
    """Gaussians 20-70 degrees across at order 5: a large share of the pixels
    they reach lie 14.5-30 degrees from the centre (the twelve-term series
    range of k2 = (angle / sin angle)^2) or farther (the atan2 form), so every
    form of k2 is checked, forward over every pixel and backward over the
    robust ones."""
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    rng = np.random.default_rng(83)
    sc = SC.make_scene(24, 3, "volume", 2.0, 6.0, 83, log_scale_mu=-0.3, log_scale_sigma=0.3, rng=rng)
    cam = SC.make_camera(rng, 5, SC.CAM_FULL)
    pr = O.preprocess(sc, cam)
    act = O.mask(cam)
    ang = np.arccos(np.clip(O.pix_vec(5, act) @ pr.dirs(), -1, 1))
    s2 = np.sin(ang[ang <= pr.rs[None, :]]) ** 2
    assert np.mean((s2 >= 1 / 16) & (s2 < 1 / 4)) > 0.2 and np.mean(s2 < 1 / 16) > 0.05
    g, c, st = PT.gpu_forward(R, sc, cam)
    rgb_o, T_o, nu_o, frag = O.render(sc, cam, pr, act, **PT.BANDS)
    worst, nfrag = PT.compare_render(st.rgb.cpu().numpy().astype(np.float64), st.T.cpu().numpy().astype(np.float64),
                                     rgb_o, T_o, frag)
    dC = rng.normal(size=(3, act.size))
    dC[:, frag > 0] = 0
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.as_tensor(dC, dtype=torch.float32, device="cuda"), None, gr)
    torch.cuda.synchronize()
    go = O.render_bwd(sc, cam, pr, act, dC, None)
    for k in ("mean", "scale", "rot", "opacity", "sh"):
        PT.grad_compare(f"wide:{k}", getattr(gr, k).cpu().numpy(), getattr(go, k))
    print("wide footprints: max err", worst, "fragile", nfrag)
