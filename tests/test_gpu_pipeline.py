"""GPU parity of the full rasterizer (bin, sort, render, backward, HSSIM)
against the FP64 oracle, through the C ABI, on seeded synthetic scenes."""
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


def _fd_scene(variant):
    wl = SC.config1_fd(variant)
    return wl.scene, wl.cameras[0]


CASES = {
    "cfg0": lambda: (SC.config0().scene, SC.config0().cameras[0]),
    "fd_overlap": lambda: _fd_scene("overlap"),
    "fd_literal": lambda: _fd_scene("literal"),
    "cfg1_small": lambda: (SC.config1(P=6000, order=6).scene, SC.config1(P=6000, order=6).cameras[0]),
}


def _big_discs():
    """700 Gaussians 10-60 degrees across at order 9: a workgroup of 256 has
    thousands of coarse tasks (more than the task scatter stages in LDS) and
    many Gaussians have more than 16 (the count walk's slots), so both
    fall-back paths of the node-order task list run.  Four of them are
    blown up to enclose the camera (r_s = pi): their discs reach the
    antipode, which the binning's near cap test must not take."""
    rng = np.random.default_rng(91)
    sc = SC.make_scene(700, 0, "volume", 2.0, 6.0, 91, log_scale_mu=-0.9, log_scale_sigma=0.5, rgb_dc=True, rng=rng)
    sc.scale[:, 100:104] *= 40.0
    return sc, SC.make_camera(rng, 9, SC.CAM_FULL)


def _order10():
    """3000 Gaussians at order 10, where the split level has 768 nodes: the
    task list's count and scatter passes take one round of 256 Gaussians per
    workgroup (two rounds below 384 nodes, as at order 9)."""
    rng = np.random.default_rng(101)
    sc = SC.make_scene(3000, 0, "volume", 2.0, 6.0, 101, log_scale_mu=-2.5, log_scale_sigma=0.6, rgb_dc=True, rng=rng)
    return sc, SC.make_camera(rng, 10, SC.CAM_FULL)


LIST_CASES = dict(CASES, big_discs=_big_discs, order10=_order10)


@pytest.mark.parametrize("case", list(LIST_CASES))
def test_tile_lists_and_order(R, case):
    sc, cam = LIST_CASES[case]()
    g, c, st = PT.gpu_forward(R, sc, cam)
    stats = PT.compare_tile_lists(R, st, sc, cam, cam["order"])
    print(case, stats)
    assert stats["pairs"] > 0


@pytest.mark.parametrize("case", list(LIST_CASES) + ["cfg1_fisheye", "cfg3_small"])
def test_sorted_bin_equals_bin_then_sort(R, case):
    """hp_bin_sorted emits exactly what hp_bin followed by the stable tile
    sort hp_sort gives: the same ids in the same order, the same ranges."""
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians
    if case == "cfg1_fisheye":
        wl = SC.config1(P=20000, order=8)
        sc, camd = wl.scene, wl.cameras[0]
    elif case == "cfg3_small":
        wl = SC.config3(P=50000, order=9)
        sc, camd = wl.scene, wl.cameras[0]
    else:
        sc, camd = LIST_CASES[case]()
    g = Gaussians.from_scene(sc)
    cam = Camera.from_dict(camd)
    proj = R.preprocess(g, cam)
    m = R.mask(cam)
    keys, vals, n = R.bin(proj, g.P, cam)
    ranges = R.sort(keys, vals, n, m.n_tiles)
    vals2, ranges2, n2 = R.bin_sorted(proj, g.P, cam)
    torch.cuda.synchronize()
    assert n2 == n
    assert torch.equal(vals[:n], vals2[:n])
    # ranges: equal lengths; equal starts where a tile has pairs (an empty
    # tile's start is arbitrary)
    r1, r2 = ranges.cpu().numpy().astype(np.int64), ranges2.cpu().numpy().astype(np.int64)
    len1, len2 = r1[:, 1] - r1[:, 0], r2[:, 1] - r2[:, 0]
    assert np.array_equal(len1, len2)
    assert np.array_equal(r1[len1 > 0, 0], r2[len2 > 0, 0])


@pytest.mark.parametrize("case", list(CASES))
def test_render_forward_full_image(R, case):
    sc, cam = CASES[case]()
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = O.mask(cam)
    pr = O.preprocess(sc, cam)
    rgb_o, T_o, nu, frag = O.render(sc, cam, pr, act, **PT.BANDS)
    rgb_g = st.rgb.cpu().numpy().astype(np.float64)
    T_g = st.T.cpu().numpy().astype(np.float64)
    worst, nfrag = PT.compare_render(rgb_g, T_g, rgb_o, T_o, frag)
    print(case, "max err", worst, "fragile px", nfrag, "of", act.size)
    # n_contrib: oracle walk of its own tile lists, on pixels without fragile decisions
    tc, tr = O.tile_caps(cam["order"])
    gg, tt, m, inn = O.tile_sets(cam["order"], pr, act, caps=(tc, tr), report_band=1e-4)
    lst, ranges = O.sorted_tile_lists(cam["order"], pr, gg, tt, inn)
    nc_o = O.n_contrib(sc, cam, pr, lst, ranges, act)
    fr_tiles = set(tt[np.abs(m) <= PT.bin_band(pr.rs[gg], tr[tt])].tolist())
    kt = O.tile_order(cam["order"])
    ptile = act >> (2 * (cam["order"] - kt))
    ok = (frag == 0) & np.array([t not in fr_tiles for t in ptile])
    nc_g = st.n_contrib.cpu().numpy()
    assert np.array_equal(nc_g[ok], nc_o[ok]), np.count_nonzero(nc_g[ok] != nc_o[ok])
    # Gaussians composited per pixel: exact on pixels without fragile decisions
    _, _, _, nu_g = R.render_fwd(st.projected, g.P, st.vals, st.ranges, c, want_used=True)
    nu_g = nu_g.cpu().numpy()
    assert np.array_equal(nu_g[frag == 0], nu[frag == 0])


def test_render_forward_sampled_config1(R):
    """Config 1 scene (100K SH-3 Gaussians, 180-degree fisheye, Nside 256),
    checked on 3000 sampled active pixels."""
    wl = SC.config1()
    sc, cam = wl.scene, wl.cameras[0]
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    assert np.array_equal(act, O.mask(cam))
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(act.size, size=3000, replace=False))
    pr = O.preprocess(sc, cam)
    rgb_o, T_o, nu, frag = O.render(sc, cam, pr, act[idx], **PT.BANDS)
    rgb_g = st.rgb.cpu().numpy().astype(np.float64)[:, idx]
    T_g = st.T.cpu().numpy().astype(np.float64)[idx]
    worst, nfrag = PT.compare_render(rgb_g, T_g, rgb_o, T_o, frag)
    print("cfg1 sampled: max err", worst, "fragile", nfrag, "pairs", st.n_pairs)


def _grads_gpu(R, g, st, dC, dT):
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    z = lambda t: torch.zeros_like(t)
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.as_tensor(dC, dtype=torch.float32, device="cuda"),
               None if dT is None else torch.as_tensor(dT, dtype=torch.float32, device="cuda"), gr)
    torch.cuda.synchronize()
    return {k: getattr(gr, k).cpu().numpy() for k in ("mean", "scale", "rot", "opacity", "sh")}


@pytest.mark.parametrize("case", ["fd_overlap", "fd_literal", "cfg0"])
def test_render_backward_matches_oracle(R, case):
    sc, cam = CASES[case]()
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = O.mask(cam)
    rng = np.random.default_rng(7)
    dC = rng.normal(size=(3, act.size)).astype(np.float32)
    dT = rng.normal(size=act.size).astype(np.float32)
    gg = _grads_gpu(R, g, st, dC, dT)
    pr = O.preprocess(sc, cam)
    # pixels with a fragile decision carry a discontinuity: leave them out on both sides
    _, _, _, frag = O.render(sc, cam, pr, act, **PT.BANDS)
    dC[:, frag > 0] = 0
    dT[frag > 0] = 0
    gg = _grads_gpu(R, g, st, dC, dT)
    go = O.render_bwd(sc, cam, pr, act, dC.astype(np.float64), dT.astype(np.float64))
    for k in ("mean", "scale", "rot", "opacity", "sh"):
        e = PT.grad_compare(f"{case}:{k}", gg[k], getattr(go, k))
        print(case, k, "rel err", e)


@pytest.mark.parametrize("zones", [False, True])
@pytest.mark.parametrize("order,masked", [(0, False), (1, False), (2, False), (2, True), (3, False), (4, False),
                                          (5, True), (6, True), (3, True), (7, False)])
def test_hssim_and_loss(R, order, masked, zones):
    """hp_ssim (mean, L1, loss, map, dL/dimg) and its split entry points
    against the oracle, with the isotropic chart window and with the
    zone-specific windows (polar caps weighted by great-circle distance).
    Orders 0-2 (tiles narrower than 8 pixels, windows wider than a face)
    take the direct path."""
    import torch
    from paper_2606_29794_amd.raster import Camera
    rng = np.random.default_rng(order)
    if masked:
        cam = SC.make_camera(rng, order, SC.CAM_FISHEYE, fov_x=math.radians(200), fov_y=math.radians(160))
    else:
        cam = SC.make_camera(rng, order, SC.CAM_FULL)
    m = R.mask(Camera.from_dict(cam))
    act = O.mask(cam)
    img = rng.random((3, act.size)).astype(np.float32)
    ref = (0.6 * img + 0.4 * rng.random((3, act.size))).astype(np.float32)
    ti = torch.as_tensor(img, device="cuda"); tr_ = torch.as_tensor(ref, device="cuda")
    up = torch.tensor([1.7], dtype=torch.float32, device="cuda")
    sp = A_default_ssim(zones=int(zones))
    out, smap, dimg = R.ssim_loss(ti, tr_, Camera.from_dict(cam), sp=sp, dL_dloss=up, want_map=True)
    torch.cuda.synchronize()
    s_o, map_o, g_o = O.hssim(order, act, img, ref, want_map=True, want_grad=True, zones=zones)
    L_o, gL_o = O.loss(order, act, img, ref, want_grad=True, zones=zones)
    out = out.cpu().numpy()
    assert abs(out[0] - s_o) < 2e-6 and abs(out[2] - L_o) < 2e-6
    assert abs(out[1] - np.mean(np.abs(img.astype(np.float64) - ref))) < 1e-6
    assert np.abs(smap.cpu().numpy() - map_o).max() < 2e-5
    PT.grad_compare("hssim-loss grad", dimg.cpu().numpy(), 1.7 * gL_o)
    # the split entry points (partials kept between forward and backward)
    # run the same kernels: identical results
    out2, smap2, ws = R.ssim_forward_saved(ti, tr_, Camera.from_dict(cam), sp=sp, want_map=True)
    dimg2 = R.ssim_backward_saved(ti, tr_, Camera.from_dict(cam), sp, ws, up)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), out)
    assert torch.equal(smap2, smap) and torch.equal(dimg2, dimg)


def A_default_ssim(**kw):
    from paper_2606_29794_amd import _abi as A
    return A.default_ssim_params(**kw)
