"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on outputs the oracle can compute one by one:

* colours / T / composited counts at sampled active pixels of config 2
  (1M SH-3 Gaussians, full sphere at Nside 512) and config 3 (3M SH-3
  Gaussians, 60-degree pinhole at Nside 2048);
* complete per-Gaussian gradients for an upstream gradient that is non-zero
  only at sampled pixels: the oracle's backward over those pixels is then the
  exact reference for every Gaussian (configs 1, 2 and 3);
* the tile lists of 10,000 sampled Gaussians against the oracle's brute-force
  tile sets, and the depth order of every whole list (configs 2 and 3);
* the L1 + HEALPix-SSIM loss, its map and its gradient on whole images: the
  config-1 render (180-degree fisheye at Nside 256) against its target, and a
  full sphere at Nside 512."""
import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC
from tests import parity as PT

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_2606_29794_amd import raster
    assert torch.cuda.is_available()
    return raster.Rasterizer()


def _workload(name):
    return {"cfg1": SC.config1, "cfg2": SC.config2, "cfg3": SC.config3}[name]()


def _sample(act_size, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(act_size, size=min(n, act_size), replace=False))


@pytest.mark.parametrize("name,n_pix", [("cfg2", 800), ("cfg3", 300)])
def test_forward_sampled_full_size(R, name, n_pix):
    wl = _workload(name)
    sc, cam = wl.scene, wl.cameras[0]
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    assert np.array_equal(act, O.mask(cam))
    idx = _sample(act.size, n_pix, 11)
    pr = O.preprocess(sc, cam)
    rgb_o, T_o, nu_o, frag = O.render(sc, cam, pr, act[idx], **PT.BANDS)
    rgb_g = st.rgb.cpu().numpy().astype(np.float64)[:, idx]
    T_g = st.T.cpu().numpy().astype(np.float64)[idx]
    worst, nfrag = PT.compare_render(rgb_g, T_g, rgb_o, T_o, frag)
    _, _, _, nu_g = R.render_fwd(st.projected, g.P, st.vals, st.ranges, c, want_used=True)
    nu_g = nu_g.cpu().numpy()[idx]
    robust = frag == 0
    assert np.array_equal(nu_g[robust], nu_o[robust])
    print(name, "pairs", st.n_pairs, "max err", worst, "fragile", nfrag, "of", idx.size,
          "mean composited", float(nu_o.mean()))


@pytest.mark.parametrize("name,n_pix", [("cfg1", 300), ("cfg2", 300), ("cfg3", 150)])
def test_backward_sparse_upstream_full_size(R, name, n_pix):
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    wl = _workload(name)
    sc, cam = wl.scene, wl.cameras[0]
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    idx = _sample(act.size, n_pix, 12)
    pr = O.preprocess(sc, cam)
    _, _, _, frag = O.render(sc, cam, pr, act[idx], **PT.BANDS)
    idx = idx[frag == 0]   # a fragile pixel carries a discontinuity
    rng = np.random.default_rng(13)
    dC_s = rng.normal(size=(3, idx.size))
    dT_s = rng.normal(size=idx.size)
    dC = np.zeros((3, act.size), np.float32)
    dT = np.zeros(act.size, np.float32)
    dC[:, idx] = dC_s
    dT[idx] = dT_s
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.as_tensor(dC, device="cuda"), torch.as_tensor(dT, device="cuda"), gr)
    torch.cuda.synchronize()
    go = O.render_bwd(sc, cam, pr, act[idx], dC[:, idx].astype(np.float64), dT[idx].astype(np.float64))
    for k in ("mean", "scale", "rot", "opacity", "sh"):
        e = PT.grad_compare(f"{name}:{k}", getattr(gr, k).cpu().numpy(), getattr(go, k))
        print(name, k, "rel err", e)


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_tile_lists_sampled_full_size(R, name):
    """hp_bin_sorted's lists at full size (the path the benchmark times, with
    its XCD-contiguous chunking and its task capacity): 10,000 random
    Gaussians' tile memberships bit-exact against the oracle's tile sets up to
    fragile pairs, in depth order inside every tile."""
    wl = _workload(name)
    sc, cam = wl.scene, wl.cameras[0]
    g, c, st = PT.gpu_forward(R, sc, cam)
    pr = O.preprocess(sc, cam)
    gids = np.sort(np.random.default_rng(21).choice(sc.P, size=10_000, replace=False))
    stats = PT.compare_tile_lists_sampled(st, pr, cam, cam["order"], gids)
    print(name, stats, "list entries", st.n_pairs)
    assert stats["pairs"] > 0


def _loss_case(R, name):
    import torch
    from paper_2606_29794_amd.raster import Camera
    if name == "cfg1":
        # the config-1 render of its scene against its seeded target
        wl = SC.config1()
        camd = wl.cameras[0]
        g, c, st = PT.gpu_forward(R, wl.scene, camd)
        img = st.rgb
        ref = torch.as_tensor(SC.target_image(wl.seed, 0, st.mask.n_active), device="cuda")
        return camd, img, ref
    rng = np.random.default_rng(9)
    camd = SC.make_camera(rng, 9, SC.CAM_FULL)
    n = R.mask(Camera.from_dict(camd)).n_active
    img = torch.as_tensor(rng.random((3, n)), dtype=torch.float32, device="cuda")
    ref = torch.as_tensor(0.5 * rng.random((3, n)), dtype=torch.float32, device="cuda") + 0.5 * img
    return camd, img, ref


@pytest.mark.parametrize("name,zones", [("cfg1", False), ("order9_full", False), ("order9_full", True)])
def test_hssim_loss_full_size(R, name, zones):
    """hp_ssim (mean SSIM, L1, loss, per-pixel map and dL/dimg) against the
    oracle on whole images at the workloads' sizes: 393K active pixels of the
    config-1 fisheye at Nside 256, and 3.1M pixels of the full sphere at Nside
    512."""
    import torch
    from paper_2606_29794_amd.raster import Camera
    camd, img, ref = _loss_case(R, name)
    cam = Camera.from_dict(camd)
    from paper_2606_29794_amd import _abi as A
    up = torch.tensor([1.3], dtype=torch.float32, device="cuda")
    out, smap, dimg = R.ssim_loss(img, ref, cam, sp=A.default_ssim_params(zones=int(zones)), dL_dloss=up,
                                  want_map=True)
    torch.cuda.synchronize()
    act = O.mask(camd)
    im = img.cpu().numpy().astype(np.float64)
    rf = ref.cpu().numpy().astype(np.float64)
    s_o, map_o, _ = O.hssim(camd["order"], act, im, rf, want_map=True, zones=zones)
    L_o, gL_o = O.loss(camd["order"], act, im, rf, want_grad=True, zones=zones)
    out = out.cpu().numpy()
    assert abs(out[0] - s_o) < 1e-5 and abs(out[2] - L_o) < 1e-5, (out, s_o, L_o)
    assert abs(out[1] - np.mean(np.abs(im - rf))) < 1e-5
    err_map = np.abs(smap.cpu().numpy() - map_o).max()
    assert err_map < 2e-5, err_map
    e = PT.grad_compare(f"{name}: dL/dimg", dimg.cpu().numpy(), 1.3 * gL_o)
    print(name, "pixels", act.size, "ssim", out[0], "map err", err_map, "grad rel err", e)


def test_timed_step_equals_plain_views_full_size(R):
    """The step the benchmark times on config 2 (four full-sphere views at
    Nside 512, stages 1-2 prepared on two side streams while earlier views
    render, loss and backward accumulating into the parameters' .grad) gives
    the same images, bit for bit, and the same gradients, up to the order of
    float atomics, as rendering each view through the plain forward, which
    the tests above check against the oracle."""
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians
    from paper_2606_29794_amd.render import hssim_loss, render
    wl = SC.config2()
    g = Gaussians.from_scene(wl.scene)
    cams = [Camera.from_dict(c) for c in wl.cameras]
    targets = [torch.as_tensor(SC.target_image(wl.seed, v, R.mask(c).n_active), device="cuda")
               for v, c in enumerate(cams)]
    out = []
    for streams in (0, 2, 2):
        params = [t.clone().requires_grad_(True) for t in (g.mean, g.scale, g.rot, g.opacity, g.sh)]
        pf = R.prefetch(Gaussians(*[p.detach() for p in params]), cams, streams=streams) if streams else None
        imgs = []
        for v, cam in enumerate(cams):
            rgb, T = render(*params, cam, R, fused_grad=True, prepared=pf.get(v) if pf else None)
            loss, _ = hssim_loss(rgb, targets[v], cam, 0.2, R)
            loss.backward()
            imgs.append(rgb.detach().clone())
        torch.cuda.synchronize()
        out.append((imgs, [p.grad.double().cpu().numpy().ravel() for p in params]))
        del params, pf
    for imgs, grads in out[1:]:
        for a, b in zip(out[0][0], imgs):
            assert torch.equal(a, b)
        for a, b, k in zip(out[0][1], grads, ("mean", "scale", "rot", "opacity", "sh")):
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(a), k
    print("config 2 timed step: 4 views equal to the plain path")
