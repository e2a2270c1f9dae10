"""GPU parity of the grid tables, visibility mask and preprocessing against
the FP64 oracle (through the C ABI)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    from paper_2606_29794_amd import raster
    assert torch.cuda.is_available()
    return raster.Rasterizer()


@pytest.mark.parametrize("order", [2, 4, 6])
def test_grid_leaf_caps_match_oracle(R, order):
    import torch
    from paper_2606_29794_amd import _abi as A
    g = R.grid(order)
    tc, tr = O.tile_caps(order)
    kt = O.tile_order(order)
    nodes = 12 * (4 ** (kt + 1) - 1) // 3
    cap = g[: nodes * 16].view(torch.float32).view(nodes, 4).cpu().numpy().astype(np.float64)
    off = 12 * (4 ** kt - 1) // 3
    leaf = cap[off:]
    assert np.abs(leaf[:, :3] - tc).max() < 2e-7
    assert np.all(leaf[:, 3] >= tr - 1e-7) and np.abs(leaf[:, 3] - tr).max() < 2e-7
    # parents contain their children's caps
    for l in range(kt):
        o, co = 12 * (4 ** l - 1) // 3, 12 * (4 ** (l + 1) - 1) // 3
        par = cap[o:o + 12 * 4 ** l]
        ch = cap[co:co + 12 * 4 ** (l + 1)].reshape(-1, 4, 4)
        ang = np.arccos(np.clip(np.einsum("nk,nck->nc", par[:, :3], ch[:, :, :3]), -1, 1))
        assert np.all(ang + ch[:, :, 3] <= par[:, None, 3] + 1e-6)


def _cams():
    rng = np.random.default_rng(42)
    out = []
    for order in (5, 8):
        out.append(SC.make_camera(rng, order, SC.CAM_FULL))
        out.append(SC.make_camera(rng, order, SC.CAM_FISHEYE, fov_x=math.pi, fov_y=math.pi))
        out.append(SC.make_camera(rng, order, SC.CAM_FISHEYE, fov_x=math.radians(210), fov_y=math.radians(150)))
        fx = math.radians(75)
        out.append(SC.make_camera(rng, order, SC.CAM_PINHOLE, fov_x=fx, fov_y=SC.pinhole_fov_y(fx)))
    return out


@pytest.mark.parametrize("k", range(8))
def test_mask_bit_exact(R, k):
    from paper_2606_29794_amd.raster import Camera
    cam = _cams()[k]
    m = R.mask(Camera.from_dict(cam))
    ref = O.mask(cam)
    got = m.active_pix.cpu().numpy().astype(np.int64)
    assert m.n_active == ref.size
    assert np.array_equal(got, ref)
    kt = O.tile_order(cam["order"])
    assert m.n_tiles == np.unique(ref >> (2 * (cam["order"] - kt))).size


@pytest.mark.parametrize("wl_name", ["cfg0", "cfg1"])
def test_preprocess_matches_oracle(R, wl_name):
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians
    wl = SC.config0() if wl_name == "cfg0" else SC.config1(P=20000)
    cam = wl.cameras[0]
    g = Gaussians.from_scene(wl.scene)
    proj = R.preprocess(g, Camera.from_dict(cam))
    rec, depth, radius = R.projected_arrays(proj, g.P)
    rec = rec.cpu().numpy().astype(np.float64); depth = depth.cpu().numpy(); radius = radius.cpu().numpy()
    pr = O.preprocess(wl.scene, cam)
    valid = radius > 0
    assert np.array_equal(valid, pr.valid.astype(bool))
    v = valid
    u = pr.dirs()[:, v].T
    assert np.abs(rec[v, 0:3] - u).max() < 1e-6
    assert np.abs(rec[v, 3] - wl.scene.opacity[v]).max() == 0
    w, p = pr.omega[v], pr.phi[v]
    eo = np.stack([np.cos(w), -np.sin(w)], 1)
    ep = np.stack([-np.sin(p) * np.sin(w), np.cos(p), -np.sin(p) * np.cos(w)], 1)
    assert np.abs(rec[v][:, 4:6] - eo).max() < 1e-5
    assert np.abs(np.concatenate([rec[v][:, 6:8], rec[v][:, 8:9]], 1) - ep).max() < 1e-5
    assert np.allclose(depth[v], pr.rho[v], rtol=1e-6)
    assert np.allclose(radius[v], pr.rs[v], rtol=2e-5)
    Qg = rec[v][:, 9:12]
    Qo = pr.conic[:, v].T
    S = pr.sarc[:, v]
    tr = S[0] + S[2]
    disc = np.sqrt((S[0] - S[2]) ** 2 + 4 * S[1] ** 2)
    cond = (tr + disc) / np.maximum(tr - disc, 1e-300)
    err = np.linalg.norm(Qg - Qo, axis=1) / np.linalg.norm(Qo, axis=1)
    assert np.all(err <= 2e-6 * np.maximum(1.0, cond)), (err / np.maximum(1, cond)).max()
    assert np.abs(rec[v][:, 12:15] - pr.rgb[:, v].T).max() < 2e-5
