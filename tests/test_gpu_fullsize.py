"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times, on outputs the oracle can compute one by one:

* colours / T / composited counts at sampled active pixels of config 2
  (1M SH-3 Gaussians, full sphere at Nside 512) and config 3 (3M SH-3
  Gaussians, 60-degree pinhole at Nside 2048);
* complete per-Gaussian gradients for an upstream gradient that is non-zero
  only at sampled pixels: the oracle's backward over those pixels is then the
  exact reference for every Gaussian."""
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
    return {"cfg2": SC.config2, "cfg3": SC.config3}[name]()


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
    rgb_o, T_o, nu_o, frag = O.render(sc, cam, pr, act[idx], qtol=PT.qtol_for(), ttol=1e-3)
    rgb_g = st.rgb.cpu().numpy().astype(np.float64)[:, idx]
    T_g = st.T.cpu().numpy().astype(np.float64)[idx]
    worst, nfrag = PT.compare_render(rgb_g, T_g, rgb_o, T_o, frag)
    _, _, _, nu_g = R.render_fwd(st.projected, g.P, st.vals, st.ranges, c, want_used=True)
    nu_g = nu_g.cpu().numpy()[idx]
    robust = frag == 0
    assert np.array_equal(nu_g[robust], nu_o[robust])
    print(name, "pairs", st.n_pairs, "max err", worst, "fragile", nfrag, "of", idx.size,
          "mean composited", float(nu_o.mean()))


@pytest.mark.parametrize("name,n_pix", [("cfg2", 300), ("cfg3", 150)])
def test_backward_sparse_upstream_full_size(R, name, n_pix):
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    wl = _workload(name)
    sc, cam = wl.scene, wl.cameras[0]
    g, c, st = PT.gpu_forward(R, sc, cam)
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    idx = _sample(act.size, n_pix, 12)
    pr = O.preprocess(sc, cam)
    _, _, _, frag = O.render(sc, cam, pr, act[idx], qtol=PT.qtol_for(), ttol=1e-3)
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
