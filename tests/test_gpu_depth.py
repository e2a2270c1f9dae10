"""GPU parity of the inverse radial depth channel (Sec. 3.2 depth
supervision: r^-1 composited like a colour, gradient -t / r^3) and of the
radian-space density-control statistics against the FP64 oracle."""
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


def _case(name):
    if name == "cfg0":
        wl = SC.config0()
    else:
        wl = SC.config1_fd(name)
    return wl.scene, wl.cameras[0]


def _forward(R, sc, camd):
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians
    g = Gaussians.from_scene(sc)
    cam = Camera.from_dict(camd)
    st = R.forward(g, cam, want_depth=True)
    torch.cuda.synchronize()
    return g, cam, st


@pytest.mark.parametrize("case", ["cfg0", "overlap", "literal"])
def test_inverse_depth_forward_matches_oracle(R, case):
    sc, camd = _case(case)
    g, cam, st = _forward(R, sc, camd)
    act = O.mask(camd)
    pr = O.preprocess(sc, camd)
    rgb_o, T_o, nu, frag, D_o = O.render(sc, camd, pr, act, **PT.BANDS, want_depth=True)
    D_g = st.inv_depth.cpu().numpy().astype(np.float64)
    robust = frag == 0
    err = np.abs(D_g - D_o)
    print(case, "max inv-depth err", err[robust].max(), "max value", D_o.max(), "fragile", (~robust).sum())
    assert err[robust].max() <= PT.COLOUR_ATOL
    # colour and T unchanged by the extra channel
    st0 = R.forward(g, cam)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(st0.rgb, st.rgb) and torch.equal(st0.T, st.T) and torch.equal(st0.n_contrib, st.n_contrib)


@pytest.mark.parametrize("case", ["overlap", "literal", "cfg0"])
def test_inverse_depth_backward_matches_oracle(R, case):
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    sc, camd = _case(case)
    g, cam, st = _forward(R, sc, camd)
    act = O.mask(camd)
    pr = O.preprocess(sc, camd)
    _, _, _, frag = O.render(sc, camd, pr, act, **PT.BANDS)
    rng = np.random.default_rng(23)
    dC = rng.normal(size=(3, act.size)) * 0.5
    dD = rng.normal(size=act.size)
    dC[:, frag > 0] = 0
    dD[frag > 0] = 0
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.as_tensor(dC, dtype=torch.float32, device="cuda"), None, gr,
               dL_dinv_depth=torch.as_tensor(dD, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    go = O.render_bwd(sc, camd, pr, act, dC, None, dLdD=dD)
    for k in ("mean", "scale", "rot", "opacity", "sh"):
        e = PT.grad_compare(f"{case}:{k}", getattr(gr, k).cpu().numpy(), getattr(go, k))
        print(case, k, "rel err", e)


def test_depth_only_gradient_reaches_means(R):
    """With only a depth upstream the colour and SH gradients vanish and the
    means still move (through alpha and through 1/r)."""
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    sc, camd = _case("overlap")
    g, cam, st = _forward(R, sc, camd)
    act = O.mask(camd)
    pr = O.preprocess(sc, camd)
    _, _, _, frag = O.render(sc, camd, pr, act, **PT.BANDS)
    dD = np.random.default_rng(29).normal(size=act.size)
    dD[frag > 0] = 0
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    zero = torch.zeros((3, act.size), dtype=torch.float32, device="cuda")
    R.backward(g, st, zero, None, gr, dL_dinv_depth=torch.as_tensor(dD, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    go = O.render_bwd(sc, camd, pr, act, np.zeros((3, act.size)), None, dLdD=dD)
    assert torch.count_nonzero(gr.sh).item() == 0
    for k in ("mean", "scale", "rot", "opacity"):
        PT.grad_compare(f"depth-only:{k}", getattr(gr, k).cpu().numpy(), getattr(go, k))


def test_autograd_depth_equals_direct_calls(R):
    import torch
    from paper_2606_29794_amd.raster import Gaussians
    from paper_2606_29794_amd.render import render
    sc, camd = _case("overlap")
    _, cam, st = _forward(R, sc, camd)
    g = Gaussians.from_scene(sc)
    params = [t.clone().requires_grad_(True) for t in (g.mean, g.scale, g.rot, g.opacity, g.sh)]
    rgb, T, invd = render(*params, cam, R, want_depth=True)
    w = torch.linspace(-1, 1, invd.numel(), device="cuda")
    (invd * w).sum().backward()
    z = torch.zeros_like
    gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
    R.backward(g, st, torch.zeros_like(st.rgb), None, gr, dL_dinv_depth=w)
    torch.cuda.synchronize()
    assert torch.equal(invd.detach(), st.inv_depth)
    for p, k in zip(params, ("mean", "scale", "rot", "opacity", "sh")):
        a = p.grad.double().cpu().numpy().ravel()
        b = getattr(gr, k).double().cpu().numpy().ravel()
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 1e-5 * max(nb, 1e-30), k


def test_density_stats_match_oracle_definition(R):
    import torch
    sc, camd = _case("overlap")
    g, cam, st = _forward(R, sc, camd)
    act = O.mask(camd)
    pr = O.preprocess(sc, camd)
    _, _, _, frag = O.render(sc, camd, pr, act, **PT.BANDS)
    rng = np.random.default_rng(31)
    dC = rng.normal(size=(3, act.size)); dC[:, frag > 0] = 0
    acc = torch.zeros((10, g.P), dtype=torch.float32, device="cuda")
    R.backward_pixels(st, torch.as_tensor(dC, dtype=torch.float32, device="cuda"), None, acc)
    rs_max = torch.full((g.P,), 0.01, dtype=torch.float32, device="cuda")
    gacc = torch.zeros(g.P, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(g.P, dtype=torch.int32, device="cuda")
    for _ in range(2):   # two identical views: the max is idempotent, the sums double
        R.density_stats(st, acc, rs_max, gacc, cnt)
    torch.cuda.synchronize()
    # oracle: visibility = at least one tile, gradients w.r.t. (omega, phi)
    gg, tt, m, inn = O.tile_sets(camd["order"], pr, act, report_band=1e-4)
    vis = np.zeros(g.P, bool); vis[gg[inn == 1]] = True
    band = np.zeros(g.P, bool); band[gg[np.abs(m) <= PT.bin_band(pr.rs[gg], 0.3)]] = True
    _, ang = O.render_bwd(sc, camd, pr, act, dC, None, want_angles=True)
    r1, a1, c1 = O.density_stats(pr.rs, vis, ang, pr.phi, np.full(g.P, 0.01), np.zeros(g.P), np.zeros(g.P, np.int64))
    r2, a2, c2 = O.density_stats(pr.rs, vis, ang, pr.phi, r1, a1, c1)
    ok = ~band
    assert np.array_equal(cnt.cpu().numpy()[ok], c2[ok])
    assert np.abs(rs_max.cpu().numpy()[ok] - r2[ok]).max() <= 1e-5 * max(1.0, r2.max())
    PT.grad_compare("grad accum", gacc.cpu().numpy()[ok], a2[ok])
    assert vis.sum() > 10
