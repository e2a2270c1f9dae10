"""Pins of the oracle's inverse radial depth channel (Sec. 3.2: depth
supervision with r^-1 and its gradient -t / r^3) and of the radian-space
density-control statistics: closed forms for one Gaussian and for a scene at
constant depth, and finite differences of a depth loss."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC
from tests.test_oracle_grad import _get


def _cam(order):
    return dict(W=np.eye(3, dtype=np.float32), b=np.zeros(3, np.float32), center=np.zeros(3, np.float32),
                cam_type=0, fov_x=2 * math.pi, fov_y=math.pi, order=order)


def test_single_gaussian_inverse_depth_is_alpha_over_r():
    order = 5
    d0 = np.array([0.2, 0.4, -0.8]); d0 /= np.linalg.norm(d0)
    r = 2.5
    sc = SC.Scene((d0 * r)[:, None].astype(np.float32), np.full((3, 1), 0.12, np.float32),
                  np.array([[1], [0], [0], [0]], np.float32), np.array([0.7], np.float32),
                  np.zeros((1, 3, 1), np.float32), 0)
    cam = _cam(order)
    act = np.arange(O.npix(order))
    pr = O.preprocess(sc, cam)
    rgb, T, nu, fr, D = O.render(sc, cam, pr, act, want_depth=True)
    alpha = 1 - T
    rho = float(np.linalg.norm(sc.mean[:, 0].astype(np.float64)))
    assert alpha.max() > 0.3
    assert np.abs(D - alpha / rho).max() < 1e-13


def test_constant_depth_scene_telescopes():
    """Every Gaussian at the same distance r: the weights alpha_i T_i sum to
    1 - T_final, so the inverse depth is (1 - T) / r at every pixel."""
    order = 4
    rng = np.random.default_rng(3)
    P = 300
    d = rng.normal(size=(3, P)); d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = 3.0
    sc = SC.Scene((d * r).astype(np.float32), np.exp(rng.normal(-1.3, 0.3, size=(3, P))).astype(np.float32),
                  rng.normal(size=(4, P)).astype(np.float32), rng.uniform(0.2, 0.9, P).astype(np.float32),
                  np.zeros((1, 3, P), np.float32), 0)
    cam = _cam(order)
    act = np.arange(O.npix(order))
    pr = O.preprocess(sc, cam)
    rgb, T, nu, fr, D = O.render(sc, cam, pr, act, want_depth=True)
    rho = np.linalg.norm(sc.mean.astype(np.float64), axis=0)
    assert np.abs(rho - r).max() < 1e-5
    # per pixel the composited 1/rho lies between (1 - T)/max rho and (1 - T)/min rho
    lo, hi = (1 - T) / rho.max(), (1 - T) / rho.min()
    assert (D >= lo - 1e-12).all() and (D <= hi + 1e-12).all()
    assert (T < 0.999).sum() > act.size // 4
    assert np.abs(D - (1 - T) / r).max() < 2e-6


def _depth_loss(scene, cam, act, wD):
    pr = O.preprocess(scene, cam)
    rgb, T, nu, fr, D = O.render(scene, cam, pr, act, qtol=1e-4, ttol=1e-6, want_depth=True)
    return float((wD * D).sum()), nu, fr


def test_depth_gradients_match_finite_differences():
    wl = SC.config1_fd("overlap")
    sc, cam = wl.scene, wl.cameras[0]
    act = O.mask(cam)
    rng = np.random.default_rng(17)
    wD = rng.normal(size=act.size)
    pr = O.preprocess(sc, cam)
    zero = np.zeros((3, act.size))
    g = O.render_bwd(sc, cam, pr, act, zero, None, dLdD=wD)
    _, _, nu, _ = O.render(sc, cam, pr, act)
    hit = np.nonzero(np.abs(g.opacity) > 0)[0]
    assert hit.size >= 20
    checked = 0
    for i in hit[:10]:
        for group, ncomp in [("mean", 3), ("scale", 3), ("rot", 4), ("opacity", 1)]:
            for c in range(ncomp):
                arr = _get(sc, group)
                idx = (i,) if group == "opacity" else (c, i)
                x0 = float(arr[idx])
                h = 2e-4 * max(1.0, abs(x0))
                vals, ok = [], True
                for sgn in (+1, -1):
                    sc2 = SC.Scene(sc.mean.copy(), sc.scale.copy(), sc.rot.copy(), sc.opacity.copy(), sc.sh.copy(),
                                   sc.sh_degree)
                    _get(sc2, group)[idx] = np.float32(x0 + sgn * h)
                    L, nu2, fr2 = _depth_loss(sc2, cam, act, wD)
                    ok = ok and np.array_equal(nu2, nu) and fr2.max() == 0
                    vals.append(L)
                if not ok:
                    continue
                h_eff = float(np.float32(x0 + h)) - float(np.float32(x0 - h))
                num = (vals[0] - vals[1]) / h_eff
                an = float({"mean": g.mean, "scale": g.scale, "rot": g.rot, "opacity": g.opacity}[group][idx])
                scale = max(1e-4, abs(an), abs(num))
                assert abs(num - an) <= 2e-3 * scale, (i, group, c, num, an)
                checked += 1
    assert checked > 60
    # depth gradients reach the mean even with no colour upstream, through
    # d(1/r)/dt = -t / r^3 as well as through alpha
    assert np.abs(g.mean[:, hit]).max() > 0


def test_density_statistics_definition():
    """r_s,max keeps the running maximum over views where the Gaussian is
    visible; the accumulator adds |(dL/domega / cos phi, dL/dphi)|."""
    rs = np.array([0.1, 0.5, 0.2, 0.0])
    vis = np.array([True, True, False, False])
    ang = np.array([[0.3, -1.0, 5.0, 1.0], [0.4, 0.0, 5.0, 1.0]])
    phi = np.array([0.0, math.pi / 3, 0.1, 0.2])
    rs_max, acc, cnt = O.density_stats(rs, vis, ang, phi, np.array([0.2, 0.1, 0.3, 0.0]), np.zeros(4), np.zeros(4, np.int64))
    assert np.allclose(rs_max, [0.2, 0.5, 0.3, 0.0])
    assert np.allclose(acc, [0.5, 2.0, 0.0, 0.0])
    assert np.array_equal(cnt, [1, 1, 0, 0])
