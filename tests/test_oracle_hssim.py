"""Pins of the oracle's HEALPix-SSIM and loss (Sec. 4.1; supp. masked HSSIM
average) -- no GPU."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O


def test_identity_constant_and_symmetry():
    order = 4
    act = np.arange(O.npix(order))
    rng = np.random.default_rng(0)
    x = rng.random((3, act.size)); y = rng.random((3, act.size))
    assert abs(O.hssim(order, act, x, x)[0] - 1) < 1e-12
    c = np.full((3, act.size), 0.37)
    assert abs(O.hssim(order, act, c, c)[0] - 1) < 1e-12
    assert abs(O.hssim(order, act, x, y)[0] - O.hssim(order, act, y, x)[0]) < 1e-12
    assert O.hssim(order, act, x, y)[0] < 0.2


def test_interior_equals_planar_ssim():
    """Away from face edges the chart is the face's own (x, y) grid and HSSIM
    is planar SSIM with a normalised 11x11, sigma 1.5 Gaussian window (Wang et
    al. 2004) -- scipy's gaussian_filter with radius 5."""
    order = 5
    N = 1 << order
    act = np.arange(O.npix(order))
    rng = np.random.default_rng(1)
    img = rng.random((3, act.size)); ref = rng.random((3, act.size))
    _, smap, _ = O.hssim(order, act, img, ref, want_map=True)
    f = 6
    xs, ys = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    pix = O.xyf2nest(order, xs.ravel(), ys.ravel(), np.full(N * N, f)).reshape(N, N)
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    filt = lambda a: ndimage.gaussian_filter(a, 1.5, truncate=5 / 1.5, mode="constant")
    for ch in range(3):
        X = img[ch][pix]; Y = ref[ch][pix]
        mx, my = filt(X), filt(Y)
        vx = filt(X * X) - mx * mx; vy = filt(Y * Y) - my * my; cxy = filt(X * Y) - mx * my
        s = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
        inner = (slice(5, N - 5), slice(5, N - 5))
        assert np.allclose(s[inner], smap[ch][pix][inner], atol=1e-12)


def test_seven_neighbour_renormalisation():
    """At the 24 pixels of the eight three-face vertices one 3x3 neighbour is
    missing; the window weights that remain are renormalised, so a constant
    image still gives SSIM exactly 1 there and on a masked (partial) sphere."""
    order = 3
    act = np.arange(O.npix(order))
    c = np.full((3, act.size), 0.6)
    _, m, _ = O.hssim(order, act, c, c * 0 + 0.6, want_map=True)
    assert np.allclose(m, 1, atol=1e-14)
    # masked half sphere: renormalisation over active neighbours only
    half = act[O.pix_vec(order, act)[:, 2] > 0.1]
    rng = np.random.default_rng(2)
    x = rng.random((3, half.size))
    assert abs(O.hssim(order, half, x, x)[0] - 1) < 1e-12


@pytest.mark.parametrize("masked", [False, True])
def test_hssim_and_loss_gradient_fd(masked):
    order = 3
    act = np.arange(O.npix(order))
    if masked:
        act = act[O.pix_vec(order, act)[:, 2] > -0.2]
    rng = np.random.default_rng(3)
    img = rng.random((3, act.size)); ref = rng.random((3, act.size))
    s, _, g = O.hssim(order, act, img, ref, want_grad=True)
    L, gL = O.loss(order, act, img, ref, want_grad=True)
    idx = rng.choice(3 * act.size, size=40, replace=False)
    h = 1e-6
    for k in idx:
        ch, p = divmod(int(k), act.size)
        xp = img.copy(); xp[ch, p] += h
        xm = img.copy(); xm[ch, p] -= h
        num = (O.hssim(order, act, xp, ref)[0] - O.hssim(order, act, xm, ref)[0]) / (2 * h)
        assert abs(num - g[ch, p]) < 1e-7 + 1e-5 * abs(g[ch, p])
        numL = (O.loss(order, act, xp, ref)[0] - O.loss(order, act, xm, ref)[0]) / (2 * h)
        assert abs(numL - gL[ch, p]) < 1e-7 + 1e-5 * abs(gL[ch, p])


# ---- zone-specific windows (Sec. 4.1: isotropic in the equatorial zone,
# anisotropic in the polar zones where the pixels are compressed) ----------
def _tangent_moments(order, p, zones):
    """Second moments of the raw window over the great-circle offsets of the
    neighbours, in the tangent plane at p: (2x2 tensor, sum of weights)."""
    q, w = O.hssim_window(order, p, zones=zones)
    up = O.pix_vec(order, np.array([p]))[0]
    e1 = np.cross([0.0, 1.0, 0.0], up)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(up, e1)
    ok = q.ravel() >= 0
    v = O.pix_vec(order, q.ravel()[ok])
    ww = w.ravel()[ok]
    d = np.arctan2(np.linalg.norm(np.cross(up, v), axis=1), v @ up)
    t = v - np.outer(v @ up, up)
    t *= (d / np.maximum(np.linalg.norm(t, axis=1), 1e-300))[:, None]
    D = np.stack([t @ e1, t @ e2], 1)
    return (ww[:, None, None] * D[:, :, None] * D[:, None, :]).sum(0), ww.sum()


POLAR = [(5, 29, 29, 0), (5, 24, 24, 0), (5, 19, 14, 0), (5, 24, 16, 1), (7, 125, 125, 0), (7, 67, 62, 0),
         (7, 120, 120, 2), (6, 3, 3, 9), (6, 8, 12, 11)]


@pytest.mark.parametrize("order,x,y,f", POLAR)
def test_polar_zone_window_is_isotropic_on_the_sphere(order, x, y, f):
    """In a polar cap the zone window weighs neighbours by great-circle
    distance: its second-moment tensor over the tangent-plane offsets has
    equal eigenvalues (ratio <= 1.07), where the chart window there is
    stretched (ratio >= 1.5: the rings compress the pixels), and its trace per
    unit weight is the 2 sigma^2 Omega of a sigma-pitch Gaussian, shortened
    a little by the 11 x 11 truncation (0.8 .. 1.0 of it)."""
    p = int(O.xyf2nest(order, np.array([x]), np.array([y]), np.array([f]))[0])
    z = O.pix_ringinfo(order, np.array([p]))[2][0]
    assert abs(z) > 2 / 3
    Mz, Sz = _tangent_moments(order, p, True)
    Mi, _ = _tangent_moments(order, p, False)
    ev_z = np.linalg.eigvalsh(Mz)
    ev_i = np.linalg.eigvalsh(Mi)
    assert ev_z[1] / ev_z[0] <= 1.07, ev_z
    assert ev_i[1] / ev_i[0] >= 1.5, ev_i
    omega = 4 * math.pi / O.npix(order)
    r = np.trace(Mz) / Sz / (2 * 1.5 ** 2 * omega)
    assert 0.8 <= r <= 1.0, r


def test_equatorial_zone_window_is_the_chart_window():
    """Equatorial-belt pixels (|z| <= 2/3, the ring at z = 2/3 included) keep
    exp(-(a^2 + b^2) / (2 sigma^2)) over chart offsets in zone mode; polar
    pixels get different weights, with weight 1 at their own centre."""
    order = 5
    N = 1 << order
    a = np.arange(-5, 6)
    chart = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2 * 1.5 ** 2))
    for (x, y, f) in [(16, 16, 5), (3, 28, 4), (N - 1, N - 1, 1), (0, 0, 0)]:
        p = int(O.xyf2nest(order, np.array([x]), np.array([y]), np.array([f]))[0])
        jr = O.pix_ringinfo(order, np.array([p]))[0][0]
        q, w = O.hssim_window(order, p, zones=True)
        q0, w0 = O.hssim_window(order, p, zones=False)
        assert np.array_equal(q, q0)
        assert np.array_equal(w0[q0 >= 0], chart[q0 >= 0])
        if N <= jr <= 3 * N:
            assert np.array_equal(w, w0), (x, y, f)
        else:
            assert w[5, 5] == 1.0 and np.abs(w - w0).max() > 0.05


def test_zone_hssim_identity_and_equatorial_map():
    """Zone mode: HSSIM(x, x) = 1 and constant images give 1; the SSIM map of
    equatorial pixels equals the isotropic one exactly, polar pixels differ."""
    order = 5
    act = np.arange(O.npix(order))
    rng = np.random.default_rng(4)
    x = rng.random((3, act.size)); y = rng.random((3, act.size))
    assert abs(O.hssim(order, act, x, x, zones=True)[0] - 1) < 1e-12
    c = np.full((3, act.size), 0.4)
    assert abs(O.hssim(order, act, c, c, zones=True)[0] - 1) < 1e-12
    _, mz, _ = O.hssim(order, act, x, y, want_map=True, zones=True)
    _, mi, _ = O.hssim(order, act, x, y, want_map=True)
    jr = O.pix_ringinfo(order, act)[0]
    N = 1 << order
    eq = (jr >= N) & (jr <= 3 * N)
    assert np.array_equal(mz[:, eq], mi[:, eq])
    assert np.abs(mz[:, ~eq] - mi[:, ~eq]).max() > 1e-3


@pytest.mark.parametrize("masked", [False, True])
def test_zone_hssim_gradient_fd(masked):
    """The backward through the non-separable polar windows (the transposed
    gather with each centre's own window) against central differences."""
    order = 3
    act = np.arange(O.npix(order))
    if masked:
        act = act[O.pix_vec(order, act)[:, 1] > -0.4]
    rng = np.random.default_rng(5)
    img = rng.random((3, act.size)); ref = rng.random((3, act.size))
    s, _, g = O.hssim(order, act, img, ref, want_grad=True, zones=True)
    jr = O.pix_ringinfo(order, act)[0]
    polar = np.nonzero((jr < 8) | (jr > 24))[0]
    idx = np.concatenate([rng.choice(polar, 20, replace=False), rng.choice(act.size, 10, replace=False)])
    h = 1e-6
    for p in idx:
        ch = int(rng.integers(3))
        xp = img.copy(); xp[ch, p] += h
        xm = img.copy(); xm[ch, p] -= h
        num = (O.hssim(order, act, xp, ref, zones=True)[0] - O.hssim(order, act, xm, ref, zones=True)[0]) / (2 * h)
        assert abs(num - g[ch, p]) < 1e-7 + 1e-5 * abs(g[ch, p])
