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
