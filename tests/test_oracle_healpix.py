"""Pins of the oracle's HEALPix geometry, charts and masks against closed forms
and invariants of the grid (Sec. 3.1; Gorski et al. 2005) -- no GPU."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("order", [0, 1, 2, 3, 5])
def test_npix_and_nested_roundtrip(order):
    N = 1 << order
    p = np.arange(O.npix(order))
    assert p.size == 12 * N * N                       # Npix = 12 Nside^2
    x, y, f = O.nest2xyf(order, p)
    assert x.min() >= 0 and x.max() < N and y.min() >= 0 and y.max() < N
    assert np.array_equal(O.xyf2nest(order, x, y, f), p)
    assert np.array_equal(f, p // (N * N))


@pytest.mark.parametrize("order", [1, 2, 4, 6])
def test_ring_bijection_and_ring_sizes(order):
    N = 1 << order
    p = np.arange(O.npix(order))
    r = O.nest2ring(order, p)
    assert np.array_equal(np.sort(r), p)              # a permutation of [0, Npix)
    jr, jp, z, phi = O.pix_ringinfo(order, p)
    counts = np.bincount(jr, minlength=4 * N)[1:]
    i = np.arange(1, 4 * N)
    expect = 4 * np.minimum(np.minimum(i, N), 4 * N - i)
    assert np.array_equal(counts, expect)
    # ring z closed forms
    for ring in [1, N - 1, N, 2 * N, 3 * N, 4 * N - 1]:
        if ring < 1:
            continue
        zz = z[jr == ring]
        if ring < N:
            zr = 1 - ring * ring / (3.0 * N * N)
        elif ring <= 3 * N:
            zr = 4.0 / 3 - 2.0 * ring / (3 * N)
        else:
            s = 4 * N - ring
            zr = -(1 - s * s / (3.0 * N * N))
        assert np.allclose(zz, zr, atol=1e-15)
    # ring ordering puts ring jr first and positions ascending within a ring
    inv = np.argsort(r)
    assert np.all(np.diff(jr[inv]) >= 0)


def test_base_pixel_centres():
    # Nside 1: faces 0-3 at z = 2/3, 4-7 on the equator, 8-11 at z = -2/3
    p = np.arange(12)
    jr, jp, z, phi = O.pix_ringinfo(0, p)
    assert np.allclose(z, np.repeat([2 / 3, 0, -2 / 3], 4))
    assert np.allclose(phi[:4], np.pi / 4 + np.arange(4) * np.pi / 2)
    assert np.allclose(phi[4:8], np.arange(4) * np.pi / 2)
    assert np.allclose(phi[8:], np.pi / 4 + np.arange(4) * np.pi / 2)
    # Nside 2, nested pixel 0 (face 0, x = y = 0): z = 1/3, phi = pi/4
    jr, jp, z, phi = O.pix_ringinfo(1, np.array([0]))
    assert abs(z[0] - 1 / 3) < 1e-15 and abs(phi[0] - np.pi / 4) < 1e-15


@pytest.mark.parametrize("order", [3, 5])
def test_ring_symmetries(order):
    """90-degree rotation about the pole maps the grid onto itself (ring
    position j -> j + n_r/4) and the N-S mirror maps ring i to 4N - i."""
    N = 1 << order
    p = np.arange(O.npix(order))
    jr, jp, z, phi = O.pix_ringinfo(order, p)
    key = {(a, b): (zz, pp) for a, b, zz, pp in zip(jr, jp, z, phi)}
    for (a, b), (zz, pp) in list(key.items())[:: max(1, len(key) // 3000)]:
        nr = 4 * min(a, N, 4 * N - a)
        b2 = (b - 1 + nr // 4) % nr + 1
        z2, p2 = key[(a, b2)]
        assert abs(z2 - zz) < 1e-15
        assert abs(((p2 - pp) % (2 * np.pi)) - np.pi / 2) < 1e-12
        zm, pm = key[(4 * N - a, b)]
        assert abs(zm + zz) < 1e-15 and abs(pm - pp) < 1e-12
    # equal spacing in longitude within every ring
    for a in [1, N // 2 or 1, N, 2 * N + 1]:
        ph = np.sort(phi[jr == a])
        nr = ph.size
        assert np.allclose(np.diff(ph), 2 * np.pi / nr, atol=1e-12)


@pytest.mark.parametrize("order", [2, 4])
def test_pixel_vectors_unit_and_frame(order):
    p = np.arange(O.npix(order))
    v = O.pix_vec(order, p)
    assert np.allclose(np.linalg.norm(v, axis=1), 1, atol=1e-15)
    jr, jp, z, phi = O.pix_ringinfo(order, p)
    # camera frame: pole = +y, longitude omega = atan2(t_x, t_z) = HEALPix phi
    assert np.allclose(v[:, 1], z, atol=1e-15)
    om = np.mod(np.arctan2(v[:, 0], v[:, 2]), 2 * np.pi)
    assert np.allclose(np.cos(om - phi), 1, atol=1e-12)


def _neighbours(order, p):
    x, y, f = O.nest2xyf(order, np.array([p]))
    out = {}
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            if a or b:
                out[(a, b)] = O.chart_pixel(order, int(f[0]), int(x[0]) + a, int(y[0]) + b)
    return out


@pytest.mark.parametrize("order", [1, 2, 3])
def test_neighbour_count_and_symmetry(order):
    """8 Npix - 24 neighbour links: the 24 pixels at the eight three-face
    vertices have 7 neighbours (Sec. 4.1); the relation is symmetric."""
    n = O.npix(order)
    total = 0
    seven = 0
    nbs = {}
    for p in range(n):
        nb = [q for q in _neighbours(order, p).values() if q >= 0]
        assert len(set(nb)) == len(nb) and p not in nb
        nbs[p] = set(nb)
        total += len(nb)
        seven += len(nb) == 7
        assert len(nb) in (7, 8)
    assert total == 8 * n - 24
    assert seven == 24
    for p, s in nbs.items():
        for q in s:
            assert p in nbs[q]


@pytest.mark.parametrize("order", [3, 4])
def test_chart_window_symmetric_offsets(order):
    """If q is p's chart neighbour at offset (a, b), then p is q's chart
    neighbour at an offset of the same length (11x11 windows)."""
    N = 1 << order
    rng = np.random.default_rng(0)
    ps = rng.choice(O.npix(order), size=120, replace=False)
    # include pixels at face corners and edges
    extra = []
    for f in range(12):
        for (x, y) in [(0, 0), (N - 1, 0), (0, N - 1), (N - 1, N - 1), (N - 1, N // 2), (N // 2, 0)]:
            extra.append(int(O.xyf2nest(order, [x], [y], [f])[0]))
    ps = np.concatenate([ps, extra])

    def window(p):
        x, y, f = O.nest2xyf(order, np.array([p]))
        d = {}
        for a in range(-5, 6):
            for b in range(-5, 6):
                q = O.chart_pixel(order, int(f[0]), int(x[0]) + a, int(y[0]) + b)
                if q >= 0:
                    d.setdefault(q, []).append(a * a + b * b)
        return d

    for p in ps:
        wp = window(int(p))
        for q, lens in wp.items():
            wq = window(q)
            assert int(p) in wq, (p, q)
            assert sorted(wq[int(p)]) == sorted(lens)


@pytest.mark.parametrize("order", [4, 5])
def test_chart_is_locally_affine(order):
    """Geometric pin of the face-extended chart: around every pixel, the
    directions of the window pixels follow u_p + a e_x + b e_y to first order,
    with e_x, e_y taken from the +-1 neighbours.  A wrongly rotated or mirrored
    face crossing puts pixels on the wrong side and fails this."""
    N = 1 << order
    pitch = math.sqrt(4 * math.pi / O.npix(order))
    pixels = []
    for f in range(12):
        for (x, y) in [(0, 0), (N - 1, 0), (0, N - 1), (N - 1, N - 1), (N - 2, 3), (2, N - 3), (N // 2, N - 1),
                       (N - 1, N // 2), (0, N // 2), (N // 2, 0)]:
            pixels.append((f, x, y))
    worst = 0.0
    for f, x, y in pixels:
        p = int(O.xyf2nest(order, [x], [y], [f])[0])
        up = O.pix_vec(order, [p])[0]

        def vec(a, b):
            q = O.chart_pixel(order, f, x + a, y + b)
            return None if q < 0 else O.pix_vec(order, [q])[0]

        vxp, vxm, vyp, vym = vec(1, 0), vec(-1, 0), vec(0, 1), vec(0, -1)
        ex = (vxp - vxm) / 2 if vxp is not None and vxm is not None else (vxp - up if vxp is not None else up - vxm)
        ey = (vyp - vym) / 2 if vyp is not None and vym is not None else (vyp - up if vyp is not None else up - vym)
        for a in range(-3, 4):
            for b in range(-3, 4):
                v = vec(a, b)
                if v is None:
                    continue
                pred = up + a * ex + b * ey
                err = np.linalg.norm(v - pred) / (pitch * max(1.0, math.hypot(a, b)))
                worst = max(worst, err)
    # Curvature and the 120-degree face corners at three-face vertices bend
    # the chart (worst about 0.95 here); a crossing without the right
    # rotation errs by about 7 pitches per unit offset.
    assert worst < 1.5, worst


def test_mask_full_and_fisheye_360():
    for cam_type, fx in [(0, 2 * math.pi), (1, 2 * math.pi)]:
        cam = dict(W=np.eye(3), b=np.zeros(3), center=np.zeros(3), cam_type=cam_type, fov_x=fx, fov_y=fx, order=3)
        m = O.mask(cam)
        assert np.array_equal(m, np.arange(O.npix(3)))


@pytest.mark.parametrize("fov_deg", [120.0, 180.0, 200.0])
def test_fisheye_mask_solid_angle(fov_deg):
    """Active pixels x Omega_pix ~= 2 pi (1 - cos theta) (Sec. 3.1 Omega_in)."""
    from paper_2606_29794_amd.scenes import random_rotation
    order = 6
    rng = np.random.default_rng(3)
    W = random_rotation(rng)
    th = math.radians(fov_deg) / 2
    cam = dict(W=W, b=np.zeros(3), center=np.zeros(3), cam_type=1, fov_x=2 * th, fov_y=2 * th, order=order)
    n = O.mask(cam).size
    om = 4 * math.pi / O.npix(order)
    expect = O.omega_in("fisheye", theta=th) / om
    # boundary pixels: about the perimeter length over the pitch
    perim = 2 * math.pi * math.sin(th) / math.sqrt(om)
    assert abs(n - expect) < 2 * perim


def test_pinhole_mask_solid_angle_and_config3_count():
    """Active pixels x Omega_pix ~= 4 asin(sin theta_x sin theta_y) (the
    perspective Omega_in of Sec. 3.1).  At the 60-degree 16:9 pinhole the
    count scales to about 2.48M pixels at Nside 2048."""
    from paper_2606_29794_amd.scenes import pinhole_fov_y
    fx = math.radians(60.0)
    fy = pinhole_fov_y(fx)
    order = 8
    cam = dict(W=np.eye(3), b=np.zeros(3), center=np.zeros(3), cam_type=2, fov_x=fx, fov_y=fy, order=order)
    n = O.mask(cam).size
    om = 4 * math.pi / O.npix(order)
    sa = O.omega_in("pinhole", theta_x=fx / 2, theta_y=fy / 2)
    assert abs(sa - 0.6202) < 1e-3
    assert abs(n * om - sa) / sa < 0.01
    n2048 = sa / (4 * math.pi / O.npix(11))
    assert 2.47e6 < n2048 < 2.49e6


def test_nside_rule_printed_values():
    """Sec. 3.1 rule N* = sqrt(4 pi W H / (12 Omega_in)); the paper's '31.9%
    fewer sampled pixels' for 6080x3040 ERP at the lower order (supp. cross-
    resolution discussion) pins k_L = 10 for that input."""
    k, kl, kh = O.orders_for(6080, 3040, O.omega_in("erp"))
    assert (kl, kh) == (10, 11)
    fewer = 1 - 12 * (1 << kl) ** 2 / (6080 * 3040)
    assert abs(fewer - 0.319) < 0.001
    # 3040x1520 ERP -> Ours(L) is Nside 512 and 1520x760 -> 256
    assert O.orders_for(3040, 1520, O.omega_in("erp"))[1] == 9
    assert O.orders_for(1520, 760, O.omega_in("erp"))[1] == 8
    # 1920x1080 pinhole, 60 deg horizontal FoV -> N* ~ 1871 -> Nside 2048
    fx = math.radians(30.0)
    fy = math.atan(math.tan(fx) * 9 / 16)
    n_star = O.nside_star(1920, 1080, O.omega_in("pinhole", theta_x=fx, theta_y=fy))
    assert 1860 < n_star < 1880
    assert O.orders_for(1920, 1080, O.omega_in("pinhole", theta_x=fx, theta_y=fy))[0] == 11
