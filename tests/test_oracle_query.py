"""Pins of the oracle's paper-literal tile queries (Sec. 3.3; Alg. 2 NESTED
quadtree traversal, Alg. 3 RING sequential scan) and of its render over
given tile lists.

What fixes them, independently of the oracle's own formulas:
* RING, pixel level (tile order = query order): every pixel whose centre lies
  in the disc is reported, and nothing beyond one ring step (pi / (2 Nside))
  outside it; the exact set equals a construction in which the longitude
  half-width of Eq. ring_phi_range is found by bisection on true angular
  distances instead of the closed form; closed forms at the pole and for a
  radius of pi.
* NESTED: the set equals, by brute force, the tiles holding a node of order
  kt .. kt + log2 f whose centre lies in the disc (the traversal's reading);
  at f = 1 that is the tiles whose own centre lies in the disc.
* Both grow with the radius (the GPU parity brackets rely on it).
* The list render with the exact binning lists equals the brute-force render.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_29794_amd import scenes as SC


def _proj(om, ph, rs):
    n = len(om)
    z = np.zeros(n)
    return O.Projected(np.ones(n, np.int32), np.asarray(om, float), np.asarray(ph, float), np.ones(n),
                       np.zeros((3, n)), np.zeros((3, n)), np.asarray(rs, float), np.zeros((3, n)))


def _discs(rng, n, N):
    """Disc centres and radii: uniform centres plus poles, near-poles and the
    longitude seam; radii from a third of a pixel to beyond a hemisphere."""
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    om = np.arctan2(v[:, 0], v[:, 2])
    ph = np.arcsin(v[:, 1])
    special_ph = [0.5 * math.pi, -0.5 * math.pi, 0.5 * math.pi - 1e-3, -0.5 * math.pi + 2e-3, 0.0, 0.3]
    special_om = [0.0, 1.0, math.pi, -math.pi + 1e-4, math.pi - 1e-4, -2.0]
    om = np.concatenate([om, special_om])
    ph = np.concatenate([ph, special_ph])
    pitch = math.sqrt(math.pi / 3) / N
    rs = np.exp(rng.uniform(math.log(0.3 * pitch), math.log(2.2), size=om.size))
    return om, ph, rs


def _angles(order, om, ph):
    """Angle from (om, ph) to every pixel centre at `order`."""
    v = O.pix_vec(order, np.arange(O.npix(order)))
    u = np.array([math.cos(ph) * math.sin(om), math.sin(ph), math.cos(ph) * math.cos(om)])
    c = np.cross(v, u)
    return np.arctan2(np.linalg.norm(c, axis=1), v @ u)


def _sets(g, t, n):
    out = [set() for _ in range(n)]
    for a, b in zip(g.tolist(), t.tolist()):
        out[a].add(b)
    return out


def _pixel_level(mode, order, om, ph, rs):
    """Query at pixel level: tile order = query order = `order` (f = 1, B = 1)."""
    prm = O.params(tile_log2=0)
    act = np.arange(O.npix(order))
    g, t = O.query_tiles(mode, order, _proj(om, ph, rs), act, 1, prm=prm)
    return _sets(g, t, len(om))


@pytest.mark.parametrize("order", [2, 3, 5])
def test_ring_contains_disc_and_is_bounded(order):
    rng = np.random.default_rng(order)
    N = 1 << order
    om, ph, rs = _discs(rng, 60, N)
    S = _pixel_level(O.QUERY_RING, order, om, ph, rs)
    step = math.pi / (2 * N)
    for k in range(len(om)):
        a = _angles(order, om[k], ph[k])
        inside = set(np.nonzero(a <= rs[k] * (1 - 1e-9))[0].tolist())
        assert inside <= S[k], (k, sorted(inside - S[k])[:5])
        got = np.array(sorted(S[k]), np.int64)
        assert np.all(a[got] <= rs[k] + step + 1e-9), (k, float(a[got].max() - rs[k]), step)


def _bisect_halfwidth(ph_r, om, ph, r):
    """Largest x in [0, pi] with dist((ph_r, om + x), (ph, om)) <= r, by bisection
    on the true angle (monotone in x); None when even x = 0 is outside, pi when
    the whole ring is inside."""
    def dist(x):
        a = np.array([math.cos(ph_r) * math.sin(om + x), math.sin(ph_r), math.cos(ph_r) * math.cos(om + x)])
        b = np.array([math.cos(ph) * math.sin(om), math.sin(ph), math.cos(ph) * math.cos(om)])
        return math.atan2(np.linalg.norm(np.cross(a, b)), float(a @ b))
    if dist(0.0) > r:
        return None
    if dist(math.pi) <= r:
        return math.pi
    lo, hi = 0.0, math.pi
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if dist(mid) <= r:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("order", [2, 4])
def test_ring_equals_bisection_construction(order):
    """Alg. 3's set with Delta omega from bisection on true distances: the
    rings whose centre latitude lies within r_s of the disc's, and on each the
    pixels from floor to ceil of the window ends in pixel units."""
    rng = np.random.default_rng(10 + order)
    N = 1 << order
    om, ph, rs = _discs(rng, 40, N)
    S = _pixel_level(O.QUERY_RING, order, om, ph, rs)
    p = np.arange(O.npix(order))
    jr, jp, z, lon = O.pix_ringinfo(order, p)
    checked = 0
    for k in range(len(om)):
        want = set()
        fragile = False
        for ir in range(1, 4 * N):
            sel = np.nonzero(jr == ir)[0]
            zr = float(z[sel[0]])
            ph_r = math.asin(zr)
            lo_lat = max(-0.5 * math.pi, ph[k] - rs[k])
            hi_lat = min(0.5 * math.pi, ph[k] + rs[k])
            if not (math.sin(lo_lat) <= zr <= math.sin(hi_lat)):
                continue
            if abs(ph_r - ph[k]) > rs[k] - 1e-9 and abs(ph_r - ph[k]) < rs[k] + 1e-9:
                fragile = True
            x = _bisect_halfwidth(ph_r, om[k], ph[k], rs[k])
            if x is None:
                continue
            nr = sel.size
            pos = jp[sel] - 1                          # 0-based position along the ring
            om0 = float(lon[sel][pos == 0][0])        # longitude of the ring's first pixel
            if x >= math.pi:
                want.update(sel.tolist())
                continue
            a = (om[k] - x - om0) * nr / (2 * math.pi)
            b = (om[k] + x - om0) * nr / (2 * math.pi)
            if min(abs(a - round(a)), abs(b - round(b))) < 1e-7:
                fragile = True
            lo, hi = math.floor(a), math.ceil(b)
            ids = {(i % nr) for i in range(lo, hi + 1)}
            want.update(sel[np.isin(pos, list(ids))].tolist())
        if fragile:
            continue
        checked += 1
        assert S[k] == want, (k, sorted(S[k] ^ want)[:6])
    assert checked >= len(om) - 3


def test_ring_pole_and_full_sphere_closed_forms():
    order = 4
    N = 1 << order
    npx = O.npix(order)
    theta = np.array([0.05, 0.2, 0.7, 1.9, 3.0])
    S = _pixel_level(O.QUERY_RING, order, np.zeros(theta.size), np.full(theta.size, 0.5 * math.pi), theta)
    jr, jp, z, lon = O.pix_ringinfo(order, np.arange(npx))
    colat = np.arccos(np.clip(z, -1, 1))
    for k, r in enumerate(theta):
        want = set(np.nonzero(colat <= r)[0].tolist())
        assert S[k] == want
    S = _pixel_level(O.QUERY_RING, order, [0.3, -2.0], [0.1, -1.2], [math.pi, math.pi])
    assert S[0] == set(range(npx)) and S[1] == set(range(npx))
    del N


@pytest.mark.parametrize("order,fl", [(4, 0), (4, 1), (5, 2), (6, 2)])
def test_nested_equals_node_centre_brute_force(order, fl):
    """Alg. 2's tiles are those holding a node of order kt .. kt + fl whose
    centre lies in the disc (with PixRad bounding the descendant centres, the
    traversal prunes nothing else); kt = order - 2 here (B = 4)."""
    rng = np.random.default_rng(20 + order + fl)
    prm = O.params(tile_log2=2)
    kt = order - 2
    if kt + fl > order:
        pytest.skip("query deeper than the pixels")
    om, ph, rs = _discs(rng, 50, 1 << order)
    act = np.arange(O.npix(order))
    g, t = O.query_tiles(O.QUERY_NESTED, order, _proj(om, ph, rs), act, 1 << fl, prm=prm)
    S = _sets(g, t, len(om))
    angs = {o: None for o in range(kt, kt + fl + 1)}
    for k in range(len(om)):
        want = set()
        fragile = False
        for o in angs:
            a = _angles(o, om[k], ph[k])
            fragile |= bool(np.any(np.abs(a - rs[k]) < 1e-9))
            want.update((np.nonzero(a <= rs[k])[0] >> (2 * (o - kt))).tolist())
        if fragile:
            continue
        assert S[k] == want, (k, sorted(S[k] ^ want)[:6])
        if fl == 0:
            a = _angles(kt, om[k], ph[k])
            assert S[k] == set(np.nonzero(a <= rs[k])[0].tolist())


def test_pixrad_table():
    R = O.pixrad(6)
    assert R[6] == 0.0
    assert np.all(np.diff(R) < 0)
    # a node's descendants at the next order sit a fraction of a node away
    for o in range(6):
        assert 0.2 < R[o] * (1 << o) < 1.0
    # every base pixel's centre sees its farthest order-6 centre near a corner
    assert abs(R[0] - 0.84) < 0.05


@pytest.mark.parametrize("mode", [O.QUERY_RING, O.QUERY_NESTED])
def test_queries_grow_with_radius(mode):
    rng = np.random.default_rng(30 + mode)
    order = 6
    om, ph, rs = _discs(rng, 80, 1 << order)
    prm = O.params(tile_log2=2)
    act = np.arange(O.npix(order))
    pr = _proj(om, ph, rs)
    for f in (1, 2, 4):
        a = _sets(*O.query_tiles(mode, order, pr, act, f, prm=prm), len(om))
        b = _sets(*O.query_tiles(mode, order, pr, act, f, prm=prm, drs_rel=1e-3, drs_abs=1e-4), len(om))
        c = _sets(*O.query_tiles(mode, order, pr, act, f, prm=prm, drs_rel=-1e-3, drs_abs=-1e-4), len(om))
        for k in range(len(om)):
            assert c[k] <= a[k] <= b[k]


def test_query_respects_active_tiles():
    wl = SC.config1(P=3000, order=6)
    sc, cam = wl.scene, wl.cameras[0]
    act = O.mask(cam)
    pr = O.preprocess(sc, cam)
    ta = O.tile_active(cam["order"], act)
    for mode in (O.QUERY_RING, O.QUERY_NESTED):
        g, t = O.query_tiles(mode, cam["order"], pr, act, 2)
        assert g.size > 0 and np.all(ta[t] == 1)
        assert np.all(pr.valid[g] == 1)


def test_render_lists_with_exact_lists_equals_render():
    wl = SC.config1_fd("overlap")
    sc, cam = wl.scene, wl.cameras[0]
    act = O.mask(cam)
    pr = O.preprocess(sc, cam)
    g, t, m, inn = O.tile_sets(cam["order"], pr, act)
    lst, ranges = O.sorted_tile_lists(cam["order"], pr, g, t, inn)
    a = O.render(sc, cam, pr, act)
    b = O.render_lists(sc, cam, pr, lst, ranges, act)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
