"""Pins of the oracle's image synthesis between the sphere and camera images
(Eq. camera_synthesis Interp_H; supp. camera models; supp. Eq.
supp_image_to_healpix): closed-form rays of each camera model, the ray /
projection round trip, agreement of the synthesis domain with the camera
mask, the interpolation's reproduction of pixel values at pixel centres and
of fields linear in colatitude or longitude, its second-order convergence,
and the bilinear image sampler's exactness on affine images."""
import math

import numpy as np
import pytest

import oracle as O

_POSE = dict(W=np.eye(3).reshape(-1).tolist(), b=[0.0, 0.0, 0.0], center=[0.0, 0.0, 0.0])
PIN = dict(_POSE, cam_type=2, fov_x=math.radians(70), fov_y=math.radians(45), order=6)
FISH = dict(_POSE, cam_type=1, fov_x=math.radians(210), fov_y=math.radians(170), order=6)
FULL = dict(_POSE, cam_type=0, fov_x=0.0, fov_y=0.0, order=6)


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def test_pinhole_rays_closed_form():
    W, H = 96, 60
    fx32, fy32 = float(np.float32(PIN["fov_x"])), float(np.float32(PIN["fov_y"]))
    tx, ty = math.tan(fx32 / 2), math.tan(fy32 / 2)
    uv = [[W / 2, H / 2], [W, H / 2], [0, H / 2], [W / 2, 0], [W, 0], [0, H]]
    d, ok = O.cam_rays(PIN, W, H, uv)
    assert ok.all()
    want = [_unit([0, 0, 1]), _unit([tx, 0, 1]), _unit([-tx, 0, 1]), _unit([0, ty, 1]),
            _unit([tx, ty, 1]), _unit([-tx, -ty, 1])]   # image top looks up (+y)
    assert np.abs(d - np.array(want)).max() < 1e-12


def test_fisheye_rays_closed_form():
    W, H = 80, 64
    fx32, fy32 = float(np.float32(FISH["fov_x"])), float(np.float32(FISH["fov_y"]))
    d, ok = O.cam_rays(FISH, W, H, [[W / 2, H / 2], [W, H / 2], [W / 2, 0], [0, H / 2]])
    assert ok.all()
    # incident angle at the ellipse's ends is half the field of view
    ang = np.arccos(np.clip(d[:, 2], -1, 1))
    assert abs(ang[0]) < 1e-12
    assert abs(ang[1] - fx32 / 2) < 1e-9 and abs(ang[3] - fx32 / 2) < 1e-9
    assert abs(ang[2] - fy32 / 2) < 1e-9
    assert d[1, 0] > 0 and abs(d[1, 1]) < 1e-12    # right: +x
    assert d[3, 0] < 0                              # left: -x
    assert d[2, 1] > 0 and abs(d[2, 0]) < 1e-12    # top: +y
    # outside the ellipse (image corner) is not in the domain
    _, ok2 = O.cam_rays(FISH, W, H, [[0.5, 0.5]])
    assert not ok2[0]


def test_panorama_rays_closed_form():
    W, H = 64, 32
    d, ok = O.cam_rays(FULL, W, H, [[W / 2, H / 2], [3 * W / 4, H / 2], [W / 4, H / 2], [W / 2, 0], [W / 2, H], [0, H / 2]])
    assert ok.all()
    want = [[0, 0, 1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, -1]]
    assert np.abs(d - np.array(want, np.float64)).max() < 1e-12


@pytest.mark.parametrize("cam,W,H", [(PIN, 96, 60), (FISH, 80, 64), (FULL, 64, 32)])
def test_ray_projection_round_trip(cam, W, H):
    rng = np.random.default_rng(5)
    uv = np.stack([rng.uniform(0, W, 4000), rng.uniform(0, H, 4000)], 1)
    d, ok = O.cam_rays(cam, W, H, uv)
    uv2, ok2 = O.cam_project(cam, W, H, d[ok])
    assert ok.sum() > 1000 and ok2.all()
    err = np.abs(uv2 - uv[ok])
    if cam["cam_type"] == 0:
        err[:, 0] = np.minimum(err[:, 0], W - err[:, 0])   # longitude wraps
    assert err.max() < 1e-8


@pytest.mark.parametrize("cam,W,H", [(PIN, 96, 60), (FISH, 80, 64), (FULL, 64, 32)])
def test_synthesis_domain_is_the_camera_mask(cam, W, H):
    """A HEALPix pixel is active (Sec. 3.1 mask) exactly when its centre
    projects into the camera's valid image domain."""
    order = cam["order"]
    allp = np.arange(O.npix(order))
    _, ok = O.cam_project(cam, W, H, O.pix_vec(order, allp))
    act = O.mask(cam)
    assert np.array_equal(np.flatnonzero(ok), act)


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_interp_reproduces_pixel_values_at_centres(order):
    p = np.arange(O.npix(order))
    pix, w = O.interp_weights(order, O.pix_vec(order, p))
    k = w.argmax(1)
    assert np.abs(w.max(1) - 1).max() < 1e-12
    assert np.array_equal(pix[np.arange(p.size), k], p)


def test_interp_weights_partition_of_unity_and_locality():
    order = 5
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pix, w = O.interp_weights(order, d)
    assert (w >= -1e-15).all()
    assert np.abs(w.sum(1) - 1).max() < 1e-12
    # every pixel with weight lies within two pixel sizes of the point
    pitch = math.sqrt(4 * math.pi / O.npix(order))
    v = O.pix_vec(order, pix.reshape(-1)).reshape(-1, 4, 3)
    ang = np.arccos(np.clip(np.einsum("nkc,nc->nk", v, d), -1, 1))
    assert ang[w > 1e-12].max() < 2.0 * pitch


def test_interp_linear_in_colatitude_between_rings():
    order = 4
    N = 1 << order
    p = np.arange(O.npix(order))
    v = O.pix_vec(order, p)
    theta_p = np.arctan2(np.hypot(v[:, 0], v[:, 2]), v[:, 1])  # colatitude from the pole (+y)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(5000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    th = np.arctan2(np.hypot(d[:, 0], d[:, 2]), d[:, 1])
    keep = (th > theta_p.min() + 1e-9) & (th < theta_p.max() - 1e-9)
    pix, w = O.interp_weights(order, d[keep])
    got = (w * theta_p[pix]).sum(1)
    assert np.abs(got - th[keep]).max() < 1e-12


def test_interp_linear_in_longitude_on_a_ring():
    order = 3
    p = np.arange(O.npix(order))
    jr, jp, z, phi = O.pix_ringinfo(order, p)
    rng = np.random.default_rng(3)
    for ring in (1, 3, 8, 12, 16, 21, 31):
        sel = np.flatnonzero(jr == ring)
        ph = np.sort(phi[sel])
        # points on the ring between two of its pixel centres, away from the wrap
        t = rng.uniform(ph[0] + 1e-6, ph[-1] - 1e-6, 50)
        zz = z[sel[0]]
        s = math.sqrt(1 - zz * zz)
        d = np.stack([s * np.sin(t), np.full_like(t, zz), s * np.cos(t)], 1)
        pix, w = O.interp_weights(order, d)
        _, _, _, phi_pix = O.pix_ringinfo(order, pix.reshape(-1))
        got = (w * phi_pix.reshape(-1, 4)).sum(1)
        assert np.abs(got - t).max() < 1e-10, ring


def test_interp_at_the_poles():
    for order in (2, 5):
        pix, w = O.interp_weights(order, [[0, 1, 0], [0, -1, 0]])
        assert np.abs(w - 0.25).max() < 1e-12
        jr, _, _, _ = O.pix_ringinfo(order, pix.reshape(-1))
        N = 1 << order
        assert set(jr[:4]) == {1} and set(jr[4:]) == {4 * N - 1}
        assert len(set(pix[0])) == 4 and len(set(pix[1])) == 4


def test_interp_convergence():
    """Second order away from the poles; first order inside the first ring
    around a pole, where the ring has only four pixels to interpolate along."""
    f = lambda v: np.sin(2 * v[:, 0]) + v[:, 1] ** 2 + 0.5 * v[:, 2]
    rng = np.random.default_rng(4)
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    far, cap = [], []
    for order in (4, 5, 6):
        vals = f(O.pix_vec(order, np.arange(O.npix(order))))
        pix, w = O.interp_weights(order, d)
        e = np.abs((w * vals[pix]).sum(1) - f(d))
        polar = np.abs(d[:, 1]) > 0.98          # within 11.5 degrees of a pole
        far.append(e[~polar].max())
        cap.append(e[polar].max())
    assert far[1] < far[0] / 3 and far[2] < far[1] / 3, far
    assert cap[1] < cap[0] / 1.6 and cap[2] < cap[1] / 1.6, cap


@pytest.mark.parametrize("cam,W,H", [(PIN, 96, 60), (FISH, 80, 64), (FULL, 64, 32)])
def test_sphere_to_image_constant_field(cam, W, H):
    act = O.mask(cam)
    img = np.tile(np.array([[0.25], [0.5], [0.75]]), (1, act.size))
    out, ok = O.sphere_to_image(cam, act, img, W, H)
    assert ok.sum() > 0.5 * ok.size if cam["cam_type"] != 1 else ok.sum() > 0.6 * ok.size
    assert np.abs(out[:, ok] - img[:, :1]).max() < 1e-12
    assert (out[:, ~ok] == 0).all()


@pytest.mark.parametrize("cam,W,H", [(PIN, 96, 60), (FULL, 64, 32)])
def test_image_to_sphere_exact_on_affine_images(cam, W, H):
    """Bilinear sampling reproduces an affine image exactly inside the
    pixel-centre hull."""
    act = O.mask(cam)
    jj, ii = np.mgrid[0:H, 0:W]
    u, v = ii + 0.5, jj + 0.5
    img = np.stack([2 * u + 3 * v, u - v, 0 * u + 1])
    out, ok = O.image_to_sphere(cam, act, img, W, H)
    uv, ok2 = O.cam_project(cam, W, H, O.pix_vec(cam["order"], act))
    assert ok.all() and ok2.all()
    inner = (uv[:, 0] > 0.5) & (uv[:, 0] < W - 0.5) & (uv[:, 1] > 0.5) & (uv[:, 1] < H - 0.5)
    assert inner.sum() > 0.8 * act.size
    assert np.abs(out[0, inner] - (2 * uv[inner, 0] + 3 * uv[inner, 1])).max() < 1e-9
    assert np.abs(out[1, inner] - (uv[inner, 0] - uv[inner, 1])).max() < 1e-9
    assert np.abs(out[2] - 1).max() < 1e-12


def test_round_trip_of_a_smooth_field():
    """sphere -> panorama -> sphere returns a smooth field up to the
    interpolation error, which shrinks with resolution."""
    f = lambda v: 0.5 + 0.3 * v[:, 0] * v[:, 2] + 0.2 * v[:, 1]
    errs = []
    for order, W in ((4, 128), (5, 256)):
        cam = dict(FULL, order=order)
        act = O.mask(cam)
        vals = np.tile(f(O.pix_vec(order, act)), (3, 1))
        im, ok = O.sphere_to_image(cam, act, vals, W, W // 2)
        back, ok2 = O.image_to_sphere(cam, act, im, W, W // 2)
        assert ok.all() and ok2.all()
        errs.append(np.abs(back - vals).max())
    assert errs[0] < 0.02 and errs[1] < errs[0] / 2.5, errs
