"""Shared helpers of the GPU parity tests: run the HIP pipeline through the
C ABI, run the oracle on the same seeded inputs, compare under the stated
tolerances with fragile decisions excluded and counted."""
from __future__ import annotations

import math

import numpy as np

import oracle as O

# tolerances
COLOUR_ATOL = 1e-4
GRAD_REL = 1e-3
# a binning decision is fragile when the oracle's FP64 margin is within this
# band: float32 direction (~1e-7 rad), r_s (~1e-6 relative) and cap radius
# rounding on the GPU side
def bin_band(rs, R):
    return 2e-6 + 2e-5 * (rs + R)


def gpu_forward(R, wl_scene, cam_dict):
    import torch
    from paper_2606_29794_amd.raster import Camera, Gaussians
    g = Gaussians.from_scene(wl_scene)
    cam = Camera.from_dict(cam_dict)
    st = R.forward(g, cam)
    torch.cuda.synchronize()
    return g, cam, st


def gpu_tile_lists(R, st, order):
    """Per full tile id: list of Gaussian ids in GPU order."""
    act = st.mask.active_pix.cpu().numpy().astype(np.int64)
    kt = O.tile_order(order)
    tiles = np.unique(act >> (2 * (order - kt)))   # compact id = rank
    vals = st.vals[: max(st.n_pairs, 1)].cpu().numpy().astype(np.int64)[: st.n_pairs]
    ranges = st.ranges.cpu().numpy().astype(np.int64)
    out = {}
    for c, t in enumerate(tiles):
        a, b = ranges[c]
        out[int(t)] = vals[a:b]
    return out, tiles


def compare_tile_lists(R, st, wl_scene, cam, order, max_report=5):
    """Bit-exact comparison of tile membership (fragile pairs excluded) and of
    the per-tile front-to-back order.  Returns stats."""
    pr = O.preprocess(wl_scene, cam)
    act = O.mask(cam)
    tc, tr = O.tile_caps(order)
    g, t, m, inn = O.tile_sets(order, pr, act, caps=(tc, tr), report_band=1e-4)
    gl, tiles = gpu_tile_lists(R, st, order)
    gpu_pairs = set()
    for tt, lst in gl.items():
        for gg in lst:
            gpu_pairs.add((int(gg), tt))
    band = bin_band(pr.rs[g], tr[t])
    fragile = np.abs(m) <= band
    ora_in = {(int(a), int(b)) for a, b, i_, f_ in zip(g, t, inn, fragile) if i_ and not f_}
    ora_out_nonfrag = {(int(a), int(b)) for a, b, i_, f_ in zip(g, t, inn, fragile) if (not i_) and not f_}
    frag_pairs = {(int(a), int(b)) for a, b, f_ in zip(g, t, fragile) if f_}
    missing = ora_in - gpu_pairs
    extra = gpu_pairs - ora_in - frag_pairs
    assert not missing, f"{len(missing)} pairs missing on the GPU, e.g. {list(missing)[:max_report]}"
    assert not extra, f"{len(extra)} extra GPU pairs, e.g. {list(extra)[:max_report]}"
    assert not (gpu_pairs & ora_out_nonfrag)
    # order inside each tile: by (rho, id); near-ties of 4 float32 ulps either way
    bad = 0
    for tt, lst in gl.items():
        if lst.size < 2:
            continue
        rho = pr.rho[lst]
        d = np.diff(rho)
        tie = np.abs(d) <= 4 * np.spacing(rho[1:].astype(np.float32)).astype(np.float64)
        ok = (d > 0) | ((d == 0) & (np.diff(lst) > 0)) | tie
        bad += int((~ok).sum())
    assert bad == 0, f"{bad} order violations"
    return dict(pairs=len(gpu_pairs), fragile=len(frag_pairs))


def compare_render(rgb_g, T_g, rgb_o, T_o, frag, atol=COLOUR_ATOL):
    """Colour/T parity: atol on robust pixels, atol + fragile allowance on the
    others.  Returns (max error on robust pixels, number of fragile pixels)."""
    err = np.maximum(np.abs(rgb_g - rgb_o).max(axis=0), np.abs(T_g - T_o))
    robust = frag == 0
    worst = float(err[robust].max()) if robust.any() else 0.0
    assert worst <= atol, f"max colour/T error {worst:.3g} on robust pixels"
    assert np.all(err[~robust] <= atol + frag[~robust] + 1e-6)
    return worst, int((~robust).sum())


def qtol_for(scale_err=1.0):
    """Absolute band around q = 9 inside which the FP32 q may land on the
    other side: float32 offsets (~1e-7 rad) against footprints down to 1e-3 rad."""
    return 2e-3 * scale_err


def grad_compare(name, g_gpu, g_ref, rel=GRAD_REL):
    g_gpu = np.asarray(g_gpu, np.float64).ravel()
    g_ref = np.asarray(g_ref, np.float64).ravel()
    nref = np.linalg.norm(g_ref)
    if nref == 0:
        assert np.linalg.norm(g_gpu) == 0, name
        return 0.0
    e = np.linalg.norm(g_gpu - g_ref) / nref
    assert e <= rel, f"{name}: relative L2 error {e:.3g}"
    rms = math.sqrt(np.mean(g_ref ** 2))
    elem = np.abs(g_gpu - g_ref) <= rel * np.abs(g_ref) + rel * rms
    assert np.all(elem), f"{name}: {np.count_nonzero(~elem)} of {elem.size} elements beyond tolerance"
    return e
