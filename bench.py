#!/usr/bin/env python3
"""Benchmark of the HEALPix Gaussian rasterizer on one MI355X.

Workload (default): 1,000,000 SH-3 Gaussians (log-uniform radius 1..20 around
the origin), four full-sphere views at Nside 512 (3,145,728 pixels each) from
camera centres in a ball of radius 0.5; per view the forward render, the
L1 + HEALPix-SSIM loss against a seeded noise target and the full backward
to means, scales, rotations, opacities and SH (gradients accumulated over the
four views).  A step is those four views; renders/s counts views.

Prints ONE JSON line.  The optimiser update is not part of the measured
fwd+bwd render rate.  With --serve the line also carries the continuous-
batching serving latencies (p50/p99) of the request-stream workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector FMA issue: 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (non-packed)
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--P", type=int, default=1_000_000)
    ap.add_argument("--views", type=int, default=4)
    ap.add_argument("--order", type=int, default=9)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=3072)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement (one JSON line)")
    ap.add_argument("--profile-only", action="store_true", help="run warmup+steps without the extra passes")
    ap.add_argument("--no-queries", action="store_true", help="skip the paper-query (RING / NESTED x f) comparison")
    ap.add_argument("--prefetch-streams", type=int, default=2,
                    help="side streams that prepare later views during the step (0: none)")
    ap.add_argument("--query", default=None,
                    help="mode:f (ring:4, nested:4, ...): the timed steps use the paper's own tile query")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device (known bytes for scaling FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": 1 << 30, "copies": 3}))


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.serve_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serve_bench(args.serve_requests)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2606_29794_amd import scenes as SC
    from paper_2606_29794_amd import _abi as A
    from paper_2606_29794_amd.raster import Camera, Gaussians, Rasterizer
    from paper_2606_29794_amd.render import hssim_loss, render

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = SC.config2(P=args.P, n_views=args.views, order=args.order)
    R = Rasterizer(dev)
    cams = [Camera.from_dict(c) for c in wl.cameras]
    g0 = Gaussians.from_scene(wl.scene, dev)
    params = [t.clone().requires_grad_(True) for t in (g0.mean, g0.scale, g0.rot, g0.opacity, g0.sh)]
    m = R.mask(cams[0])
    targets = [torch.as_tensor(SC.target_image(wl.seed, v, m.n_active), device=dev) for v in range(len(cams))]

    g_det = Gaussians(*[p.detach() for p in params])

    inflight = []

    def step(query=None):
        for p in params:
            p.grad = None
        # preprocess + binning of every view on a side stream, overlapping the
        # rendering of the views before it
        pf = R.prefetch(g_det, cams, query, args.prefetch_streams) if args.prefetch_streams > 0 else None
        for v, cam in enumerate(cams):
            rgb, T = render(*params, cam, R, fused_grad=True, query=query, prepared=pf.get(v) if pf else None)
            loss, _ = hssim_loss(rgb, targets[v], cam, 0.2, R)
            loss.backward()
        # at most two steps in flight: the host waits for the previous step,
        # not this one, so the GPU has the next step queued when this one ends
        done = torch.cuda.Event()
        done.record()
        inflight.append(done)
        if len(inflight) > 1:
            inflight.pop(0).synchronize()
        # every finished view's list count against the capacity it ran with
        # (raises if a list buffer was too small; the capacities settle in the
        # warm-up); the rest are checked by the blocking verify after the loop
        R.verify(block=False)

    def drain():
        torch.cuda.synchronize()
        inflight.clear()
        R.verify()

    query = None
    if args.query:
        mode, f = args.query.split(":")
        query = (mode, int(f))
    for _ in range(args.warmup):
        step(query)
    drain()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(query)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    drain()
    ms_per_step = dt * 1e3 / args.steps
    renders_per_s = args.steps * len(cams) / dt

    out = {
        "metric": "fwd+bwd HEALPix renders/s, 1M Gaussians @ Nside 512; serve p50/p99 latency",
        "value": renders_per_s, "unit": "renders/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded, config-2 distributions)",
        "config": {"workload": f"cfg2: {args.P} SH-3 Gaussians, {len(cams)} full-sphere views at Nside "
                               f"{1 << args.order}, L1+HSSIM loss, fwd+bwd per view",
                   "views_per_step": len(cams), "n_active": m.n_active},
    }
    if query is not None:
        out["config"]["tile_query"] = args.query
    if not args.profile_only:
        out.update(kernel_breakdown(R, params, cams, targets, torch, A))
        # Gaussian-pixel evaluations per second over the whole fwd+bwd step (view 0's counts)
        out["gaussian_pixel_evaluations_per_s"] = out["evaluated_pixel_pairs"] * renders_per_s
        if not args.no_queries:
            out["tile_queries"] = query_bench(R, params, cams, targets, torch, step, drain, args.steps)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(wl, args.cpu_pixels)
        if not args.no_serve:
            out["serve"] = serve_in_child(args.serve_requests)
    print(json.dumps(out), flush=True)


def serve_in_child(n_requests):
    """The serving measurement in a process of its own (started as a child,
    so this process keeps its GPU state): it then starts from an empty
    allocator and a cold cache of camera models, as a server would."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--serve-only", "--serve-requests",
                        str(n_requests)], capture_output=True, text=True, timeout=900)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        raise RuntimeError(f"serving measurement failed (status {r.returncode}): {r.stderr[-2000:]}")
    return json.loads(lines[-1])


QUERIES = [("exact", None), ("ring_x1", ("ring", 1)), ("ring_x2", ("ring", 2)), ("ring_x4", ("ring", 4)),
           ("nested_x1", ("nested", 1)), ("nested_x2", ("nested", 2)), ("nested_x4", ("nested", 4))]


def query_bench(R, params, cams, targets, torch, step, drain, steps):
    """The paper's own tile queries (RING scan, NESTED traversal at search
    depth f) against the exact binning on view 0: binning time, pairs kept,
    and forward / backward render time over each query's lists (HIP events,
    median of 3); then whole training steps (all views, loss, fwd+bwd) with
    R x4 and D x4, the pair the paper's ablation times."""
    from paper_2606_29794_amd.raster import FwdState, Gaussians
    g = Gaussians(*[p.detach() for p in params])
    cam = cams[0]
    m = R.mask(cam)
    proj = R.preprocess(g, cam)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    up = torch.ones(1, device=g.mean.device)
    res = {}
    for name, q in QUERIES:
        tb, tf, tw = [], [], []
        for _ in range(3):
            e = [ev() for _ in range(6)]
            e[0].record()
            vals, ranges, cnt = R.bin_lists(proj, g.P, cam, q)
            e[1].record()
            e[2].record()
            rgb, T, nc = R.render_fwd(proj, g.P, vals, ranges, cam)
            e[3].record()
            _, _, dimg = R.ssim_loss(rgb, targets[0], cam, dL_dloss=up)
            st = FwdState(cam, m, proj, vals, ranges, cnt, rgb, T, nc, g.P)
            acc = torch.zeros((10, g.P), dtype=torch.float32, device=g.mean.device)
            e[4].record()
            R.backward_pixels(st, dimg, None, acc)
            e[5].record()
            torch.cuda.synchronize()
            tb.append(e[0].elapsed_time(e[1]))
            tf.append(e[2].elapsed_time(e[3]))
            tw.append(e[4].elapsed_time(e[5]))
        cand = cnt.value(0)
        n = cand if q is None else cnt.value(1)
        r = {"bin_ms": float(np.median(tb)), "render_fwd_ms": float(np.median(tf)),
             "render_bwd_ms": float(np.median(tw)), "pairs": int(n), "candidates": int(cand)}
        r["bin_render_ms"] = r["bin_ms"] + r["render_fwd_ms"] + r["render_bwd_ms"]
        res[name] = r
    # whole training steps with the two queries the ablation compares
    whole = {}
    for name, q in (("ring_x4", ("ring", 4)), ("nested_x4", ("nested", 4)), ("exact", None)):
        step(q)
        drain()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(q)
        torch.cuda.synchronize()
        whole[name] = (time.perf_counter() - t0) * 1e3 / steps
        drain()
    res["step_ms"] = whole
    res["nested_x4_over_ring_x4_step"] = whole["nested_x4"] / whole["ring_x4"]
    return res


def serve_bench(n_requests):
    """Config-4 serving trace: resident 2M SH-3 scene, Poisson arrivals at
    200 req/s, random pose / camera model / FoV / Nside per request.  The
    same trace runs through the continuous-batching server and through the
    sequential one-request-at-a-time pipeline; both replay arrivals in real
    time.  Latency = completion - arrival."""
    import torch
    from paper_2606_29794_amd import scenes as SC
    from paper_2606_29794_amd.raster import Gaussians, Rasterizer
    from paper_2606_29794_amd.serve import Server, requests_from_workload
    wl = SC.config4(n_requests=n_requests)
    g = Gaussians.from_scene(wl.scene)
    reqs = requests_from_workload(wl)
    def fresh():
        # every measured run starts from the same state: a new rasterizer
        # (no masks or list hints of the trace's camera models), warmed on
        # the trace's first 16 requests (grid tables of the four orders,
        # workspaces, the allocator)
        srv = Server(g, Rasterizer(), max_batch=8, n_streams=2, hbm_budget_bytes=64 << 30)
        srv.serve(reqs[:16], realtime=False)
        srv.serve_sequential(reqs[:16], realtime=False)
        torch.cuda.synchronize()
        return srv

    # throughput: the whole backlog queued at t = 0 (the server is never idle)
    n_sat = min(len(reqs), 600)
    sat_b = fresh().serve(reqs[:n_sat], realtime=False)
    sat_s = fresh().serve_sequential(reqs[:n_sat], realtime=False)
    # latency: the trace replayed at its arrival times
    batched = fresh().serve(reqs, realtime=True)
    seq = fresh().serve_sequential(reqs, realtime=True)
    return {"workload": f"cfg4: 2M SH-3 Gaussians resident, {n_requests} requests, Poisson 200 req/s, "
                        "pinhole 60-90 / fisheye 180-220 / full sphere, Nside 128-1024",
            "saturated": {"n": n_sat, "batched": sat_b.summary(), "sequential": sat_s.summary(),
                          "speedup": sat_b.summary()["renders_per_s"] / sat_s.summary()["renders_per_s"]},
            "realtime": {"batched": batched.summary(), "sequential": seq.summary()}}


def kernel_breakdown(R, params, cams, targets, torch, A):
    """One instrumented view: HIP events (torch's current stream, the stream
    every call is issued on) around each stage; algorithmic work per stage.
    Each stage runs REPS times back to back between its two events, behind
    a ~0.1 ms fill kernel queued first, so that the timed span holds the
    stage's GPU work and not the host's launch latency (which the GPU would
    otherwise sit idle through)."""
    from paper_2606_29794_amd.raster import FwdState, Gaussians
    g = Gaussians(*[p.detach() for p in params])
    cam = cams[0]
    dev = g.mean.device
    ev = lambda: torch.cuda.Event(enable_timing=True)
    filler = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    times = {}
    REPS = 4

    def timed(name, fn):
        filler.fill_(0.0)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(REPS):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        times.setdefault(name, []).append(e0.elapsed_time(e1) / REPS)
        return out

    up = torch.ones(1, device=dev)
    z = torch.zeros_like
    for _ in range(3):
        proj = timed("preprocess", lambda: R.preprocess(g, cam))
        m = R.mask(cam)
        vals, ranges, cnt = timed("bin_and_sort", lambda: R.bin_lists(proj, g.P, cam))
        rgb, T, nc, nu = timed("render_fwd", lambda: R.render_fwd(proj, g.P, vals, ranges, cam, want_used=True))
        _, _, dimg = timed("ssim_fwd_bwd", lambda: R.ssim_loss(rgb, targets[0], cam, dL_dloss=up))
        st = FwdState(cam, m, proj, vals, ranges, cnt, rgb, T, nc, g.P)
        gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
        acc = torch.zeros((10, g.P), dtype=torch.float32, device=dev)
        timed("render_bwd", lambda: R.backward_pixels(st, dimg, None, acc))  # k_render_bwd alone
        timed("preprocess_bwd", lambda: R.backward_preprocess(g, cam, acc, gr))
    R.verify()
    med = {k: float(np.median(v)) for k, v in times.items()}
    n = cnt.value(0)
    evals = int(nc.to(torch.int64).sum().item())
    used = int(nu.to(torch.int64).sum().item())
    P = g.P
    K = g.sh.shape[0]
    # algorithmic bytes: preprocess reads the Gaussian SoA (mean 3, scale 3,
    # rot 4, opacity 1, SH 3K floats) and writes a 64 B record, depth, radius
    # and the 16 B disc entry the binning reads
    pre_bytes = P * (4 * (11 + 3 * K) + 88)
    res = {
        "stage_ms": med,
        "pairs": n,
        "evaluated_pixel_pairs": evals,
        "composited_pixel_pairs": used,
        "roofline": {
            "bound": "alu", "kernel": "k_render_bwd",
            "achieved": None, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s", "frac": None, "traffic": None,
        },
        "stage_roofline": {
            "preprocess_GBs": pre_bytes / (med["preprocess"] * 1e-3) / 1e9,
        },
    }
    # algorithmic flops (FMA = 2) per pixel-Gaussian pair:
    # every evaluated pair: offset projections a, b and the Mahalanobis bound
    # qt (21 flop); every composited pair in addition: c, the distance factor,
    # q, alpha and the compositing update (33 flop) in the forward, and the
    # recomputation plus gradient terms (93 flop) in the backward
    fwd_flops = 21 * evals + 33 * used
    bwd_flops = 21 * evals + 93 * used
    res["roofline"]["achieved"] = bwd_flops / (med["render_bwd"] * 1e-3) / 1e12
    res["roofline"]["frac"] = res["roofline"]["achieved"] / PEAK_VALU_TFLOPS
    res["roofline"]["traffic"] = measured_traffic("paper_2606_29794_amd/csrc/k_render.hip",
                                                  "profiles/k_render_bwd_cfg2_counters.md")
    res["roofline"]["flop_per_launch"] = bwd_flops
    # the packed-FP32 peak, which this build does not use (packed FP32 is disabled)
    res["roofline"]["frac_of_packed_fp32_peak"] = res["roofline"]["achieved"] / (2 * PEAK_VALU_TFLOPS)
    res["stage_roofline"]["render_fwd_TFLOPs"] = fwd_flops / (med["render_fwd"] * 1e-3) / 1e12
    # whole-view roofline: per stage the ideal time is its algorithmic bytes at
    # the HBM peak or its algorithmic flops at the VALU peak; the fraction is
    # the sum of ideal times over the sum of measured stage times
    n_act = int(m.n_active)
    ideal_s = {
        "preprocess": pre_bytes / (PEAK_HBM_GBS * 1e9),
        # count/scan per Gaussian, 12 B per emitted pair, one read + write of
        # 12 B key/value per pair for the ordering, 8 B of range per tile
        "bin_and_sort": (24 * P + 36 * n + 8 * int(m.n_tiles)) / (PEAK_HBM_GBS * 1e9),
        "render_fwd": fwd_flops / (PEAK_VALU_TFLOPS * 1e12),
        # image and reference read, gradient written: 36 B per active pixel;
        # separable 11-tap window sums (two passes) of the weight and 5
        # statistics x 3 channels in the forward (16 x 22 FMA = 704 flop), of
        # 3 gradient partials x 3 channels in the backward (396 flop), plus
        # the per-pixel SSIM algebra (~90 flop)
        "ssim_fwd_bwd": max(36 * n_act / (PEAK_HBM_GBS * 1e9), 1190 * n_act / (PEAK_VALU_TFLOPS * 1e12)),
        "render_bwd": bwd_flops / (PEAK_VALU_TFLOPS * 1e12),
        # accumulators read, parameters read, gradients read and written
        "preprocess_bwd": P * (4 * 9 + 3 * 4 * (11 + 3 * K)) / (PEAK_HBM_GBS * 1e9),
    }
    res["overall_roofline"] = {
        "ideal_ms": 1e3 * sum(ideal_s.values()),
        "measured_ms": sum(med[k] for k in ideal_s),
        "frac": 1e3 * sum(ideal_s.values()) / sum(med[k] for k in ideal_s),
        "per_stage_frac": {k: 1e3 * v / med[k] for k, v in ideal_s.items()},
    }
    return res


def measured_traffic(kernel_src: str, summary: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes, scaled by the copy-kernel
    calibration), or None when the kernel source has changed since the
    counters were taken (the summary records the source's SHA-256)."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, summary)).read()
        src = open(os.path.join(ROOT, kernel_src), "rb").read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(wl, n_pix):
    """The FP64 oracle on the host: preprocessing of all Gaussians plus
    forward and backward at a bounded sample of pixels of view 0, scaled to
    one full fwd+bwd render."""
    import oracle as O
    sc, cam = wl.scene, wl.cameras[0]
    O.build()
    threads = O.num_threads()
    t0 = time.perf_counter()
    pr = O.preprocess(sc, cam)
    t1 = time.perf_counter()
    npix = O.npix(cam["order"])
    rng = np.random.default_rng(0)
    pix = np.sort(rng.choice(npix, size=n_pix, replace=False))
    rgb, T, nu, fr = O.render(sc, cam, pr, pix)
    t2 = time.perf_counter()
    dC = np.ones((3, n_pix))
    O.render_bwd(sc, cam, pr, pix, dC, None)
    t3 = time.perf_counter()
    per_px = (t3 - t1) / n_pix
    full = (t1 - t0) + per_px * npix
    # the same on one core, over a sample 16x smaller (about as long)
    n1 = max(16, n_pix // 16)
    O.set_threads(1)
    try:
        s0 = time.perf_counter()
        pr1 = O.preprocess(sc, cam)
        s1 = time.perf_counter()
        O.render(sc, cam, pr1, pix[:n1])
        O.render_bwd(sc, cam, pr1, pix[:n1], np.ones((3, n1)), None)
        s2 = time.perf_counter()
    finally:
        O.set_threads(threads)
    full1 = (s1 - s0) + (s2 - s1) / n1 * npix
    return {"value": 1.0 / full, "unit": "renders/s", "cores": threads, "kind": "oracle",
            "sample": f"view 0: preprocess of all {sc.P} Gaussians ({t1 - t0:.2f} s) + brute-force fwd+bwd at "
                      f"{n_pix} random pixels ({t3 - t1:.2f} s), extrapolated to {npix} pixels",
            "single_core": {"value": 1.0 / full1, "unit": "renders/s", "cores": 1,
                            "sample": f"the same on one thread: preprocess ({s1 - s0:.2f} s) + fwd+bwd at the first "
                                      f"{n1} of those pixels ({s2 - s1:.2f} s), extrapolated"}}


if __name__ == "__main__":
    main()
