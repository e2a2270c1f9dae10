"""Continuous-batching render server over a device-resident Gaussian scene.

Requests (camera pose, camera model, field of view, HEALPix order) arrive
over time.  A dispatcher admits the requests that have arrived whenever a
stream slot is free and the HBM budget allows, and hands them as one batch
to that slot's worker thread:

  masks of the batch's cameras -> one preprocessing launch that reads every
  Gaussian once for all views -> per request: tile lists in per-tile depth
  order into a buffer sized from earlier counts -> one batched render launch
  for every (request, tile) pair of the batch.

Nothing in a batch waits for the host.  Batches on different slots overlap
on the device, and a worker waiting on its batch does not hold up the
others, so requests that arrive while others are on the GPU start as soon as
a slot and memory free up.  Latency is completion time minus arrival time;
the forward pass has no atomics, so a request renders bit-identically alone
or inside a batch.
"""
from __future__ import annotations

import collections
import ctypes as C
import math
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from .raster import Camera, Gaussians, MaskInfo, Rasterizer, _bytes, _p

MAX_VIEWS_PER_PREPROCESS = 8
MAX_REQ_PER_RENDER = 16


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds from the start of the trace
    camera: Camera
    deadline: float | None = None   # longest wait for admission, seconds after arrival
    cancelled: bool = False         # set by cancel(), from any thread

    def cancel(self) -> None:
        """Withdraw the request.  Before admission it is dropped; after, its
        render still runs (launched work is not recalled) but its output is
        discarded."""
        self.cancelled = True


# outcome of a request
OK, ERROR, CANCELLED, TIMEOUT = "ok", "error", "cancelled", "timeout"


@dataclass
class Result:
    rid: int
    arrival: float
    done: float
    rgb: torch.Tensor | None = None
    T: torch.Tensor | None = None
    status: str = OK
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Batch:
    reqs: list
    stream: torch.cuda.Stream
    event: torch.cuda.Event
    nbytes: int
    outs: list = field(default_factory=list)
    keep: list = field(default_factory=list)


def select_batch(pending, estimate, mem_in_use: int, budget: int, max_batch: int, gpu_busy: bool) -> list:
    """Admission policy: take requests from the front of `pending` (FIFO)
    while the batch has room and their estimated bytes fit the HBM budget.
    A request larger than the whole budget is admitted only when the GPU is
    otherwise idle (alone), so it cannot starve.  Removes the taken requests
    from `pending` and returns them."""
    batch = []
    est = 0
    while pending and len(batch) < max_batch:
        e = estimate(pending[0])
        if mem_in_use + est + e > budget:
            if batch or gpu_busy:
                break
        batch.append(pending.popleft())
        est += e
        if mem_in_use + est > budget:
            break
    return batch


class BatchTimeout(RuntimeError):
    """A batch did not complete within the serving loop's batch_timeout."""


def device_error(e: BaseException) -> bool:
    """Errors after which the device cannot be trusted and serving stops:
    the library's HP_ERR_DEVICE, a HIP runtime error surfaced by torch, and
    anything that is not an Exception (interrupts).  Other errors (a refused
    argument, a capacity the retry could not meet) fail only the batch that
    raised them."""
    if not isinstance(e, Exception):
        return True
    if isinstance(e, A.HPError):
        return e.status == A.HP_ERR_DEVICE
    msg = str(e)
    return isinstance(e, RuntimeError) and ("HIP error" in msg or "hipError" in msg)


def run_continuous(requests: list, n_slots: int, estimate, reserve: int, budget: int, max_batch: int, run_batch,
                   realtime: bool = True, fatal=device_error, batch_timeout: float | None = None,
                   worker_init=None, inline_idle: bool = False):
    """The continuous-batching loop, independent of the device.

    A dispatcher admits arrived requests (select_batch: FIFO, HBM budget)
    into a batch whenever one of n_slots worker threads is free; the worker
    calls run_batch(batch, slot), which returns one (rgb, T) pair per request
    once the batch has completed.  `estimate(request)` gives a request's
    bytes in flight and `reserve` the bytes held for the whole run.

    Failure handling:
    * a batch whose run_batch raises an error that `fatal` does not call
      fatal fails its own requests (status ERROR, with the message), its
      slot and bytes are released, and serving goes on;
    * a fatal error ends the loop and is raised;
    * a request cancelled before admission is dropped (CANCELLED); one
      cancelled while in flight is rendered but its output is discarded;
    * a request still waiting for admission `deadline` seconds after its
      arrival is dropped (TIMEOUT);
    * a batch in flight for longer than batch_timeout seconds ends the loop
      with BatchTimeout: the device is presumed hung, and its worker thread
      is left behind (daemon) rather than waited for.

    With inline_idle (and no batch_timeout), a batch of one request formed
    while nothing else is in flight runs on the dispatcher's own thread:
    under light load a request then starts as soon as it arrives, as in
    one-at-a-time serving, with no hand-over to a worker thread.

    Returns (results in request order, makespan in seconds)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    n = len(reqs)
    cv = threading.Condition()
    results = {}
    free = list(range(n_slots))
    busy = {}                      # slot -> time its batch was handed over
    st = {"mem": 0, "error": None}
    inbox = [queue.SimpleQueue() for _ in range(n_slots)]
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    arrival = (lambda r: r.arrival) if realtime else (lambda r: 0.0)

    def finish(r, status, t, rgb=None, T=None, error=None):
        # without real-time replay every request is queued at t = 0
        results[r.rid] = Result(r.rid, arrival(r), t, rgb, T, status, error)

    def execute(batch, est, slot) -> bool:
        """Runs one batch and records its results; False after a fatal error."""
        try:
            outs = run_batch(batch, slot)
            err = None
        except BaseException as e:
            if fatal(e):
                with cv:
                    st["error"] = e
                    cv.notify_all()
                return False
            outs, err = None, f"{type(e).__name__}: {e}"
        t = clock()
        with cv:
            for k, r in enumerate(batch):
                if err is not None:
                    finish(r, ERROR, t, error=err)
                elif r.cancelled:
                    finish(r, CANCELLED, t)
                else:
                    finish(r, OK, t, *outs[k])
            outs = None
            st["mem"] -= est
            busy.pop(slot, None)
            free.append(slot)
            cv.notify_all()
        return True

    def worker(slot):
        if worker_init is not None:
            worker_init()
        while True:
            item = inbox[slot].get()
            if item is None or not execute(*item, slot):
                return

    threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in range(n_slots)]
    for th in threads:
        th.start()
    pending = collections.deque()
    nxt = 0
    hung = False
    try:
        with cv:
            while len(results) < n and st["error"] is None:
                now = clock()
                while nxt < n and (not realtime or reqs[nxt].arrival <= now):
                    pending.append(reqs[nxt])
                    nxt += 1
                # withdrawn and expired requests leave the queue
                keep = collections.deque()
                for r in pending:
                    if r.cancelled:
                        finish(r, CANCELLED, now)
                    elif r.deadline is not None and now - arrival(r) > r.deadline:
                        finish(r, TIMEOUT, now)
                    else:
                        keep.append(r)
                pending = keep
                if batch_timeout is not None:
                    late = [k for k, ts in busy.items() if now - ts > batch_timeout]
                    if late:
                        hung = True
                        st["error"] = BatchTimeout(f"batch on slot {late[0]} still running after {batch_timeout} s")
                        break
                if pending and free:
                    batch = select_batch(pending, estimate, st["mem"] + reserve, budget, max_batch,
                                         len(free) < n_slots)
                    if batch:
                        est = sum(estimate(r) for r in batch)
                        st["mem"] += est
                        slot = free.pop(0)
                        busy[slot] = now
                        if inline_idle and batch_timeout is None and len(batch) == 1 and len(busy) == 1:
                            # nothing else in flight: the lone request runs
                            # here, without a hand-over to a worker thread
                            cv.release()
                            try:
                                execute(batch, est, slot)
                            finally:
                                cv.acquire()
                        else:
                            inbox[slot].put((batch, est))
                        continue
                # sleep until a batch completes or the next request arrives
                wait = 0.05
                if realtime and nxt < n:
                    wait = min(wait, max(0.0, reqs[nxt].arrival - clock()))
                if batch_timeout is not None and busy:
                    wait = min(wait, max(0.0, min(busy.values()) + batch_timeout - clock()) + 1e-3)
                cv.wait(timeout=wait)
    finally:
        for q in inbox:
            q.put(None)
        if not hung:
            for th in threads:
                th.join()
    if st["error"] is not None:
        raise st["error"]
    makespan = max((r.done for r in results.values()), default=0.0)
    return [results[r.rid] for r in reqs], makespan


def _percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


class Server:
    def __init__(self, gaussians: Gaussians, rasterizer: Rasterizer | None = None, max_batch: int = 8,
                 n_streams: int = 2, hbm_budget_bytes: int = 48 << 30, persistent: bool = False,
                 inline_idle: bool = False):
        if persistent:
            # hp_render_fwd_persistent is switched off in the library: its
            # launches did not end on MI355X and the cause is not known
            raise NotImplementedError("the persistent render launch is disabled; serve with persistent=False")
        self.g = gaussians
        self.R = rasterizer or Rasterizer(gaussians.mean.device)
        self.max_batch = min(max_batch, MAX_REQ_PER_RENDER)
        dev = self.g.mean.device
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
        self.budget = hbm_budget_bytes
        self.inline_idle = inline_idle

    # ---- memory accounting ---------------------------------------------------
    def _estimate(self, cam: Camera) -> int:
        """Device bytes one request holds while it is in flight, from the
        library's own sizes: its projected records (hp_projected_bytes), its
        list buffer (at most the capacity the binning will use: the hint of
        the camera model, else the largest count per active tile seen for
        its order and camera type over every tile of the sphere when its mask
        is not made yet), its tile ranges and its outputs (rgb, T,
        n_contrib).  The binning workspaces are held per stream and reserved
        from the budget up front (workspace_reserve)."""
        R, P = self.R, self.g.P
        npix = 12 << (2 * cam.order)
        ntile = 12 << (2 * max(0, cam.order - R.prm.tile_log2))
        with R._lock:
            m = R._masks.get(cam.mask_key(R.prm.tile_log2))
        # the mask's tile count when the camera model has one, else every tile
        cap = R.capacity_hint(P, cam, None, m.n_tiles if m is not None else ntile)
        if cap is None:
            cap = 64 * P   # before the first count of the order and camera type: a generous guess
        # + the allocator's rounding of the request's seven buffers (512 B each)
        return A.lib().hp_projected_bytes(P) + 4 * cap + 8 * ntile + 20 * npix + 7 * 512

    def workspace_reserve(self) -> int:
        """Held for the life of the server: one binning workspace per stream
        slot (at the largest order served)."""
        ws = max(A.lib().hp_bin_sorted_workspace_bytes(self.g.P, k, self.R.prm.tile_log2) for k in (7, 8, 9, 10))
        return len(self.streams) * ws

    def _launch(self, reqs: list, slot: int, keep: bool) -> _Batch:
        R, g = self.R, self.g
        P = g.P
        dev = g.mean.device
        prm = R.prm
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            sptr = C.c_void_p(stream.cuda_stream)
            for r in reqs:
                R.grid(r.camera.order)
            masks = [R.mask(r.camera).buf for r in reqs]
            nproj = A.lib().hp_projected_bytes(P)
            projs = [_bytes(nproj, dev) for _ in reqs]
            gs = g.struct()
            for s0 in range(0, len(reqs), MAX_VIEWS_PER_PREPROCESS):
                chunk = reqs[s0:s0 + MAX_VIEWS_PER_PREPROCESS]
                views = (A.hp_view * len(chunk))(*[r.camera.view() for r in chunk])
                ptrs = (C.c_void_p * len(chunk))(*[projs[s0 + k].data_ptr() for k in range(len(chunk))])
                A.call("hp_preprocess_batch", C.byref(gs), len(chunk), views, C.byref(prm), ptrs, nproj, sptr)
            # tile lists per request, into buffers sized from earlier counts of
            # the same camera model (the first request of a model reads its
            # count back once); the binning workspace of the slot's stream is
            # reused request after request (stream order)
            reqd = []
            outs = []
            keep_t = []
            counts = []
            nbytes = 0
            for k, r in enumerate(reqs):
                m = R.mask(r.camera)
                vals, ranges, cnt = R.bin_lists(projs[k], P, r.camera, track=False)
                rgb = torch.empty((3, max(m.n_active, 1)), dtype=torch.float32, device=dev)
                T = torch.empty(max(m.n_active, 1), dtype=torch.float32, device=dev)
                nc = torch.empty(max(m.n_active, 1), dtype=torch.int32, device=dev)
                rq = A.hp_render_req(projs[k].data_ptr(), P, vals.data_ptr(), ranges.data_ptr(), m.n_tiles,
                                     r.camera.order, m.buf.data_ptr(), m.n_active, rgb.data_ptr(), T.data_ptr(),
                                     nc.data_ptr())
                reqd.append(rq)
                outs.append((rgb[:, :m.n_active], T[:m.n_active]))
                keep_t.append((vals, ranges, nc))
                counts.append(cnt)
                nbytes += nproj + 4 * vals.numel() + 8 * m.n_tiles + 24 * m.n_active
            if len(reqs) == 1:
                # a lone request takes the single-view render (same kernel
                # body, without the batch's request table)
                r, m = reqs[0], R.mask(reqs[0].camera)
                vals, ranges, nc = keep_t[0]
                rgb, T = outs[0]
                v = r.camera.view()
                A.call("hp_render_fwd", _p(projs[0]), P, _p(vals), _p(ranges), m.n_tiles, C.byref(v), C.byref(prm),
                       _p(m.buf), m.n_active, _p(rgb), _p(T), _p(nc), None, None, sptr)
            else:
                for s0 in range(0, len(reqd), MAX_REQ_PER_RENDER):
                    chunk = reqd[s0:s0 + MAX_REQ_PER_RENDER]
                    arr = (A.hp_render_req * len(chunk))(*chunk)
                    A.call("hp_render_fwd_batch", len(chunk), arr, C.byref(prm), sptr)
            # the pair counts go to pinned host memory in the batch's stream
            # order, so they are readable once the batch's event completes
            host_counts = torch.empty(len(counts), dtype=torch.int64, pin_memory=True)
            if len(counts) == 1:
                host_counts.copy_(counts[0].dev[:1], non_blocking=True)
            else:
                host_counts.copy_(torch.stack([c.dev[0] for c in counts]), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        b = _Batch(reqs, stream, ev, nbytes, outs=outs)
        b.counts = counts
        b.host_counts = host_counts
        b.slot = slot
        b.keep = [projs, masks, keep_t]   # alive until the batch completes
        return b

    def _redo_overflowed(self, b: _Batch, keep: bool) -> _Batch:
        """After a batch completed: requests whose lists needed more entries
        than their buffers held rendered empty lists; their counts raise the
        capacity hints and they run again (once more at most)."""
        P = self.g.P
        redo = []
        # every count of the batch, copied to the host with the batch
        ns = b.host_counts.tolist()
        for k, (r, cnt, n) in enumerate(zip(b.reqs, b.counts, ns)):
            self.R.note_count(P, r.camera, None, n)
            if n > cnt.capacity:
                redo.append(k)
        if not redo:
            return b
        b2 = self._launch([b.reqs[k] for k in redo], b.slot, keep)
        b2.event.synchronize()
        for j, k in enumerate(redo):
            if b2.counts[j].overflowed:
                raise RuntimeError(f"request {b.reqs[k].rid}: tile lists exceed their buffer after a recount")
            b.outs[k] = b2.outs[j]
        b.keep.append(b2.keep)
        return b

    # ---- the request loop -----------------------------------------------------
    def serve(self, requests: list, realtime: bool = True, keep_outputs: bool = False,
              batch_timeout: float | None = None):
        """Continuous batching (run_continuous) with one worker thread per
        stream slot: a worker launches its batch (the pair-count read-backs
        inside block only that worker), waits for the batch's completion
        event and hands back its images.  Host waits release the interpreter
        lock, so while one worker waits the others keep the GPU fed."""
        dev = self.g.mean.device

        def run(batch, slot):
            b = self._launch(batch, slot, keep_outputs)
            b.event.synchronize()
            b = self._redo_overflowed(b, keep_outputs)
            # the batch's buffers go with this frame, before its bytes leave
            # the account
            return b.outs if keep_outputs else [(None, None)] * len(batch)

        torch.cuda.synchronize()
        results, makespan = run_continuous(
            requests, len(self.streams), lambda r: self._estimate(r.camera), self.workspace_reserve(), self.budget,
            self.max_batch, run, realtime=realtime, batch_timeout=batch_timeout,
            worker_init=lambda: torch.cuda.set_device(dev), inline_idle=self.inline_idle)
        return ServeStats.of(results, makespan)

    def serve_sequential(self, requests: list, realtime: bool = True, keep_outputs: bool = False):
        """Baseline: one request at a time, FIFO, the plain per-request
        pipeline (hp_preprocess, hp_bin_sorted, hp_render_fwd)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in reqs:
            if realtime:
                while time.perf_counter() - t0 < r.arrival:
                    time.sleep(min(1e-3, max(0.0, r.arrival - (time.perf_counter() - t0))))
            st = self.R.forward(self.g, r.camera)
            torch.cuda.synchronize()
            self.R.verify()
            t = time.perf_counter() - t0
            results.append(Result(r.rid, r.arrival if realtime else 0.0, t, st.rgb if keep_outputs else None,
                                  st.T if keep_outputs else None))
        makespan = max(x.done for x in results)
        return ServeStats.of(results, makespan)


@dataclass
class ServeStats:
    """Throughput and latency over the requests that rendered (status OK);
    the other outcomes are counted."""
    n: int
    makespan_s: float
    renders_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    results: list
    failed: int = 0
    cancelled: int = 0
    timed_out: int = 0

    @staticmethod
    def of(results, makespan):
        ok = [r for r in results if r.status == OK]
        lat = [r.latency * 1e3 for r in ok]
        count = lambda s: sum(r.status == s for r in results)
        return ServeStats(len(results), makespan, len(ok) / makespan if makespan > 0 else float("nan"),
                          _percentile(lat, 50), _percentile(lat, 99), float(np.mean(lat)) if lat else float("nan"),
                          results, count(ERROR), count(CANCELLED), count(TIMEOUT))

    def summary(self) -> dict:
        d = dict(n=self.n, makespan_s=self.makespan_s, renders_per_s=self.renders_per_s, p50_ms=self.p50_ms,
                 p99_ms=self.p99_ms, mean_ms=self.mean_ms)
        for k in ("failed", "cancelled", "timed_out"):
            if getattr(self, k):
                d[k] = getattr(self, k)
        return d


def requests_from_workload(wl, limit: int | None = None) -> list:
    cams = wl.cameras if limit is None else wl.cameras[:limit]
    arr = wl.extra["arrivals"]
    return [Request(k, float(arr[k]), Camera.from_dict(c)) for k, c in enumerate(cams)]
