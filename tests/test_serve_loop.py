"""The continuous-batching loop on a fake device (no GPU): admission,
failure handling, cancellation and timeouts of serve.run_continuous."""
import threading
import time

import pytest

from paper_2606_29794_amd import _abi as A
from paper_2606_29794_amd.serve import (CANCELLED, ERROR, OK, TIMEOUT, BatchTimeout, Request, ServeStats,
                                        run_continuous)


def _reqs(n, gap=0.0, **kw):
    return [Request(k, k * gap, camera=None, **kw) for k in range(n)]


class Fake:
    """run_batch of a device that takes `dt` seconds per batch, records the
    bytes in flight, and fails or stalls on chosen requests."""

    def __init__(self, dt=0.01, est=10, fail=(), fatal=(), stall=None, hook=None):
        self.dt, self.est, self.fail, self.fatal, self.stall, self.hook = dt, est, set(fail), set(fatal), stall, hook
        self.lock = threading.Lock()
        self.in_flight = 0
        self.peak = 0
        self.batches = []

    def estimate(self, r):
        return self.est

    def run(self, batch, slot):
        with self.lock:
            self.in_flight += self.est * len(batch)
            self.peak = max(self.peak, self.in_flight)
            self.batches.append([r.rid for r in batch])
        try:
            if self.hook:
                self.hook(batch)
            if self.stall is not None and any(r.rid == 0 for r in batch):
                self.stall.wait(10)
            time.sleep(self.dt)
            ids = {r.rid for r in batch}
            if ids & self.fatal:
                raise A.HPError("hp_render_fwd_batch", A.HP_ERR_DEVICE, "device error")
            if ids & self.fail:
                raise ValueError(f"refused {sorted(ids & self.fail)}")
            return [(f"img{r.rid}", f"T{r.rid}") for r in batch]
        finally:
            with self.lock:
                self.in_flight -= self.est * len(batch)


def _run(fake, reqs, slots=3, budget=10**9, max_batch=4, **kw):
    return run_continuous(reqs, slots, fake.estimate, 0, budget, max_batch, fake.run, realtime=False, **kw)


def test_every_request_served_in_order_with_its_output():
    f = Fake()
    res, span = _run(f, _reqs(20))
    assert [r.rid for r in res] == list(range(20))
    assert all(r.status == OK and r.rgb == f"img{r.rid}" and r.T == f"T{r.rid}" for r in res)
    assert span > 0 and all(len(b) <= 4 for b in f.batches)
    st = ServeStats.of(res, span)
    assert st.n == 20 and st.failed == st.cancelled == st.timed_out == 0


def test_budget_bounds_bytes_in_flight():
    f = Fake(dt=0.02, est=40)
    res, _ = _run(f, _reqs(12), slots=4, budget=100)
    assert all(r.status == OK for r in res)
    assert f.peak <= 100


def test_failed_batch_fails_only_its_requests_and_serving_goes_on():
    f = Fake(fail={5})
    res, span = _run(f, _reqs(16), max_batch=2)
    bad = {r.rid for r in res if r.status == ERROR}
    batch_of_5 = next(b for b in f.batches if 5 in b)
    assert bad == set(batch_of_5)
    assert all("refused [5]" in r.error for r in res if r.status == ERROR)
    assert all(r.status == OK for r in res if r.rid not in bad)
    st = ServeStats.of(res, span)
    assert st.failed == len(bad) and st.renders_per_s == pytest.approx((16 - len(bad)) / span)


def test_device_error_stops_serving():
    f = Fake(fatal={3})
    with pytest.raises(A.HPError) as e:
        _run(f, _reqs(30), max_batch=2)
    assert e.value.status == A.HP_ERR_DEVICE


def test_cancelled_before_admission_is_dropped():
    gate = threading.Event()
    reqs = _reqs(6)
    f = Fake(stall=gate)
    out = {}

    def serve():
        out["res"] = _run(f, reqs, slots=1, max_batch=1)[0]

    th = threading.Thread(target=serve)
    th.start()
    time.sleep(0.1)            # request 0 holds the only slot
    reqs[3].cancel()
    gate.set()
    th.join(10)
    res = out["res"]
    assert res[3].status == CANCELLED and res[3].rgb is None
    assert all(r.status == OK for r in res if r.rid != 3)
    assert all(3 not in b for b in f.batches)


def test_cancelled_in_flight_discards_the_output():
    def hook(batch):
        for r in batch:
            if r.rid == 2:
                r.cancel()      # another thread withdraws it while it renders

    f = Fake(hook=hook)
    res, _ = _run(f, _reqs(5), max_batch=1)
    assert res[2].status == CANCELLED and res[2].rgb is None
    assert any(2 in b for b in f.batches)          # it did run
    assert all(r.status == OK for r in res if r.rid != 2)


def test_deadline_expires_while_waiting_for_admission():
    f = Fake(dt=0.3)
    reqs = _reqs(3)
    reqs[2].deadline = 0.1
    res, _ = _run(f, reqs, slots=1, max_batch=1)
    assert [r.status for r in res] == [OK, OK, TIMEOUT]
    assert all(2 not in b for b in f.batches)


def test_stalled_batch_raises_batch_timeout():
    gate = threading.Event()
    f = Fake(stall=gate)
    t = time.perf_counter()
    try:
        with pytest.raises(BatchTimeout):
            _run(f, _reqs(4), slots=2, max_batch=1, batch_timeout=0.2)
        assert time.perf_counter() - t < 5
    finally:
        gate.set()              # release the abandoned worker


def test_device_error_classification():
    from paper_2606_29794_amd.serve import device_error
    assert device_error(A.HPError("x", A.HP_ERR_DEVICE, "d"))
    assert not device_error(A.HPError("x", A.HP_ERR_INVALID_ARG, "d"))
    assert device_error(RuntimeError("HIP error: an illegal memory access was encountered"))
    assert not device_error(RuntimeError("tile lists exceed their buffer after a recount"))
    assert device_error(KeyboardInterrupt())


def test_lone_request_runs_inline_when_idle():
    """With inline_idle, a batch of one formed while nothing is in flight runs
    on the dispatcher's thread; a burst still goes to the workers."""
    main = threading.get_ident()
    where = {}

    class Where(Fake):
        def run(self, batch, slot):
            for r in batch:
                where[r.rid] = threading.get_ident()
            return super().run(batch, slot)

    f = Where(dt=0.01)
    reqs = [Request(k, 0.05 * k, camera=None) for k in range(4)]        # spaced: each alone
    res, _ = run_continuous(reqs, 2, f.estimate, 0, 10**9, 4, f.run, realtime=True, inline_idle=True)
    assert all(r.status == OK for r in res)
    assert all(where[k] == main for k in range(4))
    where.clear()
    f = Where(dt=0.05)
    res, _ = run_continuous(_reqs(9), 2, f.estimate, 0, 10**9, 4, f.run, realtime=False, inline_idle=True)
    assert all(r.status == OK for r in res)
    assert any(t != main for t in where.values())
