"""Host-side tests of the serving admission policy (no GPU)."""
import collections

from paper_2606_29794_amd.serve import select_batch


def _q(*sizes):
    return collections.deque(sizes)


def test_fifo_and_batch_limit():
    q = _q(1, 2, 3, 4, 5)
    b = select_batch(q, lambda r: 10, 0, 1000, 3, False)
    assert b == [1, 2, 3] and list(q) == [4, 5]


def test_budget_stops_admission_and_keeps_order():
    q = _q("a", "b", "c")
    est = {"a": 40, "b": 70, "c": 5}.get
    b = select_batch(q, est, 0, 100, 8, True)
    assert b == ["a"] and list(q) == ["b", "c"]       # c would fit but waits its turn (FIFO)
    b = select_batch(q, est, 30, 100, 8, True)
    assert b == ["b"] and list(q) == ["c"]


def test_budget_exhausted_waits_while_busy():
    q = _q("big")
    b = select_batch(q, lambda r: 80, 50, 100, 8, True)
    assert b == [] and list(q) == ["big"]


def test_oversize_request_runs_alone_when_idle():
    q = _q("huge", "small")
    b = select_batch(q, {"huge": 500, "small": 1}.get, 0, 100, 8, False)
    assert b == ["huge"] and list(q) == ["small"]
    # while something is on the GPU it is not admitted
    q = _q("huge")
    assert select_batch(q, lambda r: 500, 0, 100, 8, True) == []


def test_empty_queue():
    assert select_batch(_q(), lambda r: 1, 0, 10, 4, False) == []


def test_mask_header_check():
    """Buffers are sized from a mask's (n_active, n_tiles); a header outside
    the grid, or with more active pixels than its tiles hold (or tiles
    without one), is refused."""
    import pytest
    from paper_2606_29794_amd.raster import check_mask_counts
    check_mask_counts(9, 4, 12 << 18, 12 << 10)          # full sphere at Nside 512
    check_mask_counts(2, 4, 192, 12)                     # order below the tile side: a tile is a face
    check_mask_counts(6, 4, 0, 0)                        # empty
    for bad in [(9, 4, (12 << 18) + 1, 12 << 10), (9, 4, 100, -1), (9, 4, -5, 0),
                (9, 4, 300, 1), (9, 4, 3, 5), (6, 4, 10, (12 << 4) + 1)]:
        with pytest.raises(RuntimeError):
            check_mask_counts(*bad)


def test_camera_model_caches_are_bounded():
    """The per-camera-model caches drop their oldest entries (and those
    entries' ready events) beyond CACHE_MODELS; what is in flight keeps its
    own references."""
    import threading
    from paper_2606_29794_amd.raster import Rasterizer
    R = Rasterizer.__new__(Rasterizer)      # the cache logic only: no device
    R._ready = {}
    R._lock = threading.RLock()
    cache = {}
    n = Rasterizer.CACHE_MODELS + 10
    for k in range(n):
        key = (7, 2, float(k), 0.0, 4)
        cache[key] = object()
        R._ready[("mask",) + key] = "event"
        R._evict(cache, ("mask",))
    assert len(cache) == Rasterizer.CACHE_MODELS
    assert (7, 2, 0.0, 0.0, 4) not in cache and (7, 2, float(n - 1), 0.0, 4) in cache
    assert len(R._ready) == Rasterizer.CACHE_MODELS
