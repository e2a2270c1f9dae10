"""The C ABI without a GPU: the library loads, exports every function that
include/hp.h declares, the Python binding names each of them, and argument
checks that happen on the host before any device work return their status."""
import ctypes as C
import os
import re

import numpy as np

from paper_2606_29794_amd import _abi as A

_HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hp.h")


def _declared():
    src = open(_HDR).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)   # comments name functions too
    return sorted(set(re.findall(r"^[A-Za-z_][\w \t\*]*?\b(hp_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    names = _declared()
    assert len(names) >= 30
    L = A.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_names_every_declared_function():
    missing = [n for n in _declared() if n not in A._PROTOS]
    assert not missing, missing


def test_status_strings():
    L = A.lib()
    L.hp_status_string.restype = C.c_char_p
    texts = {L.hp_status_string(s) for s in range(5)}
    assert len(texts) == 5 and all(t for t in texts)


def _view(order=6):
    W = np.eye(3, dtype=np.float32)
    return A.make_view(W, np.zeros(3, np.float32), np.zeros(3, np.float32), A.HP_CAM_FULL, 0.0, 0.0, order)


def _query(mode, f, order=6):
    L = A.lib()
    v = _view(order)
    prm = A.default_params()
    dummy = C.c_void_p(16)   # never dereferenced: the checks fail first
    return L.hp_bin_query(A.HP_BIN_ALL, mode, f, dummy, 10, C.byref(v), C.byref(prm), dummy, dummy, dummy, dummy, 1,
                          10, dummy, None, dummy, 1 << 20, None)


def test_bin_query_rejects_bad_mode_and_depth():
    """Mode outside {RING, NESTED}; f not a power of two, or deeper than the
    pixel order (f > B = 16, or f > Nside when the tile order is 0)."""
    inv = 1   # HP_ERR_INVALID_ARG
    assert _query(0, 4) == inv
    assert _query(3, 4) == inv
    for f in (0, 3, 6, 32, -4):
        assert _query(A.HP_QUERY_RING, f) == inv, f
    assert _query(A.HP_QUERY_NESTED, 8, order=2) == inv   # Nside 4: at most f = 4


def test_every_entry_point_checks_null_arguments_on_the_host():
    """Every hp_status entry point called with null pointers and zero sizes
    returns OK (nothing to do), INVALID_ARG or CAPACITY from its host-side
    checks, before any device work: a launch would fail here without a GPU
    and show up as HP_ERR_DEVICE."""
    L = A.lib()
    statuses = {}
    for name, (res, args) in A._PROTOS.items():
        if res is not C.c_int32 or name in ("hp_read_total",):
            continue
        vals = []
        for t in args:
            if t in (C.c_int32, C.c_int64, C.c_size_t):
                vals.append(t(0))
            else:
                vals.append(None)
        statuses[name] = int(getattr(L, name)(*vals))
    bad = {k: v for k, v in statuses.items() if v not in (0, 1, 3)}
    assert not bad, bad
    assert sum(v == 1 for v in statuses.values()) >= 15, statuses


def test_noalloc_backward_rejects_oversized_scene():
    """hp_render_bwd_noalloc's fixed accumulator array holds HP_NOALLOC_MAX_P
    Gaussians; a larger scene is refused on the host (HP_ERR_CAPACITY)."""
    W = np.eye(3, dtype=np.float32)
    v = A.make_view(W, np.zeros(3, np.float32), np.zeros(3, np.float32), A.HP_CAM_FULL, 0.0, 0.0, 6)
    g = A.hp_gaussians(A.HP_NOALLOC_MAX_P + 1, 0, 16, 16, 16, 16, 16)
    gg = A.hp_gaussians_grad(16, 16, 16, 16, 16)
    d = C.c_void_p(16)   # never dereferenced: the size check fails first
    prm = A.default_params()
    st = A.lib().hp_render_bwd_noalloc(C.byref(g), d, d, d, 1, C.byref(v), C.byref(prm), d, 1, d, d, d, None, None,
                                       C.byref(gg), None)
    assert st == A.HP_ERR_CAPACITY


def test_persistent_render_is_switched_off():
    """hp_render_fwd_persistent checks its arguments, then refuses every call
    (HP_ERR_UNSUPPORTED) without launching: the consumer is built but not
    run.  Its argument checks still come first."""
    L = A.lib()
    qn = L.hp_render_queue_bytes(1024)
    d = C.c_void_p(256)   # never dereferenced
    assert L.hp_render_fwd_persistent(d, qn, 512, 100, None) == A.HP_ERR_UNSUPPORTED
    assert L.hp_render_fwd_persistent(d, qn, 0, 100, None) == A.HP_ERR_INVALID_ARG
    assert L.hp_render_fwd_persistent(None, qn, 512, 100, None) == A.HP_ERR_INVALID_ARG
