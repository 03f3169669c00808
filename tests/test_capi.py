"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "im.h")
LIB = os.path.join(ROOT, "paper_2408_10982_amd", "libim.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(im_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for f in ("im_sample_rrr", "im_greedy_cover", "im_randgreedi", "im_stream_cover",
              "im_solve", "im_build_incidence", "im_prepare_graph"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(L, name), name
    L.im_version.restype = ctypes.c_char_p
    assert b"gfx950" in L.im_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_binding_exports_match_header():
    import paper_2408_10982_amd as im
    assert sorted(im.EXPORTS) == _declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_invalid_arguments_rejected_before_device_work():
    """IM_EINVAL comes back before any HIP call, so this runs without a GPU."""
    L = ctypes.CDLL(LIB)
    L.im_greedy_cover.restype = ctypes.c_int
    # k = 0 is invalid
    z = ctypes.c_size_t(0)
    st = L.im_greedy_cover(ctypes.c_int32(10), ctypes.c_int64(5), None, None, ctypes.c_int64(0),
                           None, None, ctypes.c_int32(0), None, None, None, None, None, z, None)
    assert st == -1
    L.im_stream_cover.restype = ctypes.c_int
    st = L.im_stream_cover(ctypes.c_int32(10), ctypes.c_int64(5), None, None, ctypes.c_int32(3),
                           ctypes.c_int32(2), None, None, None, ctypes.c_double(0.7),
                           ctypes.c_double(1.0), None, None, None, None, None, z, None)
    assert st == -1
    L.im_sample_rrr.restype = ctypes.c_int
    st = L.im_sample_rrr(None, ctypes.c_uint64(0), ctypes.c_uint32(0), ctypes.c_int64(0),
                         ctypes.c_int64(1), None, None, ctypes.c_int64(0), None, None, None, z,
                         None)
    assert st == -1


class _WsShape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("model", ctypes.c_int32), ("count", ctypes.c_int64),
                ("total", ctypes.c_int64), ("k", ctypes.c_int32), ("m", ctypes.c_int32),
                ("delta", ctypes.c_double), ("selector", ctypes.c_int32),
                ("ntasks", ctypes.c_int32), ("full", ctypes.c_int32), ("num_cus", ctypes.c_int32)]


def _ws_lib():
    L = ctypes.CDLL(LIB)
    L.im_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(_WsShape),
                                    ctypes.POINTER(ctypes.c_size_t)]
    L.im_workspace_need.argtypes = [ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]
    L.im_last_error.restype = ctypes.c_char_p
    return L


def _ws_size(L, op, **kw):
    kw.setdefault("num_cus", 256)
    sh = _WsShape(**kw)
    b = ctypes.c_size_t()
    assert L.im_workspace_size(op, ctypes.byref(sh), ctypes.byref(b)) == 0
    return b.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_workspace_sizes_host_only():
    """im_workspace_size is host arithmetic (num_cus given): it grows with
    the problem, a full-speed workspace is at least the least one, and bad
    shapes are rejected."""
    L = _ws_lib()
    WS_SAMPLE, WS_INCIDENCE, WS_GREEDY, WS_RANDGREEDI, WS_STREAM, WS_SOLVE = 1, 2, 3, 4, 5, 9
    a = _ws_size(L, WS_SAMPLE, n=1 << 20, model=1, count=1 << 16, total=1 << 20)
    b = _ws_size(L, WS_SAMPLE, n=1 << 20, model=1, count=1 << 17, total=1 << 21)
    assert 0 < a < b
    # staging: 4 bytes per member of capacity at least
    assert a >= 4 * (1 << 20)
    lo = _ws_size(L, WS_SAMPLE, n=1 << 22, model=0, count=1 << 20, total=1 << 24)
    hi = _ws_size(L, WS_SAMPLE, n=1 << 22, model=0, count=1 << 20, total=1 << 24, full=1)
    assert hi > lo and hi <= lo + (17 << 30)
    assert _ws_size(L, WS_INCIDENCE, n=1 << 20, total=1 << 28, full=1) > \
        _ws_size(L, WS_INCIDENCE, n=1 << 20, total=1 << 28)
    assert _ws_size(L, WS_GREEDY, n=1000, count=5000, k=10) >= 4 * 1000 + 5000 + 80
    assert _ws_size(L, WS_RANDGREEDI, n=1000, count=5000, k=10, m=8) >= 12 * 1000 + 8 * 5000
    assert _ws_size(L, WS_STREAM, n=1000, count=5000, k=10, m=8, delta=0.077) > 0
    g = _ws_size(L, WS_SOLVE, n=1 << 16, model=0, count=1 << 16, total=1 << 20, k=50,
                 selector=1, m=8, delta=0.077)
    assert g > 4 * (1 << 20) + 8 * (1 << 16)
    b = ctypes.c_size_t()
    bad = _WsShape(n=100, count=-1, num_cus=256)
    assert L.im_workspace_size(3, ctypes.byref(bad), ctypes.byref(b)) == -1
    assert L.im_workspace_size(12, ctypes.byref(_WsShape(n=1, num_cus=256)), ctypes.byref(b)) == -1
    # GreediRIS sizes need a valid delta
    assert L.im_workspace_size(5, ctypes.byref(_WsShape(n=10, count=10, k=4, m=2, num_cus=256)),
                               ctypes.byref(b)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_short_workspace_rejected_before_device_work():
    """A workspace below a call's minimum returns IM_ENOMEM before any HIP
    call (so this runs without a GPU), and im_workspace_need then reports
    the bytes im_workspace_size gives for the same shape."""
    L = _ws_lib()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the call stops first
    need = ctypes.c_size_t()
    n, count, k, m = 1000, 5000, 10, 8
    L.im_greedy_cover.restype = ctypes.c_int
    st = L.im_greedy_cover(ctypes.c_int32(n), ctypes.c_int64(count), fake, fake,
                           ctypes.c_int64(100), fake, fake, ctypes.c_int32(k), fake, fake, fake,
                           fake, None, ctypes.c_size_t(0), None)
    assert st == -3
    assert L.im_workspace_need(ctypes.byref(need), None) == 0
    assert need.value == _ws_size(L, 3, n=n, count=count, k=k)
    assert b"im_workspace_size" in L.im_last_error()
    # one byte short of the reported size is still short
    st = L.im_greedy_cover(ctypes.c_int32(n), ctypes.c_int64(count), fake, fake,
                           ctypes.c_int64(100), fake, fake, ctypes.c_int32(k), fake, fake, fake,
                           fake, ctypes.c_void_p(1 << 30), ctypes.c_size_t(need.value - 1), None)
    assert st == -3
    L.im_randgreedi.restype = ctypes.c_int
    st = L.im_randgreedi(ctypes.c_int32(n), ctypes.c_int64(count), fake, fake,
                         ctypes.c_int64(100), fake, fake, ctypes.c_int32(k), ctypes.c_int32(m),
                         ctypes.c_uint64(1), fake, fake, fake, fake, fake, None,
                         ctypes.c_size_t(4096), None)
    assert st == -3
    assert L.im_workspace_need(ctypes.byref(need), None) == 0
    assert need.value == _ws_size(L, 4, n=n, count=count, total=100, k=k, m=m)
    L.im_stream_cover.restype = ctypes.c_int
    st = L.im_stream_cover(ctypes.c_int32(n), ctypes.c_int64(count), fake, fake, ctypes.c_int32(k),
                           ctypes.c_int32(m), fake, fake, fake, ctypes.c_double(0.077),
                           ctypes.c_double(1.0), fake, fake, fake, fake, None, ctypes.c_size_t(0),
                           None)
    assert st == -3
    assert L.im_workspace_need(ctypes.byref(need), None) == 0
    assert need.value == _ws_size(L, 5, n=n, count=count, k=k, m=m, delta=0.077)
    L.im_build_incidence.restype = ctypes.c_int
    st = L.im_build_incidence(ctypes.c_int32(n), ctypes.c_int64(count), fake, fake,
                              ctypes.c_int64(1 << 20), fake, fake, None, ctypes.c_size_t(0), None)
    assert st == -3
    assert L.im_workspace_need(ctypes.byref(need), None) == 0
    assert need.value == _ws_size(L, 2, n=n, total=1 << 20)
    want = ctypes.c_size_t()
    assert L.im_workspace_need(None, ctypes.byref(want)) == 0 and want.value >= need.value
    assert L.im_workspace_need(None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_tune_knobs_validate_and_round_trip():
    """Launch-shape knobs: defaults, range checks (nothing changes on a
    rejected value), set/get, -1 restores the default.  Host only."""
    L = ctypes.CDLL(LIB)
    L.im_tune_set.argtypes = [ctypes.c_int32, ctypes.c_int64]
    L.im_tune_get.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    v = ctypes.c_int64()

    def get(key):
        assert L.im_tune_get(key, ctypes.byref(v)) == 0
        return v.value

    defaults = {0: 5, 1: 0, 2: 1, 3: 256, 4: 2, 5: 16, 6: 0, 7: 1}
    assert {k: get(k) for k in defaults} == defaults
    for key, bad in ((0, 0), (0, 65), (1, 3), (2, 0), (2, 17), (3, -2), (4, 0), (4, 33), (5, 0),
                     (5, 4097), (6, 2), (6, -2), (7, 2), (7, -2), (8, 1), (-1, 1)):
        assert L.im_tune_set(key, bad) == -1, (key, bad)
    assert {k: get(k) for k in defaults} == defaults
    assert L.im_tune_get(9, ctypes.byref(v)) == -1
    assert L.im_tune_get(0, None) == -1
    for key, good in ((0, 12), (1, 2), (2, 4), (3, 0), (4, 7), (5, 64), (6, 1), (7, 0)):
        assert L.im_tune_set(key, good) == 0
        assert get(key) == good
        assert L.im_tune_set(key, -1) == 0
        assert get(key) == defaults[key]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libim.so not built")
def test_imm_host_schedule_and_decisions_match_oracle():
    """The library's IMM schedule (im_imm_plan) equals the oracle's bit for
    bit, and its round test / final theta (im_imm_round, im_imm_theta) take
    the oracle's decisions: stop once n C / theta_x >= (1 + eps') n / 2^x.
    Host only."""
    import oracle as O
    import paper_2408_10982_amd as im
    for n, k, eps in ((4096, 16, 0.5), (1 << 20, 100, 0.13), (1 << 22, 100, 0.13), (500, 8, 0.4)):
        p = im.imm_plan(n, k, eps)
        o = O.imm_parameters(n, k, eps)
        for key in ("ell", "eps_prime", "log_binom", "lambda_prime", "lambda_star", "theta1",
                    "rounds"):
            assert p[key] == o[key], (n, k, eps, key)
        th = p["theta1"]
        for x in range(1, 4):
            for cov in (0, 1, th // 8, th // 3, th // 2, th):
                stop, lb = p.round(x, th, cov)
                need = (1.0 + o["eps_prime"]) * (n / 2.0 ** x)
                assert stop == (n * cov / th >= need)
                if stop:
                    assert lb == n * cov / (th * (1.0 + o["eps_prime"]))
                    assert p.theta(lb) == math.ceil(o["lambda_star"] / lb)
            th *= 2
