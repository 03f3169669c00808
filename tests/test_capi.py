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
    st = L.im_greedy_cover(ctypes.c_int32(10), ctypes.c_int64(5), None, None, ctypes.c_int64(0),
                           None, None, ctypes.c_int32(0), None, None, None, None, None)
    assert st == -1
    L.im_stream_cover.restype = ctypes.c_int
    st = L.im_stream_cover(ctypes.c_int32(10), ctypes.c_int64(5), None, None, ctypes.c_int32(3),
                           ctypes.c_int32(2), None, None, None, ctypes.c_double(0.7),
                           ctypes.c_double(1.0), None, None, None, None, None)
    assert st == -1
    L.im_sample_rrr.restype = ctypes.c_int
    st = L.im_sample_rrr(None, ctypes.c_uint64(0), ctypes.c_uint32(0), ctypes.c_int64(0),
                         ctypes.c_int64(1), None, None, ctypes.c_int64(0), None, None, None)
    assert st == -1


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

    defaults = {0: 5, 1: 0, 2: 1, 3: 256, 4: 7, 5: 16, 6: 0}
    assert {k: get(k) for k in defaults} == defaults
    for key, bad in ((0, 0), (0, 65), (1, 3), (2, 0), (2, 17), (3, -2), (4, 0), (4, 33), (5, 0),
                     (5, 4097), (6, 2), (6, -2), (7, 1), (-1, 1)):
        assert L.im_tune_set(key, bad) == -1, (key, bad)
    assert {k: get(k) for k in defaults} == defaults
    assert L.im_tune_get(9, ctypes.byref(v)) == -1
    assert L.im_tune_get(0, None) == -1
    for key, good in ((0, 12), (1, 2), (2, 4), (3, 0), (4, 2), (5, 64), (6, 1)):
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
