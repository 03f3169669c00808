"""Python face of the CPU oracle (``im_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library and its binding
never do.  The oracle shares no code with the HIP path: this wrapper only moves
numpy arrays in and out of the single-threaded C implementation, which
restates the paper's definitions and algorithms (arXiv 2408.10982).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "im_oracle.c")
_HDR = os.path.join(_HERE, "im_oracle.h")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

IC, LT = 0, 1
SEL_GREEDY, SEL_GREEDIRIS, SEL_RANDGREEDI = 0, 1, 2
TAG_ROOT, TAG_EDGE, TAG_VERT, TAG_PART, TAG_SIM_EDGE, TAG_SIM_VERT = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Rrr(C.Structure):
    _fields_ = [("count", C.c_int64), ("total", C.c_int64),
                ("off", C.POINTER(C.c_int64)), ("mem", C.POINTER(C.c_int32)),
                ("examined", C.c_int64), ("live", C.c_int64)]


class _ImmParams(C.Structure):
    _fields_ = [("ell", C.c_double), ("eps_prime", C.c_double), ("log_binom", C.c_double),
                ("lambda_prime", C.c_double), ("lambda_star", C.c_double),
                ("alpha_i", C.c_double), ("beta_i", C.c_double),
                ("theta1", C.c_int64), ("rounds", C.c_int32)]


class _ImmOpts(C.Structure):
    _fields_ = [("model", C.c_int), ("selector", C.c_int), ("lazy", C.c_int),
                ("k", C.c_int32), ("m", C.c_int32),
                ("eps", C.c_double), ("delta", C.c_double), ("alpha", C.c_double),
                ("seed", C.c_uint64), ("part_seed", C.c_uint64),
                ("theta_override", C.c_int64)]


class _OpimResult(C.Structure):
    _fields_ = [("nsel", C.c_int32), ("rounds", C.c_int32), ("theta", C.c_int64),
                ("cover1", C.c_int64), ("cover2", C.c_int64), ("upper1", C.c_int64),
                ("lower", C.c_double), ("upper", C.c_double), ("guarantee", C.c_double),
                ("theta_max", C.c_double), ("i_max", C.c_int32)]


class _ImmResult(C.Structure):
    _fields_ = [("nsel", C.c_int32), ("coverage", C.c_int64), ("theta", C.c_int64),
                ("rounds_run", C.c_int32), ("lb", C.c_double),
                ("martingale_samples", C.c_int64), ("bucket", C.c_int32),
                ("global_won", C.c_int), ("stream_len", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_draw.restype = C.c_uint32
        L.or_ic_thresholds.argtypes = [C.c_int64, P, P]
        L.or_lt_thresholds.argtypes = [C.c_int32, P, P, P]
        L.or_root.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32]
        L.or_root.restype = C.c_int32
        L.or_sample.argtypes = [C.c_int, C.c_int32, P, P, P, P, C.c_uint64, C.c_uint32,
                                C.c_uint32, C.c_int64, C.POINTER(_Rrr)]
        L.or_log.argtypes = [C.c_double]
        L.or_log.restype = C.c_double
        L.or_ic_skip_table.argtypes = [C.c_int32, P, P, P]
        L.or_rl_factor.argtypes = [C.c_uint32]
        L.or_rl_factor.restype = C.c_double
        L.or_rl_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_rl_uniform.restype = C.c_double
        L.or_rl_gap.argtypes = [C.c_double, C.c_double]
        L.or_rl_gap.restype = C.c_int64
        L.or_rrr_free.argtypes = [C.POINTER(_Rrr)]
        L.or_incidence.argtypes = [C.c_int32, C.c_int64, P, P, P, P]
        L.or_coverage.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, P]
        L.or_coverage.restype = C.c_int64
        for f in (L.or_greedy, L.or_lazy_greedy):
            f.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, P, P, P, P]
        L.or_partition.argtypes = [C.c_int32, C.c_int32, C.c_uint64, P]
        L.or_local_greedy.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, C.c_int32,
                                      C.c_int, P, P, P, P]
        L.or_trunc_len.argtypes = [C.c_int32, C.c_double]
        L.or_trunc_len.restype = C.c_int32
        L.or_num_buckets.argtypes = [C.c_int32, C.c_double]
        L.or_num_buckets.restype = C.c_int32
        L.or_bucket_thresholds.argtypes = [C.c_int64, C.c_int32, C.c_double, C.c_int32, P]
        L.or_stream_cover.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, C.c_int32, P, P,
                                      P, C.c_double, C.c_double, P, P, P, P, P]
        L.or_greedi_offline.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, C.c_int32, P, P,
                                        C.c_double, C.c_int, P, P, P, P]
        L.or_final_select.argtypes = [C.c_int32, C.c_int32, P, P, P, P, C.c_int32,
                                      C.c_int64, P, P, P]
        L.or_influence.argtypes = [C.c_int, C.c_int32, P, P, P, C.c_uint64, C.c_uint32,
                                   C.c_uint32, C.c_int64, C.c_int32, P, P]
        L.or_opim.argtypes = [C.c_int32, P, P, P, P, C.POINTER(_ImmOpts), C.c_double,
                              C.c_int64, P, C.POINTER(_OpimResult)]
        L.or_imm_parameters.argtypes = [C.c_int32, C.c_int32, C.c_double,
                                        C.POINTER(_ImmParams)]
        L.or_imm.argtypes = [C.c_int32, P, P, P, P, C.POINTER(_ImmOpts), P,
                             C.POINTER(_ImmResult)]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, tag: int, stream: int, sample: int, ident: int) -> int:
    return int(lib().or_draw(seed, tag, stream, sample, ident))


def root(seed: int, stream: int, i: int, n: int) -> int:
    return int(lib().or_root(seed, stream, i, n))


def ic_thresholds(p) -> np.ndarray:
    p = _c(p, np.float32)
    q = np.zeros(p.shape[0], np.uint32)
    if lib().or_ic_thresholds(p.shape[0], _p(p), _p(q)):
        raise ValueError("IC probability outside [0,1] or NaN")
    return q


def lt_thresholds(in_off, w) -> np.ndarray:
    in_off = _c(in_off, np.int32)
    w = _c(w, np.float32)
    c = np.zeros(w.shape[0], np.uint32)
    if lib().or_lt_thresholds(in_off.shape[0] - 1, _p(in_off), _p(w), _p(c)):
        raise ValueError("LT weight negative, infinite or NaN")
    return c


def thresholds(model: int, in_off, w) -> np.ndarray:
    return ic_thresholds(w) if model == IC else lt_thresholds(in_off, w)


def log(x: float) -> float:
    """The method's deterministic natural log (IEEE basic operations only)."""
    return float(lib().or_log(x))


def ic_skip_table(in_off, thr) -> np.ndarray:
    """Per vertex: 1/log(1 - q/2^32) if its >= 2 in-edges share one threshold
    q in (0, 0xFFFFFFFF), else 0 (one coin per in-edge)."""
    in_off = _c(in_off, np.int32)
    thr = _c(thr, np.uint32)
    n = in_off.shape[0] - 1
    out = np.zeros(n, np.float64)
    lib().or_ic_skip_table(n, _p(in_off), _p(thr), _p(out))
    return out


def rl_factor(q: int) -> float:
    """1 / ln(1 - q/2^32): the run-length table entry of threshold q."""
    return float(lib().or_rl_factor(int(q)))


def rl_uniform(seed: int, stream: int, i: int, v: int, j: int) -> float:
    """U on (0, 1] of draw pair j of (sample i, vertex v)."""
    return float(lib().or_rl_uniform(seed, stream, i, v, j))


def rl_gap(u: float, factor: float) -> int:
    """floor(ln U * factor): dead in-edges before the next live one."""
    return int(lib().or_rl_gap(float(u), float(factor)))


def _skip_arg(model, in_off, thr, skip):
    if model != IC or skip is None:
        return None
    if isinstance(skip, str) and skip == "auto":
        return ic_skip_table(in_off, thr)
    return _c(skip, np.float64)


@dataclass
class RRR:
    off: np.ndarray       # int64 [count+1]
    mem: np.ndarray       # int32 [total], ascending within each set
    examined: int
    live: int

    @property
    def count(self) -> int:
        return self.off.shape[0] - 1

    @property
    def total(self) -> int:
        return int(self.off[-1])

    def set(self, i: int) -> np.ndarray:
        return self.mem[self.off[i]:self.off[i + 1]]


def sample(model: int, in_off, in_src, thr, seed: int, stream: int, first: int,
           count: int, skip="auto") -> RRR:
    """skip: "auto" derives the run-length table for IC (what the method
    uses); None flips one coin per in-edge everywhere."""
    in_off = _c(in_off, np.int32)
    in_src = _c(in_src, np.int32)
    thr = _c(thr, np.uint32)
    sk = _skip_arg(model, in_off, thr, skip)
    r = _Rrr()
    if lib().or_sample(model, in_off.shape[0] - 1, _p(in_off), _p(in_src), _p(thr),
                       _p(sk) if sk is not None else None, seed, stream, first, count,
                       C.byref(r)):
        raise MemoryError("oracle sampling failed")
    try:
        off = np.ctypeslib.as_array(r.off, shape=(count + 1,)).copy()
        mem = (np.ctypeslib.as_array(r.mem, shape=(r.total,)).copy() if r.total
               else np.zeros(0, np.int32))
        return RRR(off, mem, int(r.examined), int(r.live))
    finally:
        lib().or_rrr_free(C.byref(r))


def incidence(n: int, rrr: RRR):
    off = _c(rrr.off, np.int64)
    mem = _c(rrr.mem, np.int32)
    inc_off = np.zeros(n + 1, np.int64)
    inc_mem = np.zeros(max(mem.shape[0], 1), np.int32)
    lib().or_incidence(n, off.shape[0] - 1, _p(off), _p(mem), _p(inc_off), _p(inc_mem))
    return inc_off, inc_mem[:mem.shape[0]]


def coverage(n: int, count: int, inc_off, inc_mem, seeds) -> int:
    inc_off = _c(inc_off, np.int64)
    inc_mem = _c(inc_mem, np.int32)
    s = _c(seeds, np.int32)
    return int(lib().or_coverage(n, count, _p(inc_off), _p(inc_mem), s.shape[0], _p(s)))


def greedy(n: int, count: int, inc_off, inc_mem, k: int, lazy: bool = False):
    """Returns (seeds int32[nsel], gains int64[nsel], coverage)."""
    inc_off = _c(inc_off, np.int64)
    inc_mem = _c(inc_mem, np.int32)
    seeds = np.zeros(k, np.int32)
    gains = np.zeros(k, np.int64)
    nsel = C.c_int32()
    cov = C.c_int64()
    f = lib().or_lazy_greedy if lazy else lib().or_greedy
    f(n, count, _p(inc_off), _p(inc_mem), k, _p(seeds), _p(gains), C.byref(nsel), C.byref(cov))
    return seeds[:nsel.value].copy(), gains[:nsel.value].copy(), int(cov.value)


def partition(n: int, m: int, pseed: int) -> np.ndarray:
    part = np.zeros(n, np.uint8)
    lib().or_partition(n, m, pseed, _p(part))
    return part


def local_greedy(n: int, count: int, inc_off, inc_mem, part, m: int, k: int,
                 lazy: bool = True):
    """Returns (lseeds int32[m,k], lgains int64[m,k], lcount int32[m], lcover int64[m])."""
    inc_off = _c(inc_off, np.int64)
    inc_mem = _c(inc_mem, np.int32)
    part = _c(part, np.uint8)
    ls = np.full((m, k), -1, np.int32)
    lg = np.zeros((m, k), np.int64)
    lc = np.zeros(m, np.int32)
    lv = np.zeros(m, np.int64)
    lib().or_local_greedy(n, count, _p(inc_off), _p(inc_mem), _p(part), m, k, int(lazy),
                          _p(ls), _p(lg), _p(lc), _p(lv))
    for p in range(m):
        ls[p, lc[p]:] = -1
        lg[p, lc[p]:] = 0
    return ls, lg, lc, lv


def trunc_len(k: int, alpha: float) -> int:
    return int(lib().or_trunc_len(k, alpha))


def num_buckets(k: int, delta: float) -> int:
    return int(lib().or_num_buckets(k, delta))


def bucket_thresholds(l: int, k: int, delta: float) -> np.ndarray:
    B = num_buckets(k, delta)
    thr = np.zeros(B, np.int64)
    lib().or_bucket_thresholds(l, k, delta, B, _p(thr))
    return thr


def stream_cover(n: int, count: int, inc_off, inc_mem, lseeds, lgains, lcount, k: int,
                 delta: float, alpha: float):
    """Returns (seeds int32[nsel], coverage, bucket, nbuckets)."""
    inc_off = _c(inc_off, np.int64)
    inc_mem = _c(inc_mem, np.int32)
    ls = _c(lseeds, np.int32)
    lg = _c(lgains, np.int64)
    lc = _c(lcount, np.int32)
    m = lc.shape[0]
    seeds = np.zeros(k, np.int32)
    nsel = C.c_int32()
    cov = C.c_int64()
    b = C.c_int32()
    nb = C.c_int32()
    lib().or_stream_cover(n, count, _p(inc_off), _p(inc_mem), m, k, _p(ls), _p(lg), _p(lc),
                          delta, alpha, _p(seeds), C.byref(nsel), C.byref(cov), C.byref(b),
                          C.byref(nb))
    return seeds[:nsel.value].copy(), int(cov.value), int(b.value), int(nb.value)


def greedi_offline(n: int, count: int, inc_off, inc_mem, lseeds, lcount, k: int,
                   alpha: float = 1.0, lazy: bool = True):
    """Alg. 4 global step (offline): returns (seeds int32[gsel], gains, C(S_g))."""
    inc_off = _c(inc_off, np.int64)
    inc_mem = _c(inc_mem, np.int32)
    ls = _c(lseeds, np.int32)
    lc = _c(lcount, np.int32)
    m = lc.shape[0]
    gs = np.zeros(k, np.int32)
    gg = np.zeros(k, np.int64)
    gsel = C.c_int32()
    gcov = C.c_int64()
    lib().or_greedi_offline(n, count, _p(inc_off), _p(inc_mem), m, k, _p(ls), _p(lc), alpha,
                            int(lazy), _p(gs), _p(gg), C.byref(gsel), C.byref(gcov))
    return gs[:gsel.value].copy(), gg[:gsel.value].copy(), int(gcov.value)


def final_select(lseeds, lcount, lcover, gseeds, gcover: int):
    """Returns (seeds, coverage, global_won)."""
    ls = _c(lseeds, np.int32)
    lc = _c(lcount, np.int32)
    lv = _c(lcover, np.int64)
    gs = _c(gseeds if len(gseeds) else np.zeros(1, np.int32), np.int32)
    m, k = ls.shape
    seeds = np.zeros(k, np.int32)
    nsel = C.c_int32()
    cov = C.c_int64()
    won = lib().or_final_select(m, k, _p(ls), _p(lc), _p(lv), _p(gs), len(gseeds), gcover,
                                _p(seeds), C.byref(nsel), C.byref(cov))
    return seeds[:nsel.value].copy(), int(cov.value), bool(won)


def influence(model: int, in_off, in_src, thr, seed: int, stream: int, first: int, nsims: int,
              seeds) -> np.ndarray:
    """Activated-vertex count of each forward simulation r in [first, first+nsims)."""
    in_off = _c(in_off, np.int32)
    in_src = _c(in_src, np.int32)
    thr = _c(thr, np.uint32)
    sd = _c(np.asarray(seeds).reshape(-1), np.int32)
    out = np.zeros(nsims, np.int64)
    if lib().or_influence(model, in_off.shape[0] - 1, _p(in_off), _p(in_src), _p(thr), seed,
                          stream, first, nsims, sd.shape[0], _p(sd), _p(out)):
        raise MemoryError("oracle influence failed")
    return out


def imm_parameters(n: int, k: int, eps: float) -> dict:
    p = _ImmParams()
    lib().or_imm_parameters(n, k, eps, C.byref(p))
    return {f: getattr(p, f) for f, _ in _ImmParams._fields_}


def imm(model: int, in_off, in_src, thr, k: int, eps: float, seed: int,
        selector: int = SEL_GREEDY, m: int = 1, delta: float = 0.077, alpha: float = 1.0,
        part_seed: int = 0, theta: int = 0, lazy: bool = True, skip="auto"):
    in_off = _c(in_off, np.int32)
    in_src = _c(in_src, np.int32)
    thr = _c(thr, np.uint32)
    sk = _skip_arg(model, in_off, thr, skip)
    o = _ImmOpts(model=model, selector=selector, lazy=int(lazy), k=k, m=m, eps=eps,
                 delta=delta, alpha=alpha, seed=seed, part_seed=part_seed,
                 theta_override=theta)
    res = _ImmResult()
    seeds = np.zeros(k, np.int32)
    if lib().or_imm(in_off.shape[0] - 1, _p(in_off), _p(in_src), _p(thr),
                    _p(sk) if sk is not None else None, C.byref(o), _p(seeds), C.byref(res)):
        raise MemoryError("oracle IMM failed")
    out = {f: getattr(res, f) for f, _ in _ImmResult._fields_}
    out["seeds"] = seeds[:res.nsel].copy()
    return out


def opim(model: int, in_off, in_src, thr, k: int, eps: float, seed: int, fail: float,
         theta_cap: int, selector: int = SEL_GREEDY, m: int = 1, delta: float = 0.077,
         alpha: float = 1.0, part_seed: int = 0, lazy: bool = True, skip="auto"):
    """OPIM rounds (R1 on stream 0, R2 on stream 1).  Returns a dict."""
    in_off = _c(in_off, np.int32)
    in_src = _c(in_src, np.int32)
    thr = _c(thr, np.uint32)
    sk = _skip_arg(model, in_off, thr, skip)
    o = _ImmOpts(model=model, selector=selector, lazy=int(lazy), k=k, m=m, eps=eps,
                 delta=delta, alpha=alpha, seed=seed, part_seed=part_seed, theta_override=0)
    res = _OpimResult()
    seeds = np.zeros(k, np.int32)
    if lib().or_opim(in_off.shape[0] - 1, _p(in_off), _p(in_src), _p(thr),
                     _p(sk) if sk is not None else None, C.byref(o), fail, theta_cap,
                     _p(seeds), C.byref(res)):
        raise MemoryError("oracle OPIM failed")
    out = {f: getattr(res, f) for f, _ in _OpimResult._fields_}
    out["seeds"] = seeds[:res.nsel].copy()
    return out
