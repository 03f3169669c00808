"""ctypes binding of libim.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; this module
only turns torch tensors (device memory) and torch's current HIP stream into
the plain pointers the C ABI takes, checks status codes, and sizes outputs
and workspaces.  The library allocates no device memory: each call gets a
workspace, a torch uint8 tensor kept per (device, stream) that grows when a
call reports IM_ENOMEM with the bytes it needs (the call is then repeated;
results never depend on the workspace size).
If libim.so is missing the import fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libim.so")

IM_OK, IM_EINVAL, IM_ERANGE, IM_ENOMEM, IM_EDEVICE = 0, -1, -2, -3, -4
IC, LT = 0, 1
SEL_GREEDY, SEL_GREEDIRIS, SEL_RANDGREEDI = 0, 1, 2
(TUNE_SAMPLE_BLOCKS, TUNE_BIG_SHAPE, TUNE_APPLY_BLOCKS, TUNE_DENSE_RATIO, TUNE_LT_BLOCKS,
 TUNE_LT_GRAB, TUNE_GRAPH, TUNE_LISTS) = 0, 1, 2, 3, 4, 5, 6, 7
(WS_PREPARE_GRAPH, WS_SAMPLE, WS_INCIDENCE, WS_GREEDY, WS_RANDGREEDI, WS_STREAM, WS_OFFLINE,
 WS_FORWARD, WS_INFLUENCE, WS_SOLVE, WS_OPIM, WS_BATCH) = range(12)

_STATUS = {IM_EINVAL: "IM_EINVAL", IM_ERANGE: "IM_ERANGE", IM_ENOMEM: "IM_ENOMEM",
           IM_EDEVICE: "IM_EDEVICE"}

# every symbol the header declares
EXPORTS = ("im_version", "im_last_error", "im_release", "im_prepare_graph", "im_sample_rrr",
           "im_build_incidence", "im_greedy_cover", "im_greedy_cover_static", "im_randgreedi", "im_stream_cover", "im_greedi_offline",
           "im_prepare_forward", "im_influence", "im_opim",
           "im_solve", "im_solve_batch", "im_imm_plan", "im_imm_round", "im_imm_theta",
           "im_workspace_size", "im_workspace_need", "im_lt_index_size", "im_tune_set",
           "im_tune_get")


class ImError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__("%s returned %s%s" % (where, _STATUS.get(status, status),
                                               (": " + detail) if detail else ""))


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("num_edges", C.c_int64), ("in_off", C.c_void_p),
                ("in_src", C.c_void_p), ("thr", C.c_void_p), ("model", C.c_int32),
                ("skip", C.c_void_p), ("lt_index", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("total", C.c_int64), ("examined", C.c_int64), ("live", C.c_int64),
                ("large_sets", C.c_int64), ("large_total", C.c_int64),
                ("large_examined", C.c_int64), ("large_live", C.c_int64),
                ("redo_examined", C.c_int64), ("ms_main", C.c_double), ("ms_large", C.c_double), ("ms_canon", C.c_double)]


class _SolveOpts(C.Structure):
    _fields_ = [("selector", C.c_int32), ("m", C.c_int32), ("delta", C.c_double),
                ("alpha", C.c_double), ("seed", C.c_uint64), ("part_seed", C.c_uint64),
                ("theta", C.c_int64)]


class _SolveResult(C.Structure):
    _fields_ = [("nsel", C.c_int32), ("coverage", C.c_int64), ("theta", C.c_int64),
                ("rounds", C.c_int32), ("lower_bound", C.c_double),
                ("martingale_samples", C.c_int64), ("bucket", C.c_int32),
                ("global_won", C.c_int32), ("stream_len", C.c_int32),
                ("final_total", C.c_int64),
                ("sample_launches", C.c_int32), ("sample_passes", C.c_int32),
                ("sampled_sets", C.c_int64), ("sampled_total", C.c_int64),
                ("sampled_examined", C.c_int64), ("sampled_live", C.c_int64),
                ("ms_sample_main", C.c_double), ("ms_sample_large", C.c_double),
                ("ms_sample_gather", C.c_double), ("ms_select", C.c_double),
                ("ms_incidence", C.c_double), ("ms_local", C.c_double),
                ("ms_global", C.c_double), ("global_cover", C.c_int64)]


class _ImmPlan(C.Structure):
    _fields_ = [("ell", C.c_double), ("eps_prime", C.c_double), ("log_binom", C.c_double),
                ("lambda_prime", C.c_double), ("lambda_star", C.c_double),
                ("theta1", C.c_int64), ("rounds", C.c_int32)]


class _OpimResult(C.Structure):
    _fields_ = [("nsel", C.c_int32), ("rounds", C.c_int32), ("theta", C.c_int64),
                ("cover1", C.c_int64), ("cover2", C.c_int64), ("upper1", C.c_int64),
                ("lower", C.c_double), ("upper", C.c_double), ("guarantee", C.c_double),
                ("theta_max", C.c_double), ("i_max", C.c_int32), ("bucket", C.c_int32),
                ("global_won", C.c_int32)]


class _WsShape(C.Structure):
    _fields_ = [("n", C.c_int32), ("model", C.c_int32), ("count", C.c_int64),
                ("total", C.c_int64), ("k", C.c_int32), ("m", C.c_int32), ("delta", C.c_double),
                ("selector", C.c_int32), ("ntasks", C.c_int32), ("full", C.c_int32),
                ("num_cus", C.c_int32)]


class _Task(C.Structure):
    _fields_ = [("graph", _Graph), ("seed", C.c_uint64), ("stream_tag", C.c_uint32),
                ("k", C.c_int32), ("theta", C.c_int64)]


class _BatchStats(C.Structure):
    _fields_ = [("sets", C.c_int64), ("total", C.c_int64), ("examined", C.c_int64),
                ("live", C.c_int64), ("ms_sample", C.c_double), ("ms_incidence", C.c_double),
                ("ms_cover", C.c_double)]


_lib = None


def lib():
    """Loads libim.so (raises if the HIP library has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libim.so not built: run paper_2408_10982_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, U32, U64, D = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64,
                                    C.c_double)
        L.im_version.restype = C.c_char_p
        L.im_last_error.restype = C.c_char_p
        L.im_release.argtypes = []
        W = [P, C.c_size_t]  # (ws, ws_bytes)
        L.im_prepare_graph.argtypes = [I32, I64, P, P, P, I32, P, P, P] + W + [P]
        L.im_lt_index_size.argtypes = [I64, C.POINTER(C.c_int64)]
        L.im_sample_rrr.argtypes = [C.POINTER(_Graph), U64, U32, I64, I64, P, P, I64,
                                    C.POINTER(C.c_int64), C.POINTER(_Stats)] + W + [P]
        L.im_build_incidence.argtypes = [I32, I64, P, P, I64, P, P] + W + [P]
        L.im_greedy_cover.argtypes = [I32, I64, P, P, I64, P, P, I32, P, P, P, P] + W + [P]
        L.im_greedy_cover_static.argtypes = [I32, I64, P, P, I64, P, P, I32, P, P, P, P, P]
        L.im_randgreedi.argtypes = ([I32, I64, P, P, I64, P, P, I32, I32, U64, P, P, P, P, P] +
                                    W + [P])
        L.im_stream_cover.argtypes = ([I32, I64, P, P, I32, I32, P, P, P, D, D, P, P, P, P] +
                                      W + [P])
        L.im_opim.argtypes = [C.POINTER(_Graph), I32, D, D, I64, C.POINTER(_SolveOpts), P,
                              C.POINTER(_OpimResult)] + W + [P]
        L.im_prepare_forward.argtypes = [I32, I64, P, P, P, P, P] + W + [P]
        L.im_influence.argtypes = ([C.POINTER(_Graph), P, P, P, U64, U32, I64, I64, P, I32, P] +
                                   W + [P])
        L.im_greedi_offline.argtypes = ([I32, I64, P, P, I64, P, P, I32, I32, P, P, P, D, P, P,
                                         P, P, P] + W + [P])
        L.im_solve.argtypes = [C.POINTER(_Graph), I32, D, C.POINTER(_SolveOpts), P,
                               C.POINTER(_SolveResult)] + W + [P]
        L.im_solve_batch.argtypes = ([C.POINTER(_Task), I32, P, P, P, P,
                                      C.POINTER(_BatchStats)] + W + [P])
        L.im_workspace_size.argtypes = [I32, C.POINTER(_WsShape), C.POINTER(C.c_size_t)]
        L.im_workspace_need.argtypes = [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.im_imm_plan.argtypes = [I32, I32, D, C.POINTER(_ImmPlan)]
        L.im_imm_round.argtypes = [C.POINTER(_ImmPlan), I32, I32, I64, I64,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.im_imm_theta.argtypes = [C.POINTER(_ImmPlan), D, C.POINTER(C.c_int64)]
        L.im_tune_set.argtypes = [I32, I64]
        L.im_tune_get.argtypes = [I32, C.POINTER(C.c_int64)]
        for f in EXPORTS[2:]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != IM_OK:
        detail = lib().im_last_error().decode() if status in (IM_EDEVICE, IM_ENOMEM) else ""
        raise ImError(status, where, detail)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ workspaces
_WS: dict = {}            # (device index, stream handle) -> uint8 device tensor
_WS_LOCK = threading.Lock()
_WS_GRAIN = 2 << 20       # workspaces grow in whole 2 MiB steps
_WS_TRIES = 8             # a call that keeps running short gives up after this many


def workspace_size(op: int, n: int = 0, model: int = IC, count: int = 0, total: int = 0,
                   k: int = 0, m: int = 0, delta: float = 0.0, selector: int = SEL_GREEDY,
                   ntasks: int = 0, full: bool = False, num_cus: int = 0) -> int:
    """Bytes of workspace the library asks for `op` (WS_*) on a shape (im_workspace_size)."""
    sh = _WsShape(n, model, count, total, k, m, delta, selector, ntasks, int(full), num_cus)
    b = C.c_size_t()
    _check(lib().im_workspace_size(op, C.byref(sh), C.byref(b)), "im_workspace_size")
    return int(b.value)


def workspace_need():
    """(need, want) of the calling thread's last call (im_workspace_need):
    the bytes it needed at least if it ran short (else 0), and the bytes its
    fastest launch shapes would have used."""
    need, want = C.c_size_t(), C.c_size_t()
    _check(lib().im_workspace_need(C.byref(need), C.byref(want)), "im_workspace_need")
    return int(need.value), int(want.value)


def _sampling_hint(g: "Graph") -> int:
    """Workspace for one sampling call on g with room for every large-set
    worker the launch can use (up to 16 GiB): a smaller workspace would run
    a first call with few workers, which on graphs with many large sets is
    orders of magnitude slower."""
    return workspace_size(WS_SAMPLE, n=g.n, model=g.model, count=1 << 20, total=1 << 20,
                          full=True)


def _ws_tensor(s, want: int) -> torch.Tensor:
    key = (s.device.index, s.cuda_stream)
    with _WS_LOCK:
        t = _WS.get(key)
        if t is not None and t.numel() >= want:
            return t
    size = max(_WS_GRAIN, -(-want // _WS_GRAIN) * _WS_GRAIN)
    # allocated on the stream that uses it, so that the caching allocator
    # reuses the old block only after that stream's queued work
    with torch.cuda.stream(s):
        if t is not None:
            with _WS_LOCK:
                _WS.pop(key, None)
            del t
        t = torch.empty(size, dtype=torch.uint8, device=s.device)
    with _WS_LOCK:
        _WS[key] = t
    return t


def _call_ws(fn, where: str, args: tuple, stream=None, hint: int = 0, ok=(IM_OK,)) -> int:
    """Calls an entry point with the stream's workspace, growing it and
    calling again while the call reports a workspace shortfall.  A call that
    could have used more (faster launch shapes) gets it from the next call
    on the stream on."""
    s = torch.cuda.current_stream() if stream is None else stream
    size = hint
    rc = IM_ENOMEM
    for _ in range(_WS_TRIES):
        ws = _ws_tensor(s, size)
        rc = fn(*args, C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(s.cuda_stream))
        need, want = workspace_need()
        if rc != IM_ENOMEM:
            if want > ws.numel():
                _ws_tensor(s, want)
            break
        if need <= ws.numel():  # not a workspace shortfall
            break
        size = max(need + need // 4, want)
    if rc not in ok:
        _check(rc, where)
    return rc


def workspace_bytes(stream=None) -> int:
    """Device bytes of the workspace held for the stream (0 if none yet)."""
    s = torch.cuda.current_stream() if stream is None else stream
    with _WS_LOCK:
        t = _WS.get((s.device.index, s.cuda_stream))
    return 0 if t is None else t.numel()


def drop_workspaces(stream=None):
    """Forgets the cached workspace of `stream`, or every cached workspace
    (their memory returns to torch's allocator once the streams' work is
    done)."""
    with _WS_LOCK:
        if stream is None:
            _WS.clear()
        else:
            _WS.pop((stream.device.index, stream.cuda_stream), None)


def _dev(t: torch.Tensor, dtype) -> torch.Tensor:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous %s device tensor" % dtype)
    return t


@dataclass
class Graph:
    """A graph prepared for sampling: in-edge CSR plus integer thresholds."""
    n: int
    num_edges: int
    model: int
    in_off: torch.Tensor   # int32 [n+1]
    in_src: torch.Tensor   # int32 [E]
    thr: torch.Tensor      # int32 storage of uint32 thresholds, [round_up(E, 4)]
    skip: torch.Tensor | None = None   # float64 [n]: IC run-length table
    lt_index: torch.Tensor | None = None   # int32 storage of the LT search index

    def struct(self) -> _Graph:
        return _Graph(self.n, self.num_edges, self.in_off.data_ptr(),
                      self.in_src.data_ptr() if self.num_edges else None,
                      self.thr.data_ptr(), self.model,
                      self.skip.data_ptr() if self.skip is not None else None,
                      self.lt_index.data_ptr() if self.lt_index is not None else None)

    def hbm_bytes(self) -> int:
        return (4 * (self.in_off.numel() + self.in_src.numel() + self.thr.numel()) +
                (8 * self.skip.numel() if self.skip is not None else 0) +
                (4 * self.lt_index.numel() if self.lt_index is not None else 0))


def lt_index_size(num_edges: int) -> int:
    """Entries of the LT search index for num_edges edges (im_lt_index_size)."""
    e = C.c_int64()
    _check(lib().im_lt_index_size(num_edges, C.byref(e)), "im_lt_index_size")
    return int(e.value)


def prepare_graph(in_off, in_src, weight, model: int, device="cuda", stream=None,
                  run_length: bool = True, lt_index: bool = True) -> Graph:
    """Uploads an in-edge CSR with fp32 weights and derives the thresholds
    (and, for IC, the run-length table unless run_length is False; for LT,
    the search index unless lt_index is False)."""
    in_off = torch.as_tensor(in_off, dtype=torch.int32).to(device).contiguous()
    in_src = torch.as_tensor(in_src, dtype=torch.int32).to(device).contiguous()
    weight = torch.as_tensor(weight, dtype=torch.float32).to(device).contiguous()
    n = in_off.numel() - 1
    E = in_src.numel()
    thr = torch.empty(max((E + 3) // 4 * 4, 4), dtype=torch.int32, device=device)
    skip = (torch.empty(n, dtype=torch.float64, device=device)
            if model == IC and run_length else None)
    index = (torch.empty(max(lt_index_size(E), 16), dtype=torch.int32, device=device)
             if model == LT and lt_index else None)
    _call_ws(lib().im_prepare_graph, "im_prepare_graph",
             (n, E, _ptr(in_off), _ptr(in_src) if E else None, _ptr(weight) if E else None,
              model, _ptr(thr), _ptr(skip), _ptr(index)), stream)
    return Graph(n, E, model, in_off, in_src, thr, skip, index)


@dataclass
class RRR:
    off: torch.Tensor   # int64 [count+1]
    mem: torch.Tensor   # int32 [total]
    total: int
    examined: int
    live: int
    large_sets: int
    stats: dict | None = None

    @property
    def count(self) -> int:
        return self.off.numel() - 1


def sample_rrr(g: Graph, seed: int, stream_tag: int, first: int, count: int,
               capacity: int | None = None, stream=None) -> RRR:
    off = torch.empty(count + 1, dtype=torch.int64, device=g.in_off.device)
    cap = int(capacity) if capacity is not None else max(4 * count, 1024)
    gs = g.struct()
    for _ in range(2):
        mem = torch.empty(max(cap, 1), dtype=torch.int32, device=g.in_off.device)
        total = C.c_int64()
        stats = _Stats()
        hint = max(workspace_size(WS_SAMPLE, n=g.n, model=g.model, count=count, total=cap),
                   _sampling_hint(g))
        st = _call_ws(lib().im_sample_rrr, "im_sample_rrr",
                      (C.byref(gs), seed, stream_tag, first, count, _ptr(off), _ptr(mem), cap,
                       C.byref(total), C.byref(stats)), stream, hint, ok=(IM_OK, IM_ERANGE))
        if st == IM_ERANGE:
            cap = int(total.value)
            continue
        sd = {f: getattr(stats, f) for f, _ in _Stats._fields_}
        return RRR(off, mem[:total.value], int(total.value), int(stats.examined),
                   int(stats.live), int(stats.large_sets), sd)
    raise ImError(IM_ERANGE, "im_sample_rrr")


def build_incidence(n: int, rrr: RRR, stream=None):
    inc_off = torch.empty(n + 1, dtype=torch.int64, device=rrr.off.device)
    inc_mem = torch.empty(max(rrr.total, 1), dtype=torch.int32, device=rrr.off.device)
    _call_ws(lib().im_build_incidence, "im_build_incidence",
             (n, rrr.count, _ptr(rrr.off), _ptr(rrr.mem), rrr.total, _ptr(inc_off),
              _ptr(inc_mem)), stream, workspace_size(WS_INCIDENCE, n=n, total=rrr.total))
    return inc_off, inc_mem[:rrr.total]


def greedy_cover(n: int, rrr: RRR, inc_off, inc_mem, k: int, stream=None):
    """Returns device tensors (seeds int32[k], gains int64[k], nsel int32[1], coverage int64[1])."""
    dev = rrr.off.device
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    gains = torch.empty(k, dtype=torch.int64, device=dev)
    nsel = torch.empty(1, dtype=torch.int32, device=dev)
    cov = torch.empty(1, dtype=torch.int64, device=dev)
    _call_ws(lib().im_greedy_cover, "im_greedy_cover",
             (n, rrr.count, _ptr(rrr.off), _ptr(rrr.mem), rrr.total, _ptr(inc_off),
              _ptr(inc_mem), k, _ptr(seeds), _ptr(gains), _ptr(nsel), _ptr(cov)), stream,
             workspace_size(WS_GREEDY, n=n, count=rrr.count, k=k))
    return seeds, gains, nsel, cov


def greedy_cover_static(n: int, rrr: RRR, inc_off, inc_mem, k: int, stream=None):
    """im_greedy_cover_static: the same greedy with the library's fixed scratch
    array (no workspace).  Returns (seeds, gains, nsel, coverage) device tensors."""
    dev = rrr.off.device
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    gains = torch.empty(k, dtype=torch.int64, device=dev)
    nsel = torch.empty(1, dtype=torch.int32, device=dev)
    cov = torch.empty(1, dtype=torch.int64, device=dev)
    st = lib().im_greedy_cover_static(n, rrr.count, _ptr(rrr.off), _ptr(rrr.mem), rrr.total,
                                      _ptr(inc_off), _ptr(inc_mem), k, _ptr(seeds), _ptr(gains),
                                      _ptr(nsel), _ptr(cov), _stream(stream))
    _check(st, "im_greedy_cover_static")
    return seeds, gains, nsel, cov


def randgreedi(n: int, rrr: RRR, inc_off, inc_mem, k: int, m: int, part_seed: int,
               stream=None):
    """Returns (part uint8[n], lseeds int32[m,k], lgains int64[m,k], lcount int32[m],
    lcover int64[m]) on the device."""
    dev = rrr.off.device
    part = torch.empty(n, dtype=torch.uint8, device=dev)
    ls = torch.empty((m, k), dtype=torch.int32, device=dev)
    lg = torch.empty((m, k), dtype=torch.int64, device=dev)
    lc = torch.empty(m, dtype=torch.int32, device=dev)
    lv = torch.empty(m, dtype=torch.int64, device=dev)
    _call_ws(lib().im_randgreedi, "im_randgreedi",
             (n, rrr.count, _ptr(rrr.off), _ptr(rrr.mem), rrr.total, _ptr(inc_off),
              _ptr(inc_mem), k, m, part_seed, _ptr(part), _ptr(ls), _ptr(lg), _ptr(lc),
              _ptr(lv)), stream,
             workspace_size(WS_RANDGREEDI, n=n, count=rrr.count, total=rrr.total, k=k, m=m))
    return part, ls, lg, lc, lv


def stream_cover(n: int, count: int, inc_off, inc_mem, lseeds, lcount, lcover, k: int,
                 delta: float, alpha: float, stream=None):
    """Returns device tensors (seeds int32[k], nsel int32[1], coverage int64[1],
    info int32[4] = (best bucket, buckets, streamed solution chosen, stream length))."""
    dev = inc_off.device
    m = lcount.numel()
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    nsel = torch.empty(1, dtype=torch.int32, device=dev)
    cov = torch.empty(1, dtype=torch.int64, device=dev)
    info = torch.empty(4, dtype=torch.int32, device=dev)
    hint = (workspace_size(WS_STREAM, n=n, count=count, k=k, m=m, delta=delta)
            if 0.0 < delta < 0.5 else 0)
    _call_ws(lib().im_stream_cover, "im_stream_cover",
             (n, count, _ptr(inc_off), _ptr(inc_mem), k, m, _ptr(lseeds), _ptr(lcount),
              _ptr(lcover), delta, alpha, _ptr(seeds), _ptr(nsel), _ptr(cov), _ptr(info)),
             stream, hint)
    return seeds, nsel, cov, info


def greedi_offline(n: int, rrr: RRR, inc_off, inc_mem, lseeds, lcount, lcover, k: int,
                   alpha: float = 1.0, stream=None):
    """Offline GreeDI aggregation of the local solutions (Alg. 4).  Returns
    device tensors (seeds int32[k], nsel int32[1], coverage int64[1], info
    int32[4] = (global chosen, gathered, |S_g|, best local part), gcover int64[1])."""
    dev = inc_off.device
    m = lcount.numel()
    seeds = torch.empty(k, dtype=torch.int32, device=dev)
    nsel = torch.empty(1, dtype=torch.int32, device=dev)
    cov = torch.empty(1, dtype=torch.int64, device=dev)
    info = torch.empty(4, dtype=torch.int32, device=dev)
    gcov = torch.empty(1, dtype=torch.int64, device=dev)
    _call_ws(lib().im_greedi_offline, "im_greedi_offline",
             (n, rrr.count, _ptr(rrr.off), _ptr(rrr.mem), rrr.total, _ptr(inc_off),
              _ptr(inc_mem), k, m, _ptr(lseeds), _ptr(lcount), _ptr(lcover), alpha, _ptr(seeds),
              _ptr(nsel), _ptr(cov), _ptr(info), _ptr(gcov)), stream,
             workspace_size(WS_OFFLINE, n=n, count=rrr.count, k=k, m=m))
    return seeds, nsel, cov, info, gcov


@dataclass
class Forward:
    """Out-edge view of a prepared graph (im_prepare_forward)."""
    out_off: torch.Tensor    # int64 [n+1]
    out_eid: torch.Tensor    # int32 [E]
    edge_dst: torch.Tensor   # int32 [E]


def prepare_forward(g: Graph, stream=None) -> Forward:
    dev = g.in_off.device
    out_off = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
    out_eid = torch.empty(max(g.num_edges, 1), dtype=torch.int32, device=dev)
    edge_dst = torch.empty(max(g.num_edges, 1), dtype=torch.int32, device=dev)
    _call_ws(lib().im_prepare_forward, "im_prepare_forward",
             (g.n, g.num_edges, _ptr(g.in_off), _ptr(g.in_src) if g.num_edges else None,
              _ptr(out_off), _ptr(out_eid), _ptr(edge_dst)), stream,
             workspace_size(WS_FORWARD, n=g.n))
    return Forward(out_off, out_eid, edge_dst)


def influence(g: Graph, fwd: Forward, seed: int, stream_tag: int, first: int, nsims: int,
              seeds, stream=None) -> torch.Tensor:
    """Activated-vertex counts of forward simulations [first, first+nsims)
    (int64 device tensor)."""
    sd = [int(x) for x in seeds]
    arr = (C.c_int32 * max(len(sd), 1))(*sd)
    counts = torch.empty(max(nsims, 1), dtype=torch.int64, device=g.in_off.device)
    gs = g.struct()
    _call_ws(lib().im_influence, "im_influence",
             (C.byref(gs), _ptr(fwd.out_off), _ptr(fwd.out_eid), _ptr(fwd.edge_dst), seed,
              stream_tag, first, nsims, arr, len(sd), _ptr(counts)), stream,
             workspace_size(WS_INFLUENCE, n=g.n, count=nsims, k=len(sd)))
    return counts[:nsims]


def solve(g: Graph, k: int, eps: float, selector: int = SEL_GREEDY, m: int = 1,
          delta: float = 0.077, alpha: float = 1.0, seed: int = 0, part_seed: int = 0,
          theta: int = 0, stream=None) -> dict:
    o = _SolveOpts(selector, m, delta, alpha, seed, part_seed, theta)
    res = _SolveResult()
    seeds = (C.c_int32 * k)()
    gs = g.struct()
    _call_ws(lib().im_solve, "im_solve", (C.byref(gs), k, eps, C.byref(o), seeds, C.byref(res)),
             stream, _sampling_hint(g))
    out = {f: getattr(res, f) for f, _ in _SolveResult._fields_}
    out["seeds"] = list(seeds)[:res.nsel]
    return out


def opim(g: Graph, k: int, eps: float, fail: float, theta_cap: int,
         selector: int = SEL_GREEDY, m: int = 1, delta: float = 0.077, alpha: float = 1.0,
         seed: int = 0, part_seed: int = 0, stream=None) -> dict:
    """OPIM rounds with the given selector (im_opim)."""
    o = _SolveOpts(selector, m, delta, alpha, seed, part_seed, 0)
    res = _OpimResult()
    seeds = (C.c_int32 * k)()
    gs = g.struct()
    _call_ws(lib().im_opim, "im_opim",
             (C.byref(gs), k, eps, fail, theta_cap, C.byref(o), seeds, C.byref(res)), stream,
             _sampling_hint(g))
    out = {f: getattr(res, f) for f, _ in _OpimResult._fields_}
    out["seeds"] = list(seeds)[:res.nsel]
    return out


def solve_batch(tasks, stream=None):
    """tasks: list of (Graph, seed, stream_tag, k, theta).  Returns a list of
    per-task dicts (seeds, gains, coverage) and the batch statistics."""
    nt = len(tasks)
    arr = (_Task * nt)()
    ks = []
    for j, (g, seed, tag, k, theta) in enumerate(tasks):
        arr[j] = _Task(g.struct(), seed, tag, k, theta)
        ks.append(k)
    dev = tasks[0][0].in_off.device
    K = sum(ks)
    seeds = torch.empty(K, dtype=torch.int32, device=dev)
    gains = torch.empty(K, dtype=torch.int64, device=dev)
    nsel = torch.empty(nt, dtype=torch.int32, device=dev)
    cov = torch.empty(nt, dtype=torch.int64, device=dev)
    st = _BatchStats()
    _call_ws(lib().im_solve_batch, "im_solve_batch",
             (arr, nt, _ptr(seeds), _ptr(gains), _ptr(nsel), _ptr(cov), C.byref(st)), stream,
             max(_sampling_hint(t[0]) for t in tasks))
    s_h, g_h, n_h, c_h = (seeds.cpu().tolist(), gains.cpu().tolist(), nsel.cpu().tolist(),
                          cov.cpu().tolist())
    out, o = [], 0
    for j, k in enumerate(ks):
        n = n_h[j]
        out.append({"seeds": s_h[o:o + n], "gains": g_h[o:o + n], "coverage": c_h[j]})
        o += k
    return out, {f: getattr(st, f) for f, _ in _BatchStats._fields_}


class ImmPlan:
    """The library's IMM schedule for (n, k, eps) and its round decisions."""

    def __init__(self, n: int, k: int, eps: float):
        self.n = n
        self.p = _ImmPlan()
        _check(lib().im_imm_plan(n, k, eps, C.byref(self.p)), "im_imm_plan")

    def __getitem__(self, key):
        return getattr(self.p, key)

    def round(self, x: int, theta_x: int, coverage: int):
        """(stop, lb) after martingale round x (im_imm_round)."""
        stop, lb = C.c_int32(), C.c_double()
        _check(lib().im_imm_round(C.byref(self.p), self.n, x, theta_x, coverage, C.byref(stop),
                                  C.byref(lb)), "im_imm_round")
        return bool(stop.value), lb.value

    def theta(self, lb: float) -> int:
        t = C.c_int64()
        _check(lib().im_imm_theta(C.byref(self.p), lb, C.byref(t)), "im_imm_theta")
        return int(t.value)


def imm_plan(n: int, k: int, eps: float) -> ImmPlan:
    return ImmPlan(n, k, eps)


def sample_into(g: Graph, seed: int, stream_tag: int, first: int, count: int,
                off: torch.Tensor, mem: torch.Tensor, stream=None):
    """Samples sets [first, first+count) into caller tensors: off (count+1
    int64, starts at 0) and mem (int32, its whole length is the capacity).
    Returns the member total, or -total if mem was too small (IM_ERANGE)."""
    gs = g.struct()
    total = C.c_int64()
    hint = max(workspace_size(WS_SAMPLE, n=g.n, model=g.model, count=count, total=mem.numel()),
               _sampling_hint(g))
    st = _call_ws(lib().im_sample_rrr, "im_sample_rrr",
                  (C.byref(gs), seed, stream_tag, first, count, _ptr(off), _ptr(mem),
                   mem.numel(), C.byref(total), None), stream, hint, ok=(IM_OK, IM_ERANGE))
    if st == IM_ERANGE:
        return -int(total.value)
    return int(total.value)


def release():
    """Waits for the device, drops the cached workspaces and the library's
    captured cover graphs."""
    _check(lib().im_release(), "im_release")
    drop_workspaces()


def tune_set(key: int, value: int):
    """Sets a launch-shape knob (TUNE_*; -1 restores its default)."""
    _check(lib().im_tune_set(key, value), "im_tune_set")


def tune_get(key: int) -> int:
    v = C.c_int64()
    _check(lib().im_tune_get(key, C.byref(v)), "im_tune_get")
    return int(v.value)


def version() -> str:
    return lib().im_version().decode()
