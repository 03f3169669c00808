"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module builds inputs only: directed graphs as in-edge CSR arrays with
fp32 edge weights.  It holds none of the method's arithmetic (no thresholds,
no sampling, no cover) and imports neither the product nor the oracle.  Its
random numbers come from numpy's PCG64 generator, seeded per workload.

The paper evaluates on SNAP/KONECT graphs with edge probabilities drawn
uniformly from [0, 0.1] (Sec. 4.1, Table 3).  Those datasets are not
available here; R-MAT and Chung-Lu power-law graphs of matching shape stand
in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

IC, LT = 0, 1

RMAT_ABC = (0.57, 0.19, 0.19)


@dataclass
class Graph:
    """Directed graph as in-edge CSR: in-edges of v are in_src[in_off[v]:in_off[v+1]]."""
    n: int
    in_off: np.ndarray   # int32 [n+1]
    in_src: np.ndarray   # int32 [E]
    weight: np.ndarray   # float32 [E]: IC probability or LT weight of the edge
    model: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_edges(self) -> int:
        return int(self.in_src.shape[0])

    def in_degree(self) -> np.ndarray:
        return np.diff(self.in_off).astype(np.int64)


def _to_in_csr(n: int, src: np.ndarray, dst: np.ndarray):
    """Sort edges by (dst, src, generation index); return in_off, in_src, order."""
    key = (dst.astype(np.int64) << 32) | src.astype(np.int64)
    order = np.argsort(key, kind="stable")
    in_src = src[order].astype(np.int32)
    cnt = np.bincount(dst, minlength=n)
    in_off = np.zeros(n + 1, np.int64)
    np.cumsum(cnt, out=in_off[1:])
    if in_off[-1] >= 2**31:
        raise ValueError("edge count exceeds int32 CSR")
    return in_off.astype(np.int32), in_src, order


def rmat_edges(scale: int, num_edges: int, seed: int, abc=RMAT_ABC):
    """R-MAT edges (Chakrabarti et al. 2004): per edge and per level one
    quadrant draw; duplicates and self-loops kept so |E| is exact; vertex
    ids relabelled by a seeded random permutation so hubs are spread out."""
    a, b, c = abc
    rng = np.random.default_rng(seed)
    cut0 = np.uint32(int(a * 2**32))
    cut1 = np.uint32(int((a + b) * 2**32))
    cut2 = np.uint32(int((a + b + c) * 2**32))
    src = np.zeros(num_edges, np.uint32)
    dst = np.zeros(num_edges, np.uint32)
    for _ in range(scale):
        r = rng.integers(0, 2**32, num_edges, dtype=np.uint32)
        sbit = r >= cut1
        dbit = ((r >= cut0) & (r < cut1)) | (r >= cut2)
        src <<= 1
        dst <<= 1
        src |= sbit
        dst |= dbit
    n = 1 << scale
    perm = rng.permutation(n).astype(np.uint32)
    return n, perm[src], perm[dst]


def chung_lu_edges(n: int, avg_deg: int, exponent: float, seed: int):
    """Directed Chung-Lu graph: n*avg_deg edges, both endpoints drawn with
    probability proportional to w_i = (i+1)^(-1/(exponent-1))."""
    rng = np.random.default_rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (exponent - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = n * avg_deg
    src = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1)
    dst = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1)
    perm = rng.permutation(n)
    return n, perm[src].astype(np.uint32), perm[dst].astype(np.uint32)


def ic_uniform_weights(E: int, seed: int, hi: float = 0.1) -> np.ndarray:
    """IC probabilities uniform in [0, hi) as fp32 (the paper's [0, 0.1])."""
    rng = np.random.default_rng(seed)
    return (rng.random(E, dtype=np.float32) * np.float32(hi)).astype(np.float32)


def ic_weighted_cascade(in_off: np.ndarray) -> np.ndarray:
    """Weighted cascade: p(u, v) = 1 / indeg(v) as fp32."""
    deg = np.diff(in_off.astype(np.int64))
    per_v = np.float32(1.0) / np.maximum(deg, 1).astype(np.float32)
    return np.repeat(per_v, deg).astype(np.float32)


def lt_normalized_weights(in_off: np.ndarray, seed: int) -> np.ndarray:
    """LT weights: uniform raw weights divided by their per-vertex sum (fp64),
    stored as fp32 so that each in-weight sum is 1 up to fp32 rounding."""
    rng = np.random.default_rng(seed)
    E = int(in_off[-1])
    raw = rng.random(E)
    deg = np.diff(in_off.astype(np.int64))
    owner = np.repeat(np.arange(deg.shape[0]), deg)
    tot = np.bincount(owner, weights=raw, minlength=deg.shape[0])
    return (raw / tot[owner]).astype(np.float32)


def make_graph(kind: str, model: int, *, scale: int = 0, num_edges: int = 0, n: int = 0,
               avg_deg: int = 0, exponent: float = 2.1, graph_seed: int, weight_seed: int,
               weights: str = "uniform", name: str = "") -> Graph:
    if kind == "rmat":
        n, src, dst = rmat_edges(scale, num_edges, graph_seed)
    elif kind == "chunglu":
        n, src, dst = chung_lu_edges(n, avg_deg, exponent, graph_seed)
    else:
        raise ValueError(kind)
    in_off, in_src, _ = _to_in_csr(n, src, dst)
    del src, dst
    if model == IC:
        w = ic_weighted_cascade(in_off) if weights == "wc" else ic_uniform_weights(
            in_src.shape[0], weight_seed)
    else:
        w = lt_normalized_weights(in_off, weight_seed)
    return Graph(n=n, in_off=in_off, in_src=in_src, weight=w, model=model, name=name,
                 meta=dict(kind=kind, scale=scale, weights=weights))


def tiny_graph(n: int, edges, weights, model: int = IC) -> Graph:
    """A hand-written graph from (u, v) pairs (edge u -> v) and weights."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(weights, dtype=np.float32)
    src = e[:, 0].astype(np.uint32)
    dst = e[:, 1].astype(np.uint32)
    in_off, in_src, order = _to_in_csr(n, src, dst)
    return Graph(n=n, in_off=in_off, in_src=in_src, weight=w[order].astype(np.float32),
                 model=model, name="tiny")


def random_small_graph(n: int, num_edges: int, seed: int, model: int = IC,
                       p_hi: float = 0.1) -> Graph:
    """Uniform random directed multigraph for small parity and pin cases."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, num_edges).astype(np.uint32)
    dst = rng.integers(0, n, num_edges).astype(np.uint32)
    in_off, in_src, _ = _to_in_csr(n, src, dst)
    if model == IC:
        w = (rng.random(num_edges, dtype=np.float32) * np.float32(p_hi)).astype(np.float32)
    else:
        w = lt_normalized_weights(in_off, seed + 1)
    return Graph(n=n, in_off=in_off, in_src=in_src, weight=w, model=model, name="random")


# --------------------------------------------------------------- named configs
@dataclass
class Workload:
    name: str
    graph: Graph
    theta: int          # 0: sample count from the IMM bound
    k: int
    eps: float = 0.13
    seed: int = 0       # sampling seed
    selector: str = "greedy"
    m: int = 1
    delta: float = 0.077
    alphas: tuple = (1.0,)
    part_seed: int = 0


def config(c: int) -> Workload:
    """The five evaluation configurations (1-based)."""
    if c == 1:
        g = make_graph("rmat", IC, scale=12, num_edges=32768, graph_seed=1001,
                       weight_seed=2001, weights="uniform", name="rmat12-ic-u0.1")
        return Workload("rmat12_ic_uniform", g, theta=16384, k=16, seed=3001)
    if c == 2:
        g = make_graph("rmat", IC, scale=20, num_edges=1 << 24, graph_seed=1002,
                       weight_seed=2002, weights="wc", name="rmat20-ic-wc")
        return Workload("rmat20_ic_wc", g, theta=1 << 20, k=100, seed=3002)
    if c == 3:
        g = make_graph("rmat", LT, scale=22, num_edges=1 << 26, graph_seed=1003,
                       weight_seed=2003, name="rmat22-lt")
        return Workload("rmat22_lt_greedirs", g, theta=0, k=100, eps=0.13, seed=3003,
                        selector="greediris", m=64, delta=0.077, alphas=(1.0, 0.125),
                        part_seed=4003)
    raise ValueError(c)


def batch_tasks(count: int = 256, seed: int = 5004):
    """Task list of the batched configuration: Chung-Lu graphs (exponent 2.1),
    n log-uniform in [2^10, 2^16], average degree in [8, 32], IC (uniform
    p in [0, 0.1)) or LT with probability 1/2, k in [8, 64], theta = 2^[14, 18]."""
    rng = np.random.default_rng(seed)
    tasks = []
    for t in range(count):
        n = int(round(2.0 ** rng.uniform(10, 16)))
        d = int(rng.integers(8, 33))
        model = int(rng.integers(0, 2))
        k = int(rng.integers(8, 65))
        theta = 1 << int(rng.integers(14, 19))
        tasks.append(dict(n=n, avg_deg=d, model=model, k=k, theta=theta,
                          graph_seed=10000 + t, weight_seed=20000 + t, seed=30000 + t))
    return tasks


def batch_graph(task: dict) -> Graph:
    return make_graph("chunglu", task["model"], n=task["n"], avg_deg=task["avg_deg"],
                      graph_seed=task["graph_seed"], weight_seed=task["weight_seed"],
                      name="chunglu-%d" % task["n"])
