"""Serving: influence-maximization queries over resident graphs with
device-resident RRR pools and continuous batching.

* A SamplePool holds the RRR sets [0, count) of one (graph, seed, stream) in
  device memory and only ever grows by sample-id range (the samples of
  earlier martingale rounds are kept, Sec. 3.2).  Because every set is a pure
  function of its ids, the prefix [0, theta) of a pool is exactly what fresh
  sampling of theta sets returns, so a query answered from pools has the same
  seeds as the same query answered alone (im_solve), bit for bit.
* solve_pooled() runs IMM (Alg. 1, greedy selector) over pool prefixes; the
  schedule and every round decision come from the library (im_imm_plan,
  im_imm_round, im_imm_theta), the same calls im_solve makes.
* Server runs queries in S slots.  Each slot is a thread with its own HIP
  stream and its own workspace (the binding keeps one per stream; the
  library allocates nothing and releases the GIL inside its calls), so the
  work of queries admitted together overlaps on the GPU.  A query is
  admitted when a slot is free and its HBM footprint estimate fits what the
  budget leaves after the resident bytes (pools and the slots' workspaces,
  both measured); others wait in arrival order.
Every step on the device is a library kernel; this module schedules them.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass, field

import torch

from . import binding as B


class SamplePool:
    """RRR sets [0, count) of (graph, seed, stream_tag), grown by id range."""

    def __init__(self, graph: B.Graph, seed: int, stream_tag: int):
        self.g = graph
        self.seed = seed
        self.tag = stream_tag
        self.lock = threading.Lock()
        dev = graph.in_off.device
        self.count = 0
        self.total = 0
        self.off = torch.zeros(1024, dtype=torch.int64, device=dev)
        self.mem = torch.empty(1 << 16, dtype=torch.int32, device=dev)
        self.extensions = 0
        self.sets_sampled = 0

    def nbytes(self) -> int:
        return self.off.numel() * 8 + self.mem.numel() * 4

    def _grow(self, t: torch.Tensor, need: int, stream) -> torch.Tensor:
        if t.numel() >= need:
            return t
        cap = max(need, 2 * t.numel())
        n = torch.empty(cap, dtype=t.dtype, device=t.device)
        with torch.cuda.stream(stream):
            n[:t.numel()].copy_(t)
        # the old tensor may have been allocated on another slot's stream and
        # is freed as soon as the pool drops it: its block must not be handed
        # to that stream's next allocation while this copy still reads it
        t.record_stream(stream)
        return n

    def prefix(self, want: int, stream):
        """(off view [want+1], mem, members) of the first `want` sets, sampling
        the missing ones first."""
        with self.lock:
            if want > self.count:
                self._extend(want, stream)
            off, mem = self.off, self.mem
        off_v = off[:want + 1]
        with torch.cuda.stream(stream):
            members = int(off_v[want].item())
        return off_v, mem, members

    def _extend(self, want: int, stream):
        add = want - self.count
        avg = (self.total / self.count) if self.count else 32.0
        off_tmp = torch.empty(add + 1, dtype=torch.int64, device=self.off.device)
        est = int(avg * add * 1.25) + 4096
        for _ in range(3):
            self.mem = self._grow(self.mem, self.total + est, stream)
            stream.synchronize()
            tail = self.mem[self.total:]
            got = B.sample_into(self.g, self.seed, self.tag, self.count, add, off_tmp, tail,
                                stream=stream)
            if got >= 0:
                break
            est = int(-got * 1.25) + 4096
        else:
            raise B.ImError(B.IM_ERANGE, "pool extension")
        self.off = self._grow(self.off, want + 1, stream)
        with torch.cuda.stream(stream):
            self.off[self.count + 1:want + 1].copy_(off_tmp[1:] + self.total)
        stream.synchronize()
        self.count = want
        self.total += got
        self.extensions += 1
        self.sets_sampled += add


class _Prefix:
    """Adapter: a pool prefix seen as a sample-major collection."""

    def __init__(self, off, mem, members):
        self.off = off
        self.mem = mem[:members]
        self.total = members

    @property
    def count(self):
        return self.off.numel() - 1


def _select(n: int, pref: _Prefix, k: int, stream):
    inc_off, inc_mem = B.build_incidence(n, pref, stream=stream)
    seeds, gains, nsel, cov = B.greedy_cover(n, pref, inc_off, inc_mem, k, stream=stream)
    with torch.cuda.stream(stream):
        c = int(cov.item())
        ns = int(nsel.item())
        s = seeds[:ns].cpu().tolist()
    return s, c


def solve_pooled(graph: B.Graph, pools: tuple, k: int, eps: float, stream) -> dict:
    """IMM with the standard greedy over resident pools (martingale pool on
    stream 0, final pool on stream 1); the library takes every decision."""
    n = graph.n
    plan = B.imm_plan(n, k, eps)
    lb = 1.0
    th = plan["theta1"]
    rounds_run = 0
    mart = 0
    for i in range(1, plan["rounds"] + 1):
        if i > 1:
            th *= 2
        off, mem, members = pools[0].prefix(th, stream)
        _, cov = _select(n, _Prefix(off, mem, members), k, stream)
        rounds_run = i
        mart = th
        stop, lbx = plan.round(i, th, cov)
        if stop:
            lb = lbx
            break
    theta = plan.theta(lb)
    off, mem, members = pools[1].prefix(theta, stream)
    seeds, cov = _select(n, _Prefix(off, mem, members), k, stream)
    return {"seeds": seeds, "coverage": cov, "theta": theta, "rounds": rounds_run,
            "lower_bound": lb, "martingale_samples": mart, "final_total": members}


class Admission:
    """Arrival-order admission by slots and HBM footprint (host logic only).

    A query is admitted when fewer than `slots` queries are in flight and its
    footprint fits what the resident bytes (`held`: pools and the slots'
    workspaces) and the in-flight queries leave of `budget`; the head of the
    line is never overtaken.  A query larger than all that is admitted alone."""

    def __init__(self, slots: int, budget: int):
        self.slots = slots
        self.budget = budget
        self.waiting = []
        self.in_flight = 0
        self.reserved = 0
        self.max_in_flight = 0

    def push(self, item, footprint: int):
        self.waiting.append((item, footprint))

    def pop(self, held: int = 0):
        if not self.waiting or self.in_flight >= self.slots:
            return None
        item, fp = self.waiting[0]
        if self.in_flight > 0 and held + self.reserved + fp > self.budget:
            return None
        self.waiting.pop(0)
        self.in_flight += 1
        self.reserved += fp
        self.max_in_flight = max(self.max_in_flight, self.in_flight)
        return item, fp

    def release(self, footprint: int):
        self.in_flight -= 1
        self.reserved -= footprint


@dataclass
class Query:
    qid: int
    graph: str
    k: int
    eps: float
    arrival: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0
    result: dict = field(default_factory=dict)
    footprint: int = 0
    error: BaseException | None = None  # set when its solve raised


class Server:
    """Continuous batching over resident graphs.

    graphs: name -> prepared Graph.  Pools are created on first use per
    (graph, stream).  slots: queries in flight at once.  hbm_budget: bytes
    that admitted queries' footprint estimates may sum to.  streams: the
    slots' streams (one per slot, default priority), to be reused across
    servers: the binding keeps a workspace per stream, so a server on
    streams that served before starts with those workspaces in place; None
    creates new ones.

    Slots overlap only if their streams sit on different hardware queues.
    HIP hands a stream its queue on first use, a new one while fewer than
    GPU_MAX_HW_QUEUES exist (default 4), so the process should set that
    variable, before HIP starts, above the number of streams it uses; with
    fewer, two slots can share a queue and run one after the other."""

    def __init__(self, graphs: dict, seed: int, slots: int = 4, hbm_budget: int = 64 << 30,
                 streams=None):
        if streams is not None and len(streams) != slots:
            raise ValueError("streams: one per slot")
        B.lib()
        self.graphs = graphs
        self.seed = seed
        self.slots = slots
        self.pools = {}
        self.pools_lock = threading.Lock()
        self.cv = threading.Condition()
        self.adm = Admission(slots, hbm_budget)
        self.done = []
        self.stopping = False
        self.avg_set = {}          # graph -> observed members per set
        self.theta_seen = {}       # graph -> largest final theta so far
        self.threads = [threading.Thread(target=self._worker, daemon=True)
                        for _ in range(slots)]
        self.streams = (list(streams) if streams is not None else
                        [torch.cuda.Stream() for _ in range(slots)])
        for j, t in enumerate(self.threads):
            t.slot = j
            t.start()

    def _pools(self, name):
        with self.pools_lock:
            if name not in self.pools:
                g = self.graphs[name]
                self.pools[name] = (SamplePool(g, self.seed, 0), SamplePool(g, self.seed, 1))
            return self.pools[name]

    def footprint(self, q: Query) -> int:
        """HBM bytes a query needs on top of the resident ones: covering
        subsets and greedy state for its largest prefix, and the pool growth
        and sampling staging an extension to that prefix can take (estimated
        from earlier queries on the same graph, else from the first
        martingale round)."""
        g = self.graphs[q.graph]
        plan = B.imm_plan(g.n, q.k, q.eps)
        theta = max(self.theta_seen.get(q.graph, 0), 8 * plan["theta1"])
        members = int(theta * self.avg_set.get(q.graph, 32.0))
        cover = 8 * (g.n + 1) + 4 * members + 4 * g.n + theta + 16 * q.k
        extension = 2 * (8 * theta + 4 * members)  # staging arena + metadata, pool growth
        return cover + extension

    def resident_bytes(self) -> int:
        """Pools plus the workspaces of the slots' streams (measured)."""
        with self.pools_lock:
            pools = sum(p0.nbytes() + p1.nbytes() for p0, p1 in self.pools.values())
        return pools + sum(B.workspace_bytes(s) for s in self.streams)

    @property
    def max_in_flight(self) -> int:
        return self.adm.max_in_flight

    def submit(self, q: Query):
        q.footprint = self.footprint(q)
        with self.cv:
            self.adm.push(q, q.footprint)
            self.cv.notify_all()

    def _worker(self):
        stream = self.streams[threading.current_thread().slot]
        while True:
            with self.cv:
                got = self.adm.pop(self.resident_bytes())
                while got is None:
                    if self.stopping and not self.adm.waiting:
                        return
                    self.cv.wait()
                    got = self.adm.pop(self.resident_bytes())
            q = got[0]
            q.admitted = time.perf_counter()
            g = self.graphs[q.graph]
            res = None
            try:
                with torch.cuda.stream(stream):
                    res = solve_pooled(g, self._pools(q.graph), q.k, q.eps, stream)
                q.result = res
            except Exception as e:  # the query finishes with its error; the slot goes on
                q.error = e
            q.finished = time.perf_counter()
            with self.cv:
                self.adm.release(q.footprint)
                self.done.append(q)
                if res is not None:
                    self.theta_seen[q.graph] = max(self.theta_seen.get(q.graph, 0), res["theta"])
                    if res["theta"]:
                        self.avg_set[q.graph] = res["final_total"] / res["theta"]
                self.cv.notify_all()

    def close(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    def pool_stats(self) -> dict:
        out = {}
        for name, (p0, p1) in self.pools.items():
            out[name] = {"martingale_sets": p0.count, "final_sets": p1.count,
                         "sets_sampled": p0.sets_sampled + p1.sets_sampled,
                         "extensions": p0.extensions + p1.extensions,
                         "hbm_bytes": p0.nbytes() + p1.nbytes()}
        return out


def run_arrivals(server: Server, queries: list, t0: float | None = None):
    """Submits queries at their arrival offsets (seconds from t0) and waits
    for all of them; returns the finished queries in id order.  Raises the
    first failed query's error (by id) once all have finished."""
    t0 = time.perf_counter() if t0 is None else t0
    for q in sorted(queries, key=lambda q: q.arrival):
        dt = t0 + q.arrival - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        q.arrival = t0 + q.arrival
        server.submit(q)
    with server.cv:
        while len(server.done) < len(queries):
            server.cv.wait()
    out = sorted(server.done, key=lambda q: q.qid)
    failed = [q for q in out if q.error is not None]
    if failed:
        raise RuntimeError("%d of %d queries failed; query %d: %r" %
                           (len(failed), len(out), failed[0].qid, failed[0].error)) from failed[0].error
    return out


def latency_summary(queries: list) -> dict:
    lat = sorted(q.finished - q.arrival for q in queries)
    span = max(q.finished for q in queries) - min(q.arrival for q in queries)

    def pct(p):
        return lat[min(len(lat) - 1, int(math.ceil(p * len(lat))) - 1)]
    return {"queries": len(lat), "queries_per_s": len(lat) / span if span > 0 else None,
            "p50_s": pct(0.50), "p99_s": pct(0.99), "mean_s": sum(lat) / len(lat),
            "makespan_s": span}
