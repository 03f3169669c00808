#!/usr/bin/env python3
"""Benchmark of the influence-maximization hot path on one MI355X.

Default workload (the paper's method end to end, every step of the path):
R-MAT scale 22 (2^22 vertices, 2^26 edges), LT with uniform in-weights
normalised per vertex, IMM with epsilon = 0.13 and k = 100, GreediRIS
selection with m = 64 partitions, delta = 0.077 and truncation alpha = 0.125.
A step is one whole im_solve: the martingale rounds (sampling, covering
subsets, RandGreedi local greedy over the 64 partitions, streaming bucket
cover, final choice, the lower-bound test), then theta fresh samples and the
same selection on them.  Inputs are resident in HBM before the timed region.
The same run also times alpha = 1 and the plain IC weighted-cascade workload
(R-MAT scale 20, theta = 2^20, greedy k = 100) and reports them as extra keys.

Prints one JSON line on stdout.  `roofline` describes the dominant kernel
(algorithmic bytes per launch over its event-timed duration, from HIP events
the library records on the solve's stream); `cpu_baseline` times the
single-threaded CPU oracle on the same solve.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
HW_QUEUES = 16                   # hardware queues per process (one per stream used here)
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit integer VALU lane-ops/s (full rate)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sampling_bytes(sets, total, examined, live, run_length=True):
    """Algorithmic bytes of IC sampling: per set its offset (8 B); per member
    its two in-CSR offsets read (8 B), its run-length table entry read (8 B,
    when the graph has the table) and its id written (4 B); per examined
    in-edge or run-length draw 4 B (the threshold; draws read nothing, so this
    over-counts them); per live in-edge its source id (4 B)."""
    return 8 * sets + (20 if run_length else 12) * total + 4 * examined + 4 * live


def lt_sampling_bytes(sets, total, examined):
    """Algorithmic bytes of LT sampling: per set its offset (8 B); per member
    its two in-CSR offsets read (8 B), the kept edge's source read (4 B) and
    its id written (4 B); per binary-search probe one threshold (4 B; the
    examined counter charges ceil(log2(indeg + 1)) probes per expanded vertex)."""
    return 8 * sets + 16 * total + 4 * examined


# Measured HBM traffic per launch of a kernel: profiles/traffic_<workload>.md
# holds lines "traffic <kernel> bytes_per_launch=<B> source_sha256=<H>", taken
# from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled against a plain copy.
# A figure counts only while the kernel's sources hash to H.
MAIN_IC = "k_sample_ic_small"
KERNEL_SOURCES = {
    MAIN_IC: ["csrc/common.h", "csrc/sample.h", "csrc/sample.hip"],
    "k_sample_big": ["csrc/common.h", "csrc/sample.h", "csrc/sample.hip"],
    "k_sample_lt": ["csrc/common.h", "csrc/sample.h", "csrc/sample.hip"],
}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2408_10982_amd", rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % workload)
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    want = kernel_source_hash(kernel)
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 4 and parts[0] == "traffic" and parts[1] == kernel:
                kv = dict(x.split("=", 1) for x in parts[2:])
                if kv.get("source_sha256") == want:
                    return int(kv["bytes_per_launch"])
    return None


def cpu_baseline(w, sample_sets):
    import numpy as np  # noqa: F401

    import oracle as O
    g = w.graph
    thr = O.thresholds(g.model, g.in_off, g.weight)
    t0 = time.perf_counter()
    r = O.sample(g.model, g.in_off, g.in_src, thr, w.seed, 0, 0, sample_sets)
    io, im_ = O.incidence(g.n, r)
    O.greedy(g.n, sample_sets, io, im_, w.k, lazy=True)
    dt = time.perf_counter() - t0
    what = ("all %d RRR sets of the workload" % w.theta if sample_sets == w.theta else
            "RRR sets 0..%d of the %d-set workload" % (sample_sets - 1, w.theta))
    return {"value": sample_sets / dt, "unit": "RRR sets/s", "cores": 1, "kind": "oracle",
            "sample": "%s (same graph, seed, stream), then covering subsets and greedy k=%d "
                      "over them; %.1f s" % (what, w.k, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 24 solves for config 3, else 5)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--tasks", type=int, default=256)
    ap.add_argument("--queries", type=int, default=120,
                    help="config 5: queries per arrival rate")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--alpha", type=float, default=0.125)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="configs 1-2: RRR sets the CPU oracle times (0: the whole workload)")
    ap.add_argument("--streams", type=int, default=3,
                    help="configs 1-2: streams the steps alternate over")
    ap.add_argument("--solve-streams", type=int, default=4,
                    help="config 3: solves in flight at once (one host thread and "
                         "stream each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="config 3: skip the alpha = 1 and weighted-cascade extra keys")
    ap.add_argument("--no-autotune", action="store_true",
                    help="config 4: keep the default launch shapes")
    ap.add_argument("--tune-tasks", type=int, default=32,
                    help="config 4: tasks the autotuner times each setting on")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 24 if args.config == 3 else 5
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    # HIP gives a stream its hardware queue when the stream is first used: a
    # new queue while fewer than GPU_MAX_HW_QUEUES exist (HIP's default is 4),
    # else the least used one, ties going to the newest.  Work of streams on
    # one queue runs one after the other, so with 4 queues two of the four
    # solve streams (or serving slots) can share one: 18.5 against 14 ms per
    # solve measured.  This process uses fewer than 16 streams, so with 16
    # each stream has a queue of its own.  It must be set before HIP starts.
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < HW_QUEUES:
        os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)

    import torch

    import paper_2408_10982_amd as im
    import workloads as W

    torch.cuda.set_device(0)
    try:
        run(args, im, W, torch)
    finally:
        # drop the workspaces and captured graphs while the runtime is whole,
        # so that exit-time teardown frees no HIP memory of ours
        torch.cuda.synchronize()
        im.release()


def run(args, im, W, torch):
    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "copies": 3}), flush=True)
        return
    if args.config == 4:
        return bench_batch(args, im, W, torch)
    if args.config == 5:
        return bench_serve(args, im, W, torch)
    t0 = time.time()
    w = W.config(args.config)
    g = w.graph
    log("workload %s: n=%d E=%d theta=%d k=%d (generated in %.1fs)" %
        (w.name, g.n, g.num_edges, w.theta, w.k, time.time() - t0))
    G = im.prepare_graph(g.in_off, g.in_src, g.weight, g.model)
    torch.cuda.synchronize()
    if args.config == 3:
        return bench_imm(args, w, G, im, W, torch)
    out = run_plain(args, w, G, im, torch)
    if not args.no_cpu_baseline:
        n_cpu = args.cpu_sample if args.cpu_sample > 0 else w.theta
        log("cpu baseline: oracle on %d sets" % n_cpu)
        out["cpu_baseline"] = cpu_baseline(w, min(n_cpu, w.theta))
    print(json.dumps(out), flush=True)


def run_plain(args, w, G, im, torch, steps=None, warmup=None):
    """Configs 1-2: a step samples theta sets, builds the covering subsets and
    runs greedy; steps alternate over --streams streams."""
    g = w.graph
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    cap = [max(4 * w.theta, 1 << 20)]

    # Step i runs on stream i mod S: its covering subsets and greedy (a chain
    # of small launches) overlap the next step's sampling.  Every step does
    # all of its work; each stream has its own workspace.
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream()
                                               for _ in range(max(args.streams, 1) - 1)]

    def step(record, s):
        with torch.cuda.stream(s):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            r = im.sample_rrr(G, w.seed, 0, 0, w.theta, capacity=cap[0])
            cap[0] = max(cap[0], r.total)
            ev[1].record()
            io, imem = im.build_incidence(g.n, r)
            ev[2].record()
            seeds, gains, nsel, cov = im.greedy_cover(g.n, r, io, imem, w.k)
            ev[3].record()
        if record is not None:
            record.append((r, ev, (seeds, gains, nsel, cov)))
        return r

    def timed(n_streams, nsteps, record):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(nsteps):
            step(record, streams[i % n_streams])
        torch.cuda.synchronize()
        return time.perf_counter() - t

    for i in range(max(warmup, len(streams))):
        step(None, streams[i % len(streams)])
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    serial = []
    ms_serial = 1e3 * timed(1, steps, serial) / steps
    recs = []
    t_total = timed(len(streams), steps, recs)
    log("timed %d steps in %.3fs on %d streams (one stream: %.3f ms/step)" %
        (steps, t_total, len(streams), ms_serial))
    ms_step = 1e3 * t_total / steps

    r0, _, out0 = recs[0]
    seeds0 = out0[0].cpu().tolist()
    cov0 = int(out0[3].item())
    for r, ev, out in recs[1:] + serial:  # every timed step computes the same result
        assert out[0].cpu().tolist() == seeds0 and int(out[3].item()) == cov0
    # per-phase and per-kernel times from the one-stream steps (no overlap)
    ms_sample = sum(ev[0].elapsed_time(ev[1]) for _, ev, _ in serial) / len(serial)
    ms_inc = sum(ev[1].elapsed_time(ev[2]) for _, ev, _ in serial) / len(serial)
    ms_greedy = sum(ev[2].elapsed_time(ev[3]) for _, ev, _ in serial) / len(serial)
    st = r0.stats
    ms_main = sum(r.stats["ms_main"] for r, _, _ in serial) / len(serial)
    ms_large = sum(r.stats["ms_large"] for r, _, _ in serial) / len(serial)
    ms_canon = sum(r.stats["ms_canon"] for r, _, _ in serial) / len(serial)

    small_sets = w.theta - st["large_sets"]
    b_main = sampling_bytes(small_sets, st["total"] - st["large_total"],
                            st["examined"] - st["large_examined"], st["live"] - st["large_live"])
    b_large = sampling_bytes(st["large_sets"], st["large_total"], st["large_examined"],
                             st["large_live"])
    kernels = {
        MAIN_IC: (b_main, ms_main, st["examined"] - st["large_examined"]),
        "k_sample_big": (b_large, ms_large, st["large_examined"]),
    }
    dom = max(kernels, key=lambda k: kernels[k][1])
    bytes_dom, ms_dom, ex_dom = kernels[dom]
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9
    # 4-edge Philox4x32-10 groups: ~200 full-rate-equivalent integer ops each
    # (the 40 32x32 multiplies run at quarter rate) -> ~50 per examined edge
    alu_tops = 50.0 * ex_dom / (ms_dom * 1e-3) / 1e12
    traffic = measured_traffic(w.name, dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "algorithmic_bytes": int(bytes_dom),
                "kernel_ms": round(ms_dom, 4),
                "alu_view": {"int_tops": round(alu_tops, 2), "peak_int_tops": INT_PEAK_TOPS,
                             "frac": round(alu_tops / INT_PEAK_TOPS, 4)}}

    value = w.theta / (ms_step * 1e-3)
    return {
        "metric": "RRR sets/s through sampling + max-k-cover (bit-exact)",
        "value": round(value, 1),
        "unit": "RRR sets/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "streams": len(streams),
        "ms_per_step_one_stream": round(ms_serial, 3),
        "config": {"workload": w.name, "graph": "R-MAT (0.57,0.19,0.19) scale %d, %d edges"
                   % (g.n.bit_length() - 1, g.num_edges),
                   "model": "IC weighted cascade" if w.name == "rmat20_ic_wc"
                   else "IC uniform [0,0.1)",
                   "theta": w.theta, "k": w.k, "selector": "greedy"},
        "sampling_sets_per_s": round(w.theta / (ms_sample * 1e-3), 1),
        "cover_ms": round(ms_inc + ms_greedy, 3),
        "breakdown_ms": {"sample": round(ms_sample, 3), "sample_main_kernel": round(ms_main, 3),
                         "sample_large_kernel": round(ms_large, 3),
                         "sample_canonical": round(ms_canon, 3),
                         "incidence": round(ms_inc, 3), "greedy": round(ms_greedy, 3)},
        "counts": {"sum_rrr": st["total"], "examined_edges": st["examined"],
                   "live_edges": st["live"], "large_sets": st["large_sets"],
                   "redo_examined": st["redo_examined"],
                   "coverage": cov0, "seeds_head": seeds0[:8]},
        "roofline": roofline,
    }


def bench_batch(args, im, W, torch):
    """Batched configuration: the Chung-Lu task list (mixed IC/LT, uneven n,
    k, theta); a step is every task sampled and covered.  Batched = one
    im_solve_batch call; per-query = the plain loop of sample + incidence +
    greedy calls per task.  Both produce the same seeds (checked)."""
    spec = W.batch_tasks(args.tasks)
    t0 = time.time()
    graphs = [W.batch_graph(t) for t in spec]
    log("generated %d graphs in %.1fs" % (len(graphs), time.time() - t0))
    prepared = [im.prepare_graph(g.in_off, g.in_src, g.weight, g.model) for g in graphs]
    tasks = [(G, t["seed"], 0, t["k"], t["theta"]) for G, t in zip(prepared, spec)]
    torch.cuda.synchronize()

    tuning = None
    if not args.no_autotune:
        # launch shapes from measurements on a spread of the tasks; every
        # setting must give the same seeds (checked by the tuner)
        from paper_2408_10982_amd import autotune as AT
        sub = tasks[::max(1, len(tasks) // max(1, args.tune_tasks))][:args.tune_tasks]

        def run():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            o, _ = im.solve_batch(sub)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1), tuple((tuple(x["seeds"]), x["coverage"]) for x in o)

        res_t = AT.tune(run, knobs=("sample_blocks", "big_shape", "dense_ratio"), log=log)
        tuning = {"settings": res_t["settings"], "tasks": len(sub),
                  "default_ms": round(res_t["default_ms"], 2), "tuned_ms": round(res_t["ms"], 2),
                  "trials": len(res_t["trials"]), "seconds": res_t["seconds"]}
        log("autotune: %s" % tuning)

    def loop():
        res = []
        for (G, seed, tag, k, theta), g in zip(tasks, graphs):
            r = im.sample_rrr(G, seed, tag, 0, theta, capacity=cap.get(id(G), 4 * theta))
            cap[id(G)] = max(cap.get(id(G), 0), r.total)
            io, imem = im.build_incidence(g.n, r)
            res.append(im.greedy_cover(g.n, r, io, imem, k))
        torch.cuda.synchronize()
        return res

    cap = {}
    for i in range(args.warmup):
        out_b, st = im.solve_batch(tasks)
        log("warmup batched %d: %s" % (i, st))
    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out_b, st = im.solve_batch(tasks)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = loop()
    dt_l = (time.perf_counter() - t0) / args.steps
    for ob, (seeds, gains, nsel, cov) in zip(out_b, res):
        n = int(nsel.item())
        assert ob["seeds"] == seeds[:n].cpu().tolist() and ob["coverage"] == int(cov.item())
    nt = len(tasks)
    out = {
        "metric": "batched queries/s (sampling + max-k-cover per task, bit-exact)",
        "tuning": tuning,
        "value": round(nt / dt_b, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt_b * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "chunglu_batch_%d" % nt, "graphs": "Chung-Lu exponent 2.1, "
                   "n log-uniform 2^10..2^16, avg degree 8..32, IC U[0,0.1) or LT",
                   "k": "8..64", "theta": "2^14..2^18", "selector": "greedy"},
        "per_query_loop_queries_per_s": round(nt / dt_l, 2),
        "speedup_vs_per_query": round(dt_l / dt_b, 3),
        "batch_stats": st,
    }
    print(json.dumps(out), flush=True)


def run_plain_arrivals(im, graphs, spec, arr, seed):
    """The plain per-query path under an arrival sequence, measured: queries
    in arrival order, one at a time, each answered alone with fresh sampling
    (im_solve) once it has arrived and the previous one has finished.
    Returns (results, latencies in s, makespan in s)."""
    import torch
    order = sorted(range(len(spec)), key=lambda j: arr[j])
    res, lat, fin = [None] * len(spec), [0.0] * len(spec), []
    t0 = time.perf_counter()
    for j in order:
        name, k, eps = spec[j]
        a = t0 + arr[j]
        dt = a - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        res[j] = im.solve(graphs[name], k, eps, seed=seed)
        torch.cuda.synchronize()
        end = time.perf_counter()
        lat[j] = end - a
        fin.append(end)
    return res, lat, max(fin) - (t0 + min(arr))


def _pcts(lat):
    import numpy as np
    s = sorted(lat)
    return {"p50_s": s[int(np.ceil(0.5 * len(s))) - 1], "p99_s": s[int(np.ceil(0.99 * len(s))) - 1],
            "mean_s": sum(s) / len(s)}


def bench_serve(args, im, W, torch):
    """Served configuration: IM queries (graph, model, k, eps) over resident
    R-MAT graphs (scales 18, 20, 22; IC weighted cascade and LT), Poisson
    arrivals at six rates around the plain path's saturation rate, then a
    burst.

    Plain path: each query alone with fresh sampling (im_solve), one at a
    time in arrival order, measured under the same arrival sequence.  Served
    path: the Server (resident pools extended on demand, continuous batching
    over --slots streams, admission by HBM footprint over the measured
    resident bytes), started with empty pools for each rate.  Every served
    result is checked equal to the plain result."""
    import numpy as np

    from paper_2408_10982_amd import serve as S
    graphs = {}
    t0 = time.time()
    for scale in (18, 20, 22):
        n, src, dst = W.rmat_edges(scale, 16 << scale, 6000 + scale)
        in_off, in_src, _ = W._to_in_csr(n, src, dst)
        del src, dst
        graphs["s%d-ic" % scale] = im.prepare_graph(in_off, in_src, W.ic_weighted_cascade(in_off),
                                                    im.IC)
        graphs["s%d-lt" % scale] = im.prepare_graph(
            in_off, in_src, W.lt_normalized_weights(in_off, 7000 + scale), im.LT)
    torch.cuda.synchronize()
    log("resident graphs ready in %.1fs" % (time.time() - t0))
    rng = np.random.default_rng(5000)
    names = sorted(graphs)
    spec = [(names[int(rng.integers(0, len(names)))], int(rng.integers(10, 201)),
             float(rng.choice([0.5, 0.25, 0.13]))) for _ in range(args.queries)]
    seed = 5005
    # the plain path's saturation rate: every query once, back to back
    im.solve(graphs[spec[0][0]], spec[0][1], spec[0][2], seed=seed)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for name, k, eps in spec:
        im.solve(graphs[name], k, eps, seed=seed)
    torch.cuda.synchronize()
    mu = len(spec) / (time.perf_counter() - t1)
    log("plain path: %.2f queries/s at saturation" % mu)
    points = []
    slot_streams = [torch.cuda.Stream() for _ in range(args.slots)]
    budget = 160 << 30
    # warm-up of the served path: every query once through a server on the
    # slot streams, so that their workspaces have grown to what the queries
    # need before any timing (the plain path's saturation pass above does
    # the same for its stream)
    server = S.Server(graphs, seed=seed, slots=args.slots, hbm_budget=budget,
                      streams=slot_streams)
    try:
        S.run_arrivals(server, [S.Query(qid=j, graph=name, k=k, eps=eps, arrival=0.0)
                                for j, (name, k, eps) in enumerate(spec)])
    finally:
        server.close()
    del server
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("served path warmed up")
    for frac in (0.1, 0.25, 0.5, 0.75, 1.0, 1.2, None):
        if frac is None:  # burst: every query arrives at once (saturation)
            lam = float("inf")
            arr = np.zeros(len(spec))
        else:
            lam = frac * mu
            gaps = np.random.default_rng(5100 + int(frac * 100)).exponential(1.0 / lam, len(spec))
            arr = np.cumsum(gaps) - gaps[0]
        plain_res, plain_lat, plain_span = run_plain_arrivals(im, graphs, spec, arr, seed)
        plain_pt = {"queries_per_s": len(spec) / plain_span, **_pcts(plain_lat)}
        log("lambda %s: plain path done in %.1fs" % (frac or "burst", plain_span))
        server = S.Server(graphs, seed=seed, slots=args.slots, hbm_budget=budget,
                          streams=slot_streams)
        qs = [S.Query(qid=j, graph=name, k=k, eps=eps, arrival=float(arr[j]))
              for j, (name, k, eps) in enumerate(spec)]
        try:
            done = S.run_arrivals(server, qs)
        finally:
            server.close()
        # each rate starts with empty pools; the slots' streams (and their
        # workspaces) carry over, as in a long-running server
        pool_stats, max_in_flight = server.pool_stats(), server.max_in_flight
        resident = server.resident_bytes()
        del server
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for q, p in zip(done, plain_res):
            if q.result["seeds"] != p["seeds"] or q.result["coverage"] != p["coverage"]:
                name, k, eps = spec[q.qid]
                again = im.solve(graphs[name], k, eps, seed=seed)
                log("MISMATCH query %d (%s, k=%d, eps=%g): served theta %s coverage %s rounds "
                    "%s | plain theta %s coverage %s rounds %s | plain again theta %s "
                    "coverage %s seeds equal to served %s, to plain %s"
                    % (q.qid, name, k, eps, q.result.get("theta"), q.result["coverage"],
                       q.result.get("rounds"), p["theta"], p["coverage"], p["rounds"],
                       again["theta"], again["coverage"], again["seeds"] == q.result["seeds"],
                       again["seeds"] == p["seeds"]))
                raise AssertionError("served result differs from the query alone")
        served_pt = S.latency_summary(done)
        served_pt["max_in_flight"] = max_in_flight
        served_pt["resident_bytes_at_close"] = resident
        served_pt["pools"] = pool_stats
        points.append({"lambda_frac_of_plain_saturation": frac if frac else "burst",
                       "lambda_qps": round(lam, 3) if frac else "burst",
                       "served": served_pt, "plain": plain_pt})
        log("lambda %s: served %.2f q/s p50 %.3fs p99 %.3fs | plain %.2f q/s p50 %.3fs p99 %.3fs"
            % (frac or "burst", served_pt["queries_per_s"], served_pt["p50_s"],
               served_pt["p99_s"], plain_pt["queries_per_s"], plain_pt["p50_s"],
               plain_pt["p99_s"]))
    top = points[-2]       # the highest Poisson rate
    burst = points[-1]
    out = {
        "metric": "served queries/s (IMM + greedy per query, bit-exact vs alone), p50/p99",
        "value": round(top["served"]["queries_per_s"], 3), "unit": "queries/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * top["served"]["makespan_s"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serve_rmat18_20_22", "graphs": "R-MAT scales 18/20/22, "
                   "edge factor 16, IC weighted cascade and LT", "queries_per_rate": len(spec),
                   "rates_of_plain_saturation": [0.1, 0.25, 0.5, 0.75, 1.0, 1.2, "burst"],
                   "reduced_from": (None if len(spec) >= 1000 else
                                    "1000 queries per rate (the workload's own size) to bound "
                                    "the run; both paths measured under the same arrivals"),
                   "k": "10..200", "eps": [0.5, 0.25, 0.13], "slots": args.slots,
                   "hbm_budget_bytes": budget, "selector": "greedy (IMM)"},
        "p50_s": round(top["served"]["p50_s"], 4), "p99_s": round(top["served"]["p99_s"], 4),
        "plain_at_same_rate": {k: round(v, 4) for k, v in top["plain"].items()},
        "plain_saturation_qps": round(mu, 3),
        "served_saturation_qps": round(burst["served"]["queries_per_s"], 3),
        "sweep": points,
    }
    print(json.dumps(out), flush=True)


def solve_steps(im, G, w, alpha, steps, warmup, torch, selector=None):
    """Times `steps` whole solves after `warmup` untimed ones; every timed
    solve must give the same seeds.  Returns (seconds per solve, results)."""
    kw = dict(selector=im.SEL_GREEDIRIS if selector is None else selector, m=w.m, delta=w.delta,
              alpha=alpha, seed=w.seed, part_seed=w.part_seed)
    for i in range(warmup):
        res = im.solve(G, w.k, w.eps, **kw)
        log("alpha %g warmup %d: theta=%d rounds=%d coverage=%d sample launches %d passes %d"
            % (alpha, i, res["theta"], res["rounds"], res["coverage"], res["sample_launches"],
               res["sample_passes"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [im.solve(G, w.k, w.eps, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for o in outs[1:]:
        assert o["seeds"] == outs[0]["seeds"] and o["theta"] == outs[0]["theta"]
    return dt, outs


def concurrent_solves(im, G, w, alpha, steps, n_streams, torch, ref_seeds):
    """Times `steps` whole solves spread round-robin over n_streams host
    threads, each with its own stream (and so its own workspace): one solve's
    selection, a chain of small launches, runs beside another's sampling.
    An untimed pass of the same solves runs first; every timed solve must
    give ref_seeds.  Returns seconds per solve."""
    import threading
    kw = dict(selector=im.SEL_GREEDIRIS, m=w.m, delta=w.delta, alpha=alpha, seed=w.seed,
              part_seed=w.part_seed)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    outs = [None] * steps
    errs = []

    def worker(j, timed_run):
        try:
            with torch.cuda.stream(streams[j]):
                for i in range(j, steps, n_streams):
                    o = im.solve(G, w.k, w.eps, **kw)
                    if timed_run:
                        outs[i] = o
        except BaseException as e:  # noqa: BLE001 -- re-raised below
            errs.append(e)

    # an untimed pass of the same shape first: it grows each stream's
    # workspace and gives each stream its hardware queue
    for timed_run in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ths = [threading.Thread(target=worker, args=(j, timed_run)) for j in range(n_streams)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        if errs:
            raise errs[0]
    for o in outs:
        assert o["seeds"] == ref_seeds
    for st in streams:  # these streams end here: so do their workspaces
        im.drop_workspaces(st)
    return dt


def bench_imm(args, w, G, im, W, torch):
    """LT + IMM + GreediRIS: a step is one whole im_solve (martingale rounds,
    final sampling, RandGreedi local greedy over m partitions, streaming
    bucket cover with truncation, final choice).  The steps are timed on one
    stream (phase and kernel times come from those) and with --solve-streams
    solves in flight (the line's value)."""
    dt1s, outs = solve_steps(im, G, w, args.alpha, args.steps, args.warmup, torch)
    res = outs[0]
    n_conc = max(args.solve_streams, 1)
    dt = dt1s
    if n_conc > 1:
        dt = concurrent_solves(im, G, w, args.alpha, args.steps, n_conc, torch, res["seeds"])
        log("%d solves on %d streams: %.3f ms per solve (one stream: %.3f)"
            % (args.steps, n_conc, dt * 1e3, dt1s * 1e3))
    samples = res["theta"] + res["martingale_samples"]
    mean = lambda key: sum(o[key] for o in outs) / len(outs)  # noqa: E731
    # the dominant kernel: the LT walk launch, one per sampling pass
    passes = res["sample_passes"]
    b_launch = lt_sampling_bytes(res["sampled_sets"], res["sampled_total"],
                                 res["sampled_examined"]) / passes
    ms_launch = mean("ms_sample_main") / passes
    achieved = b_launch / (ms_launch * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(w.name, "k_sample_lt"), "kernel": "k_sample_lt",
                "algorithmic_bytes": int(b_launch), "kernel_ms": round(ms_launch, 4),
                "launches_per_step": passes}
    ms_solve = dt * 1e3
    ws_one = im.workspace_bytes()
    out = {
        "metric": "RRR sets/s through IMM with GreediRIS selection (bit-exact)",
        "value": round(samples / dt, 1), "unit": "RRR sets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_solve, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "graph": "R-MAT (0.57,0.19,0.19) scale 22, %d edges"
                   % G.num_edges, "model": "LT, uniform weights normalised per vertex",
                   "k": w.k, "eps": w.eps, "selector": "GreediRIS", "m": w.m,
                   "delta": w.delta, "alpha": args.alpha},
        "theta": res["theta"], "martingale_samples": res["martingale_samples"],
        "rounds": res["rounds"], "coverage": res["coverage"], "bucket": res["bucket"],
        "streamed_solution_chosen": res["global_won"], "final_sum_rrr": res["final_total"],
        "seeds_head": res["seeds"][:8],
        "solves_in_flight": n_conc,
        "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
        "ms_per_step_one_stream": round(dt1s * 1e3, 3),
        "value_one_stream": round(samples / dt1s, 1),
        "sampling_sets_per_s": round(res["sampled_sets"] /
                                     ((mean("ms_sample_main") + mean("ms_sample_large") +
                                       mean("ms_sample_gather")) * 1e-3), 1),
        "cover_ms": round(mean("ms_select"), 3),
        "breakdown_ms": {"sample_main_kernel": round(mean("ms_sample_main"), 3),
                         "sample_large_kernel": round(mean("ms_sample_large"), 3),
                         "sample_gather": round(mean("ms_sample_gather"), 3),
                         "select_all_rounds": round(mean("ms_select"), 3),
                         "select_incidence": round(mean("ms_incidence"), 3),
                         "select_local_greedy": round(mean("ms_local"), 3),
                         "select_stream_cover": round(mean("ms_global"), 3)},
        "counts": {"sampled_sets": res["sampled_sets"], "sampled_sum_rrr": res["sampled_total"],
                   "probes": res["sampled_examined"], "edges_taken": res["sampled_live"],
                   "sample_launches": res["sample_launches"], "sample_passes": passes},
        # the caller-owned device workspace one solve ran in (pools, staging,
        # covering subsets, cover state), as the binding grew it
        "workspace_bytes": ws_one,
        "roofline": roofline,
    }
    if not args.no_extra:
        dt1, outs1 = solve_steps(im, G, w, 1.0, args.steps, 1, torch)
        r1 = outs1[0]
        out["alpha_1"] = {"ms_per_step": round(dt1 * 1e3, 3),
                          "value": round((r1["theta"] + r1["martingale_samples"]) / dt1, 1),
                          "coverage": r1["coverage"], "bucket": r1["bucket"],
                          "streamed_solution_chosen": r1["global_won"],
                          "cover_ms": round(sum(o["ms_select"] for o in outs1) / len(outs1), 3),
                          "seeds_head": r1["seeds"][:8]}
        log("alpha 1: %.3f ms per solve (one stream)" % (dt1 * 1e3))
        dt2, outs2 = solve_steps(im, G, w, 1.0, args.steps, 1, torch,
                                 selector=im.SEL_RANDGREEDI)
        log("RandGreedi offline: %.3f ms per solve" % (dt2 * 1e3))

        def split(os_, dt):
            mk = lambda key: round(sum(o[key] for o in os_) / len(os_), 3)  # noqa: E731
            return {"ms_per_solve": round(dt * 1e3, 3), "local_ms": mk("ms_local"),
                    "global_ms": mk("ms_global"), "coverage": os_[0]["coverage"],
                    "global_solution_chosen": os_[0]["global_won"]}
        # the paper's Table 2 contrast: the local step (partition + local
        # greedy over m parts) against the global step (streamed buckets, or
        # the offline aggregation), summed over the solve's three selections
        out["local_vs_global"] = {"greediris_alpha_0.125": split(outs, dt1s),
                                  "greediris_alpha_1": split(outs1, dt1),
                                  "randgreedi_offline": split(outs2, dt2)}
        out["local_vs_global"]["randgreedi_offline"]["global_cover"] = outs2[0]["global_cover"]
        w2 = W.config(2)
        g2 = w2.graph
        G2 = im.prepare_graph(g2.in_off, g2.in_src, g2.weight, g2.model)
        torch.cuda.synchronize()
        o2 = run_plain(args, w2, G2, im, torch, steps=20, warmup=5)
        out["rmat20_ic_wc"] = {k: o2[k] for k in ("value", "unit", "ms_per_step",
                                                  "ms_per_step_one_stream", "streams",
                                                  "sampling_sets_per_s", "cover_ms",
                                                  "breakdown_ms", "roofline")}
        out["rmat20_ic_wc"]["config"] = o2["config"]
        out["rmat20_ic_wc"]["coverage"] = o2["counts"]["coverage"]
        del G2, w2, g2
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        import oracle as O
        g = w.graph
        thr = O.thresholds(g.model, g.in_off, g.weight)
        log("cpu baseline: the oracle's whole IMM + GreediRIS solve")
        t1 = time.perf_counter()
        ores = O.imm(g.model, g.in_off, g.in_src, thr, w.k, w.eps, seed=w.seed,
                     selector=O.SEL_GREEDIRIS, m=w.m, delta=w.delta, alpha=args.alpha,
                     part_seed=w.part_seed, lazy=True)
        d1 = time.perf_counter() - t1
        same = (ores["seeds"].tolist() == res["seeds"] and ores["theta"] == res["theta"] and
                ores["coverage"] == res["coverage"])
        out["cpu_baseline"] = {
            "value": round((ores["theta"] + ores["martingale_samples"]) / d1, 1),
            "unit": "RRR sets/s", "cores": 1, "kind": "oracle",
            "sample": "the whole solve of this workload (IMM rounds, %d + %d samples, local "
                      "lazy greedy over %d partitions, streaming cover, final choice); %.1f s; "
                      "same seeds, theta and coverage as the GPU: %s"
                      % (ores["martingale_samples"], ores["theta"], w.m, d1, same)}
        assert same, "the oracle's solve differs from the GPU's"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
