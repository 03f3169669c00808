"""Launch-shape autotuner for the batched and served paths.

The library's launch shapes (workgroups per CU of the main IC sampling
launch, the large-set launch's shape, the greedy apply's grid, the
dense/sparse switch of the covering subsets) are knobs of the C ABI
(im_tune_set).  None of them changes a result, only the time.  tune() times a
caller's workload at each candidate of each knob in turn (coordinate descent:
one knob at a time, the others at their best so far), keeps the fastest,
and checks on the way that every setting returns the same result signature.
"""
from __future__ import annotations

import json
import time

from . import binding as B

# knob name -> (C ABI key, candidate values)
KNOBS = {
    "sample_blocks": (B.TUNE_SAMPLE_BLOCKS, (4, 5, 6, 8, 12)),
    "big_shape": (B.TUNE_BIG_SHAPE, (0, 1, 2)),
    "apply_blocks": (B.TUNE_APPLY_BLOCKS, (1, 2, 4)),
    "dense_ratio": (B.TUNE_DENSE_RATIO, (64, 256, 4096)),
}


def current() -> dict:
    """Values in effect for every knob."""
    return {name: B.tune_get(key) for name, (key, _) in KNOBS.items()}


def apply(settings: dict):
    for name, value in settings.items():
        B.tune_set(KNOBS[name][0], int(value))


def reset():
    """Every knob back to its default."""
    for key, _ in KNOBS.values():
        B.tune_set(key, -1)


def _measure(run, reps: int):
    run()  # warm: scratch growth and first-touch costs stay out of the timing
    best, sig = None, None
    for _ in range(reps):
        ms, sig = run()
        best = ms if best is None or ms < best else best
    return best, sig


def tune(run, knobs=None, reps: int = 2, min_gain: float = 0.02, log=None) -> dict:
    """run() -> (ms, signature): one pass of the workload, its time and a
    hashable summary of its results.  A setting replaces the current one only
    if it is faster by more than min_gain (a fraction), so timing noise keeps
    the defaults.  Returns {"settings", "ms", "default_ms", "trials",
    "seconds"} and leaves the chosen settings applied.  Raises AssertionError
    if a setting changes the signature."""
    t0 = time.time()
    names = list(knobs) if knobs is not None else list(KNOBS)
    best = current()
    best_ms, sig0 = _measure(run, reps)
    default_ms = best_ms
    trials = [{"settings": dict(best), "ms": best_ms}]
    for name in names:
        key, cands = KNOBS[name]
        keep = best[name]
        for v in cands:
            if v == keep:
                continue
            B.tune_set(key, v)
            ms, sig = _measure(run, reps)
            if sig != sig0:
                B.tune_set(key, keep)
                raise AssertionError("knob %s=%d changed the results" % (name, v))
            trial = dict(best)
            trial[name] = v
            trials.append({"settings": trial, "ms": ms})
            if log:
                log("autotune %s=%d: %.3f ms (best %.3f)" % (name, v, ms, best_ms))
            if ms < best_ms * (1.0 - min_gain):
                best_ms, best[name] = ms, v
        B.tune_set(key, best[name])
    return {"settings": best, "ms": best_ms, "default_ms": default_ms, "trials": trials,
            "seconds": round(time.time() - t0, 2)}


def save(result: dict, path: str):
    with open(path, "w") as f:
        json.dump(result, f, indent=1)


def load(path: str) -> dict:
    """Settings saved by save(); apply() them."""
    with open(path) as f:
        return json.load(f)["settings"]
