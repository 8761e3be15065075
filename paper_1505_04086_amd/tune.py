"""Autotuner for the launch options of librsoc.

The tunable options (rsoc_options) are the degree-bin thresholds (t_thread:
largest row coloured by an 8-lane group; t_wave: largest row coloured by one
wavefront), the workgroups given to the thread and wavefront bins, the run
length of consecutive ids a lane group walks (chunk), the workgroups of the
thread bin in worklist rounds (grid_list), the round-0 lookahead
and the number of worklist rounds captured per host check.  The tuner runs
coordinate descent over them: each option in turn is set to each candidate
value while the others keep their best values so far, timed with the real
entry point on a sample of the workload, and kept when it is faster.
Correctness never depends on these options (the tests run every mode under
several of them), so the search only measures time.

Results are cached in a JSON file (RSOC_TUNE_FILE, default
~/.cache/rsoc/tune.json) keyed by device architecture and a graph-class
signature (log2 of the max degree, rounded mean degree, whether ids carry
locality).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

import paper_1505_04086_amd as rsoc

torch = rsoc.torch

SPACE = {
    "t_thread": [8, 16, 24, 32],
    "t_wave": [256, 1024, 2048, 8192],
    "grid_thread": [512, 1024, 2048, 4096],
    "grid_wave": [512, 1024, 2048],
    "grid_list": [1024, 2048, 4096, 8192],
    "chunk": [1, 2, 4, 8],
    "lookahead": [-1, 1 << 18, 1 << 20, 1 << 22],
    "rounds_per_sync": [4, 8, 16],
    "small_cutoff": [-1, 256, 1024, 2048],
}


def tune_file() -> str:
    return os.environ.get("RSOC_TUNE_FILE", os.path.join(os.path.expanduser("~"), ".cache", "rsoc", "tune.json"))


def signature(row_ptr, col_idx, sample: int = 4096, seed: int = 0) -> str:
    """Graph-class key from a host CSR: max degree (log2), mean degree, id locality."""
    rp = np.asarray(row_ptr)
    ci = np.asarray(col_idx)
    n = len(rp) - 1
    deg = np.diff(rp)
    if n == 0:
        return "empty"
    rng = np.random.default_rng(seed)
    vs = rng.integers(0, n, size=min(sample, n))
    near = tot = 0
    for v in vs:
        row = ci[rp[v]:rp[v + 1]]
        near += int(np.count_nonzero(np.abs(row - v) < 8))
        tot += len(row)
    local = tot > 0 and near * 50 >= tot
    return "dmax%d-dmean%d-%s" % (int(math.log2(max(int(deg.max()), 1))), int(round(float(deg.mean()))),
                                  "local" if local else "scrambled")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache() -> dict:
    p = tune_file()
    if not os.path.exists(p):
        return {}
    try:
        return json.load(open(p))
    except Exception:
        return {}


def save(key: str, options: dict, ms: float):
    p = tune_file()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    cache = load_cache()
    cache["%s/%s" % (_arch(), key)] = {"options": options, "ms": ms, "time": time.time()}
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(key: str):
    ent = load_cache().get("%s/%s" % (_arch(), key))
    return None if ent is None else dict(ent["options"])


def coordinate_descent(measure, space=None, start=None, sweeps: int = 2, min_gain: float = 0.02, log=None):
    """Minimise measure(options_dict) -> seconds over `space`, one option at a time."""
    space = SPACE if space is None else space
    best = dict(start or {})
    best_t = measure(best)
    trials = [(dict(best), best_t)]
    for _ in range(sweeps):
        improved = False
        for name, values in space.items():
            for v in values:
                if best.get(name) == v:
                    continue
                cand = dict(best)
                cand[name] = v
                t = measure(cand)
                trials.append((dict(cand), t))
                if log:
                    log("tune %s=%s: %.3f ms (best %.3f)" % (name, v, t * 1e3, best_t * 1e3))
                if t < best_t * (1 - min_gain):
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    return best, best_t, trials


def _timer(fn, reps: int):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune_single(ctx, d_rp, d_ci, n, d_col, mode="optimistic", reps=3, space=None, sweeps=2, log=None):
    """Tune rsoc_color_device on one device-resident graph."""
    def measure(opts):
        o = rsoc.make_options(mode, **opts)
        return _timer(lambda: rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o), reps)
    return coordinate_descent(measure, space=space, sweeps=sweeps, log=log)


def tune_batch(ctx, vtx_off, nnz_off, d_rp, d_ci, d_col, mode="optimistic", reps=3, space=None, sweeps=2, log=None):
    """Tune rsoc_color_batch on a device-resident batch."""
    def measure(opts):
        o = rsoc.make_options(mode, **opts)
        return _timer(lambda: rsoc.rsoc_color_batch(ctx, vtx_off, nnz_off, d_rp, d_ci, d_col, o), reps)
    return coordinate_descent(measure, space=space, sweeps=sweeps, log=log)
