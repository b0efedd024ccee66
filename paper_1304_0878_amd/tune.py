"""Autotuner for batched factorisations: per bucket of matrix orders, the tile
size that factors and solves a batch fastest on this GPU.

The search is a plain measurement: for each bucket a batch of SPD matrices
with orders drawn uniformly inside the bucket is factored (and solved) with
every candidate tile size through dc_potrf_batched, and the fastest median
wins.  Results are cached in a JSON file keyed by the GPU architecture.
Candidate 0 means "one task per matrix" (tile = the matrix order).
"""
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")

BUCKETS = [(16, 64), (65, 128), (129, 192), (193, 256), (257, 384), (385, 512)]
CANDIDATES = [0, 64, 128, 256]


def _arch(torch):
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def tune(rt, per_bucket=192, reps=3, seed=7, candidates=CANDIDATES, buckets=BUCKETS):
    import numpy as np
    import torch
    from . import dagchol, inputs
    dev = torch.device("cuda:0")
    out = {"arch": _arch(torch), "per_bucket": per_bucket, "buckets": []}
    g = np.random.default_rng(seed)
    for lo, hi in buckets:
        ns = [int(v) for v in g.integers(lo, hi + 1, per_bucket)]
        mats = [torch.from_numpy(inputs.spd_uniform(n, seed + i)).to(dev) for i, n in enumerate(ns)]
        rhs = [torch.from_numpy(inputs.rhs(n, 1, seed + 7 + i)).to(dev) for i, n in enumerate(ns)]
        work = [m.clone() for m in mats]
        wrhs = [b.clone() for b in rhs]
        timings = {}
        for cand in candidates:
            if cand and cand >= hi:
                continue   # same as one task per matrix
            samples = []
            for rep in range(reps + 1):
                for w, m in zip(work, mats):
                    w.copy_(m)
                for w, b in zip(wrhs, rhs):
                    w.copy_(b)
                torch.cuda.synchronize()
                t = time.perf_counter()
                infos = dagchol.potrf_batched(rt, work, wrhs, [cand] * len(ns))
                torch.cuda.synchronize()
                if rep:
                    samples.append(time.perf_counter() - t)
                assert not any(infos)
            timings[str(cand)] = sorted(samples)[len(samples) // 2] * 1e3
        best = min(timings, key=timings.get)
        out["buckets"].append({"lo": lo, "hi": hi, "tile": int(best), "ms": timings})
    return out


def save(result, path=DEFAULT_CACHE):
    with open(path, "w") as f:
        json.dump(result, f, indent=1)


def load(path=DEFAULT_CACHE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def tiles_for(ns, cache):
    """Tile size per matrix order from a tuning result (0 = whole matrix)."""
    out = []
    for n in ns:
        tile = 0
        for b in cache["buckets"]:
            if b["lo"] <= n <= b["hi"]:
                tile = b["tile"]
                break
        else:
            tile = 128 if n > 512 else 0
        out.append(tile)
    return out
