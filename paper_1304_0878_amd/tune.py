"""Autotuner for batched factorisations: per bucket of matrix orders, the tile
size that makes a mixed batch factor and solve fastest on this GPU.

The search is a plain measurement on one mixed batch (matrices of every
bucket together, as a batched call sees them): every bucket starts at one
task per matrix, then, bucket by bucket from the largest orders down, each
candidate tile is timed on the whole batch with the other buckets fixed,
and the fastest median is kept.  The buckets are coupled: a multi-tile
graph for some matrices adds levels that the whole batch waits through, so
a bucket timed alone can pick a tile that slows the mix.  Results are
cached in a JSON file keyed by the GPU architecture.  Candidate 0 means
"one task per matrix" (tile = the matrix order).
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
    out = {"arch": _arch(torch), "per_bucket": per_bucket, "method": "mixed batch, coordinate search",
           "buckets": []}
    g = np.random.default_rng(seed)
    ns, bucket_of = [], []
    for bi, (lo, hi) in enumerate(buckets):
        for v in g.integers(lo, hi + 1, per_bucket):
            ns.append(int(v))
            bucket_of.append(bi)
    mats = [torch.from_numpy(inputs.spd_uniform(n, seed + i)).to(dev) for i, n in enumerate(ns)]
    rhs = [torch.from_numpy(inputs.rhs(n, 1, seed + 7 + i)).to(dev) for i, n in enumerate(ns)]
    work = [m.clone() for m in mats]
    wrhs = [b.clone() for b in rhs]

    def run(choice):
        tiles = [choice[bucket_of[i]] for i in range(len(ns))]
        samples = []
        for rep in range(reps + 1):
            for w, m in zip(work, mats):
                w.copy_(m)
            for w, b in zip(wrhs, rhs):
                w.copy_(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            infos = dagchol.potrf_batched(rt, work, wrhs, tiles)
            torch.cuda.synchronize()
            if rep:
                samples.append(time.perf_counter() - t)
            assert not any(infos)
        return sorted(samples)[len(samples) // 2] * 1e3

    choice = [0] * len(buckets)
    timings = [dict() for _ in buckets]
    best_ms = run(choice)
    for bi in reversed(range(len(buckets))):
        lo, hi = buckets[bi]
        timings[bi]["0"] = best_ms
        for cand in candidates:
            if cand == 0 or cand >= hi:
                continue   # tiles >= the largest order are one task per matrix
            trial = list(choice)
            trial[bi] = cand
            ms = run(trial)
            timings[bi][str(cand)] = ms
            if ms < best_ms:
                best_ms, choice = ms, trial
    for bi, (lo, hi) in enumerate(buckets):
        out["buckets"].append({"lo": lo, "hi": hi, "tile": int(choice[bi]), "ms": timings[bi]})
    out["batch_ms"] = best_ms
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
