#!/usr/bin/env python3
"""Benchmark: device-DAG tiled Cholesky factorisation (FP64) on one MI355X.

Workload (default): one SPD matrix of order n = 32768, A = B B^T / n + delta I
with B iid N(0, 1) drawn on the device from a seeded generator and delta set
for a 2-norm condition number of about 1e2 (largest eigenvalue of B B^T / n
estimated by power iteration; its smallest is negligible for square B).
Tile 512.  A pristine copy of A stays in HBM and is copied back before every
step, outside the timed region.

Each step is one dc_potrf call (graph build, upload, all level launches,
wait), timed with HIP events on the stream the library launches on.  The
JSON line reports GFLOP/s from the LAPACK flop count n^3/3 + n^2/2 + n/6,
the roofline of the level kernel against the FP64 MFMA peak, and the CPU
oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak (published)
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak (published)
METRIC = "Cholesky GFLOP/s + % MFMA peak (FP64 vs mixed@1e-10); solves/s with p50/p99"


def flops_potrf(n):
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0


def make_spd(torch, n, seed, kappa, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    b = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    a = torch.matmul(b, b.T)
    del b
    a.div_(n)
    # symmetrise exactly: the lower triangle is mirrored
    a = torch.tril(a) + torch.tril(a, -1).T
    v = torch.randn(n, 1, dtype=torch.float64, device=dev, generator=g)
    lam = 0.0
    for _ in range(30):
        w = a @ v
        lam = float(torch.linalg.vector_norm(w) / torch.linalg.vector_norm(v))
        v = w / torch.linalg.vector_norm(w)
    delta = lam / (kappa - 1.0)
    a.diagonal().add_(delta)
    return a.contiguous(), lam, delta


def cpu_baseline(target_s):
    """The plain C oracle (tiled FP64 factor in submission order) on a
    bounded sample sized for about target_s seconds of host work."""
    import numpy as np
    from oracle import core
    from paper_1304_0878_amd import inputs
    n0 = 2048
    a = inputs.spd_normal(n0, 1, 1e-2)
    t = time.perf_counter()
    core.potrf_tiled(a, 256)
    rate = flops_potrf(n0) / (time.perf_counter() - t)
    n = int((3.0 * rate * target_s) ** (1.0 / 3.0)) // 256 * 256
    n = max(2048, min(n, 16384))
    a = inputs.spd_normal(n, 2, 1e-2)
    t = time.perf_counter()
    l, info = core.potrf_tiled(a, 256)
    dt = time.perf_counter() - t
    assert info == 0
    return {"value": round(flops_potrf(n) / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": core.num_threads(), "kind": "oracle",
            "sample": f"tiled FP64 factorisation (tile 256) of one SPD matrix n={n}, "
                      f"A = B B^T/n + 1e-2 I, B iid N(0,1); {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--tile", type=int, default=512)
    ap.add_argument("--kappa", type=float, default=1e2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the single-GPU path only: run it with --gpus 1 "
              "(the factorisation is not sharded over several GPUs in this build)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_0878_amd import dagchol

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, tile = args.n, args.tile
    with torch.cuda.stream(stream):
        a0, lam, delta = make_spd(torch, n, args.seed, args.kappa, dev)
        a = torch.empty_like(a0)
    torch.cuda.synchronize()
    rt = dagchol.Runtime(device=0, stream=stream)
    times = []
    builds = []
    for step in range(args.warmup + args.steps):
        with torch.cuda.stream(stream):
            a.copy_(a0)
        torch.cuda.synchronize()
        if step == args.warmup:
            rt.dc_kernel_timing(True)   # per-launch HIP events over the timed steps
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = dagchol.potrf(rt, a, tile)
        e1.record(stream)
        torch.cuda.synchronize()
        if info != 0:
            raise RuntimeError(f"factorisation broke down at column {info}")
        if step >= args.warmup:
            times.append(e0.elapsed_time(e1))
            builds.append(rt.dc_last_launch()["build_ms"])
    launch = rt.dc_last_launch()
    kst = rt.dc_kernel_stats_get()
    ms = sum(times) / len(times)
    gflops = flops_potrf(n) / (ms * 1e-3) / 1e9

    # sanity check of the last factor: ||(A - L L^T) Z|| / ||A Z|| with 4
    # probe vectors, in FP64 on the device
    with torch.cuda.stream(stream):
        g = torch.Generator(device=dev)
        g.manual_seed(123)
        z = torch.randn(n, 4, dtype=torch.float64, device=dev, generator=g)
        low = torch.tril(a)
        az = a0 @ z
        r = az - low @ (low.T @ z)
        eta = float(torch.linalg.matrix_norm(r) / torch.linalg.matrix_norm(az))
        del low
    torch.cuda.synchronize()
    rt.close()

    # roofline of the dominant kernel (GEMM/SYRK updates): its algorithmic
    # flops per launch over its average launch duration
    gk = kst["gemm"]
    achieved = gk["flops"] / (gk["ms"] * 1e-3) / 1e12
    pk = kst["panel"]
    out = {
        "metric": METRIC,
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"tiled Cholesky factorisation of one SPD matrix, n={n}, "
                               f"tile {tile}, FP64, A = B B^T/n + delta I (cond ~{args.kappa:g})",
                   "n": n, "tile": tile, "kappa_target": args.kappa,
                   "lambda_max_est": round(lam, 6), "delta": delta,
                   "levels_units_workers": [launch["units"], launch["workers"]],
                   "host_graph_build_ms": round(sum(builds) / len(builds), 3)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": None, "kernel": "dc_gemm_kernel",
                     "launches_per_step": gk["launches"] / args.steps,
                     "avg_launch_us": round(gk["ms"] / gk["launches"] * 1e3, 2),
                     "flops_per_launch": gk["flops"] / gk["launches"]},
        "pct_fp64_mfma_peak_whole_factor": round(100 * gflops / 1e3 / FP64_PEAK_TFLOPS, 2),
        "panel_kernel": {"kernel": "dc_level_kernel", "launches_per_step": pk["launches"] / args.steps,
                         "avg_launch_us": round(pk["ms"] / max(pk["launches"], 1) * 1e3, 2),
                         "ms_per_step": round(pk["ms"] / args.steps, 3),
                         "tflops": round(pk["flops"] / max(pk["ms"], 1e-9) * 1e-9, 3)},
        "check": {"backward_error_probe": eta},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
