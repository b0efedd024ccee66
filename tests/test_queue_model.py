"""The ready-queue executor's protocol (csrc/queue.h) run by host threads
under ThreadSanitizer: the same pop / complete code the device kernels run,
over the graphs the runtime infers from access modes (the tiled factor with
and without the inverse-based panel solves, the solve with its
write-after-read edges, a one-task graph, a random graph), with several
workers per class.  Each item's body checks with plain loads that every
item of every predecessor has run; a missing ordering edge is a data race
the sanitizer reports.  A task whose dependency count never reaches zero
must end the run through the watchdog with every worker gone."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "queue_model", "queue_model.cpp")
CSRC = os.path.join(ROOT, "paper_1304_0878_amd", "csrc")
FAKE = 0x10000

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("qm") / "queue_model")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                    "-I", CSRC, SRC, "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def dc():
    from paper_1304_0878_amd import dagchol
    return dagchol


def _classes(dc):
    gemm = {dc.DC_GEMM, dc.DC_SYRK}
    return lambda kind: (1, 1) if kind in gemm else (0, 0)   # (class, paired)


def _graph(dc, submit):
    """Submits through a host-only runtime and returns [(kind, prio, preds)]."""
    out = []
    with dc.Runtime(device=-1) as rt:
        log = []
        orig = rt.dc_task_submit

        def rec(kind, bufs, modes, cl_args=None, priority=0):
            orig(kind, bufs, modes, cl_args, priority)
            log.append((kind, priority))
        rt.dc_task_submit = rec
        submit(rt)
        for t, (kind, prio) in enumerate(log):
            out.append((kind, prio, rt.dc_graph_preds(t)))
    return out


def _cholesky(dc, T, tile=64, inverse=False, solve=False):
    n = T * tile

    def submit(rt):
        a = rt.dc_matrix_register(FAKE, n, n, n, dc.DC_F64)
        t = rt.dc_matrix_partition(a, tile)
        w = None
        if inverse:
            wh = rt.dc_matrix_register(FAKE + (1 << 32), T * tile, tile, tile, dc.DC_F64)
            w = [row[0] for row in rt.dc_matrix_partition(wh, tile)]
        R, RW, W = dc.DC_R, dc.DC_RW, dc.DC_W
        for k in range(T):
            rt.dc_task_submit(dc.DC_POTRF, [t[k][k]], [RW])
            if inverse and k + 1 < T:
                rt.dc_task_submit(dc.DC_TRSM, [t[k][k], t[k + 1][k]], [R, RW])
                if k + 2 < T:
                    rt.dc_task_submit(dc.DC_TRTRI, [t[k][k], w[k]], [R, W])
                    for i in range(k + 2, T):
                        rt.dc_task_submit(dc.DC_TRSM_INV, [t[k][k], w[k], t[i][k]], [R, R, RW],
                                          priority=1)
            else:
                for i in range(k + 1, T):
                    rt.dc_task_submit(dc.DC_TRSM, [t[k][k], t[i][k]], [R, RW],
                                      priority=0 if i == k + 1 else 1)
            for i in range(k + 1, T):
                rt.dc_task_submit(dc.DC_SYRK, [t[i][k], t[i][i]], [R, RW],
                                  priority=0 if i == k + 1 else 2)
                for j in range(k + 1, i):
                    rt.dc_task_submit(dc.DC_GEMM, [t[i][k], t[j][k], t[i][j]], [R, R, RW],
                                      priority=1 if j == k + 1 else 2)
        if solve:
            b = rt.dc_matrix_register(FAKE + (1 << 34), n, 1, 1, dc.DC_F64)
            bt = [row[0] for row in rt.dc_matrix_partition(b, tile)]
            for k in range(T):
                rt.dc_task_submit(dc.DC_TRSM_L, [t[k][k], bt[k]], [R, RW])
                for i in range(k + 1, T):
                    rt.dc_task_submit(dc.DC_GEMM_RHS_N, [t[i][k], bt[k], bt[i]], [R, R, RW])
            for k in range(T - 1, -1, -1):
                rt.dc_task_submit(dc.DC_TRSM_LT, [t[k][k], bt[k]], [R, RW])
                for i in range(k - 1, -1, -1):
                    rt.dc_task_submit(dc.DC_GEMM_RHS_T, [t[k][i], bt[k], bt[i]], [R, R, RW])
    return _graph(dc, submit)


def _write(path, dc, graph, seed=0):
    rng = random.Random(seed)
    cls = _classes(dc)
    with open(path, "w") as f:
        f.write(f"{len(graph)}\n")
        for kind, prio, preds in graph:
            c, paired = cls(kind)
            items = rng.randint(1, 8)
            f.write(f"{c} {min(prio, 3)} {paired} {items} {len(preds)} "
                    + " ".join(map(str, preds)) + "\n")


def _run(model, path, workers, *extra, timeout=600):
    r = subprocess.run([model, path, str(workers), *map(str, extra)], capture_output=True,
                       text=True, timeout=timeout,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.parametrize("T,inverse,solve", [(1, False, False), (4, False, True),
                                             (8, True, False), (16, True, True),
                                             (40, True, False)])
def test_cholesky_graphs(model, dc, tmp_path, T, inverse, solve):
    g = _cholesky(dc, T, inverse=inverse, solve=solve)
    p = str(tmp_path / "g.txt")
    _write(p, dc, g, seed=T)
    out = _run(model, p, 4)
    assert out.startswith("ok tasks=%d" % len(g)), out


def test_single_task_each_class(model, tmp_path):
    for c in range(4):
        p = str(tmp_path / f"one{c}.txt")
        with open(p, "w") as f:
            f.write(f"1\n{c} 0 0 1 0\n")
        assert _run(model, p, 8).startswith("ok tasks=1")


def test_random_graph_staggered_workers(model, tmp_path):
    rng = random.Random(7)
    n = 600
    p = str(tmp_path / "rand.txt")
    with open(p, "w") as f:
        f.write(f"{n}\n")
        for t in range(n):
            preds = sorted(rng.sample(range(t), min(t, rng.randint(0, 4))))
            f.write(f"{rng.randint(0, 3)} {rng.randint(0, 3)} {rng.randint(0, 1)} "
                    f"{rng.randint(1, 5)} {len(preds)} " + " ".join(map(str, preds)) + "\n")
    assert _run(model, p, 3, -1, 300).startswith("ok tasks=%d" % n)


def test_workers_yield_cus_to_a_class_not_resident(model, dc, tmp_path):
    """Fewer CU tokens than workers, GEMM workers first: the panel workers
    can only start after idle GEMM workers give up their CU."""
    g = _cholesky(dc, 12, inverse=True)
    p = str(tmp_path / "yield.txt")
    _write(p, dc, g)
    out = _run(model, p, 6, -1, 0, 6)
    assert out.startswith("ok tasks=%d" % len(g)), out
    assert int(out.split("yielded=")[1]) >= 1, out


def test_watchdog_ends_a_stuck_graph(model, dc, tmp_path):
    g = _cholesky(dc, 8, inverse=True)
    p = str(tmp_path / "stuck.txt")
    _write(p, dc, g)
    out = _run(model, p, 4, len(g) // 2)
    assert out.startswith("ok watchdog"), out
