"""Executors on the GPU.

* The level executor's per-task trace respects every dependency edge (a
  task starts after all its predecessors ended), and the CU cap changes no
  bit of the result.
* dc_acquire after dc_flush waits for the flushed graph.
* The ready-queue executor is disabled on device runtimes (-ENOSYS): its
  first GPU run did not complete, and its tests (bitwise agreement with the
  level executor, the watchdog) are skipped until the cause is known.  Its
  protocol is tested on the CPU (tests/test_queue_model.py).
"""
import struct

import numpy as np
import pytest

from oracle import core
from paper_1304_0878_amd import inputs

pytestmark = pytest.mark.gpu
QUEUE_OFF = ("the ready-queue executor is disabled: its first GPU run (this test, "
             "n=1536, tile 256) was still inside dc_potrf after 120 s with no cause shown")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def dc():
    from paper_1304_0878_amd import dagchol
    return dagchol


def _gpu(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _both(dc, torch_dev, fn, **kw):
    out = []
    for ex in (dc.DC_EXEC_QUEUE, dc.DC_EXEC_LEVELS):
        with dc.Runtime(device=0, executor=ex, **kw) as rt:
            out.append(fn(rt))
        torch_dev[0].cuda.synchronize()
    return out


@pytest.mark.skip(reason=QUEUE_OFF)
@pytest.mark.parametrize("n,tile", [(1536, 256), (1000, 128), (700, 512), (64, 16)])
def test_factor_and_solve_bitwise_across_executors(dc, torch_dev, n, tile):
    a = inputs.spd_normal(n, 3, 1e-2)
    b = inputs.rhs(n, 3, 4)

    def run(rt):
        ta, tb = _gpu(torch_dev, a), _gpu(torch_dev, b)
        assert dc.potrf(rt, ta, tile) == 0
        dc.potrs(rt, ta, tb, tile)
        return np.tril(ta.cpu().numpy()), tb.cpu().numpy()

    (lq, xq), (ll, xl) = _both(dc, torch_dev, run)
    assert np.array_equal(lq, ll)
    assert np.array_equal(xq, xl)
    lr, info = core.potrf_tiled(a, tile)
    assert info == 0
    assert np.abs(lq - np.tril(lr)).max() <= 1e-12 * np.abs(lr).max()


@pytest.mark.skip(reason=QUEUE_OFF)
@pytest.mark.parametrize("upd", ["f32", "bf16"])
def test_mixed_refinement_bitwise_across_executors(dc, torch_dev, upd):
    n, tile = 1024, 256
    a = inputs.spd_cond(n, 5, 1e4)
    b = inputs.rhs(n, 5, 2)
    u = dc.DC_F32 if upd == "f32" else dc.DC_BF16

    def run(rt):
        ta, tb = _gpu(torch_dev, a), _gpu(torch_dev, b)
        tx = torch_dev[0].zeros_like(tb)
        rep = dc.posv_ir(rt, ta, tb, tx, tile, upd=u)
        return tx.cpu().numpy(), (rep["iterations"], rep["converged"], rep["final_prec"])

    (xq, rq), (xl, rl) = _both(dc, torch_dev, run)
    assert rq == rl and rq[1] == 1
    assert np.array_equal(xq, xl)


@pytest.mark.skip(reason=QUEUE_OFF)
def test_batched_bitwise_across_executors(dc, torch_dev):
    ns, rs = inputs.batch_shapes(40, 11, nmin=16, nmax=300)
    mats = [inputs.spd_uniform(n, 100 + i) for i, n in enumerate(ns)]
    rhs = [inputs.rhs(n, 200 + i, r) for i, (n, r) in enumerate(zip(ns, rs))]
    tiles = [0 if n <= 128 else 128 for n in ns]

    def run(rt):
        ta = [_gpu(torch_dev, m) for m in mats]
        tb = [_gpu(torch_dev, v) for v in rhs]
        info = dc.potrf_batched(rt, ta, tb, tiles)
        assert info == [0] * len(ns)
        return [np.tril(t.cpu().numpy()) for t in ta] + [t.cpu().numpy() for t in tb]

    q, lv = _both(dc, torch_dev, run)
    for x, y in zip(q, lv):
        assert np.array_equal(x, y)


def test_queue_executor_is_rejected(dc, torch_dev):
    with pytest.raises(dc.DagcholError) as e:
        dc.Runtime(device=0, executor=dc.DC_EXEC_QUEUE)
    assert e.value.code == -38


def test_worker_cap_and_small_graphs(dc, torch_dev):
    """A CU cap (down to one CU for each kernel) changes no bit of the
    factor; one-task graphs at the smallest sizes."""
    n, tile = 640, 128
    a = inputs.spd_uniform(n, 9)
    ref = None
    for workers in (0, 1, 2, 3, 17):
        with dc.Runtime(device=0, workers=workers) as rt:
            ta = _gpu(torch_dev, a)
            assert dc.potrf(rt, ta, tile) == 0
            got = np.tril(ta.cpu().numpy())
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), workers
    with dc.Runtime(device=0) as rt:
        for n1 in (1, 2, 16):
            a1 = inputs.spd_uniform(n1, n1)
            ta = _gpu(torch_dev, a1)
            assert dc.potrf(rt, ta, 16) == 0
            lr, _ = core.potrf_tiled(a1, 16)
            assert np.abs(np.tril(ta.cpu().numpy()) - np.tril(lr)).max() <= 1e-13 * n1


def _submit_factor(dc, rt, tiles, W):
    """The tiled factor with inverse-based panel solves, through dc_task_submit."""
    R, RW, Wm = dc.DC_R, dc.DC_RW, dc.DC_W
    T = len(tiles)
    kinds = []

    def sub(kind, bufs, modes, prio=0):
        rt.dc_task_submit(kind, bufs, modes, priority=prio)
        kinds.append(kind)
    for k in range(T):
        sub(dc.DC_POTRF, [tiles[k][k]], [RW])
        if k + 1 < T:
            sub(dc.DC_TRSM, [tiles[k][k], tiles[k + 1][k]], [R, RW])
            if k + 2 < T:
                sub(dc.DC_TRTRI, [tiles[k][k], W[k]], [R, Wm])
                for i in range(k + 2, T):
                    sub(dc.DC_TRSM_INV, [tiles[k][k], W[k], tiles[i][k]], [R, R, RW], 1)
        for i in range(k + 1, T):
            sub(dc.DC_SYRK, [tiles[i][k], tiles[i][i]], [R, RW], 0 if i == k + 1 else 2)
            for j in range(k + 1, i):
                sub(dc.DC_GEMM, [tiles[i][k], tiles[j][k], tiles[i][j]], [R, R, RW],
                    1 if j == k + 1 else 2)
    return kinds


def test_trace_respects_dependencies(dc, torch_dev):
    torch, dev = torch_dev
    n, tile = 4096, 512
    T = n // tile
    a = inputs.spd_normal(n, 1, 1e-2)
    ta = _gpu(torch_dev, a)
    tw = torch.zeros((T * tile, tile), dtype=torch.float64, device=dev)
    with dc.Runtime(device=0, trace=True) as rt:
        ha = rt.register_tensor(ta)
        hw = rt.register_tensor(tw)
        tiles = rt.dc_matrix_partition(ha, tile)
        W = [row[0] for row in rt.dc_matrix_partition(hw, tile)]
        kinds = _submit_factor(dc, rt, tiles, W)
        preds = [rt.dc_graph_preds(t) for t in range(len(kinds))]
        rt.dc_wait_all()
        tr = [rt.dc_trace_get(t) for t in range(len(kinds))]
        rt.dc_matrix_unpartition(hw)
        rt.dc_matrix_unpartition(ha)
        rt.dc_unregister(hw)
        rt.dc_unregister(ha)
    for t, (s, e, w, k) in enumerate(tr):
        assert k == kinds[t] and w >= 0 and e >= s
        for p in preds[t]:
            assert s >= tr[p][1] - 1000, (t, p, s, tr[p][1])
    # lookahead: the POTRF of step k + 1 starts before the last update of
    # step k ended, for some k
    step = []
    k = -1
    for t, kind in enumerate(kinds):
        if kind == dc.DC_POTRF:
            k += 1
        step.append(k)
    overlap = 0
    for k in range(T - 2):
        potrf_next = next(t for t in range(len(kinds))
                          if kinds[t] == dc.DC_POTRF and step[t] == k + 1)
        last_upd = max(tr[t][1] for t in range(len(kinds))
                       if step[t] == k and kinds[t] == dc.DC_GEMM)
        overlap += tr[potrf_next][0] < last_upd
    print(f"steps whose next diagonal factor started before their last update ended: "
          f"{overlap} of {T - 2}")
    l = np.tril(ta.cpu().numpy())
    assert core.backward_error_fro(a, l) <= 1e-13


@pytest.mark.skip(reason=QUEUE_OFF)
def test_watchdog_returns_etimedout_and_runtime_recovers(dc, torch_dev):
    torch, dev = torch_dev
    n, tile = 4096, 512
    a = inputs.spd_normal(n, 2, 1e-2)
    ta = _gpu(torch_dev, a)
    with dc.Runtime(device=0, watchdog_ms=1, trace=True) as rt:
        h = rt.register_tensor(ta)
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_potrf(h, tile)
        assert e.value.code == -110
        # a graph that needs no wait still runs on the same runtime
        x = torch.arange(1000, dtype=torch.float32, device=dev)
        hx = rt.register_tensor(x)
        rt.dc_task_submit(dc.DC_SCAL, [hx], [dc.DC_RW], cl_args=struct.pack("f", 2.0))
        rt.dc_wait_all()
        assert torch.equal(x.cpu(), 2 * torch.arange(1000, dtype=torch.float32))
        rt.dc_unregister(hx)
        rt.dc_unregister(h)
    with dc.Runtime(device=0) as rt:
        tb = _gpu(torch_dev, a)
        assert dc.potrf(rt, tb, tile) == 0
        assert core.backward_error_fro(a, np.tril(tb.cpu().numpy())) <= 1e-13


def test_acquire_after_flush_waits_for_the_graph(dc, torch_dev):
    torch, dev = torch_dev
    own = torch.cuda.Stream()
    x0 = torch.arange(1 << 24, dtype=torch.float32, device=dev) % 1000
    x = x0.clone()
    torch.cuda.synchronize()
    with dc.Runtime(device=0, stream=own) as rt:
        h = rt.register_tensor(x)
        for f in [2.0] * 12 + [0.5] * 11:
            rt.dc_task_submit(dc.DC_SCAL, [h], [dc.DC_RW], cl_args=struct.pack("f", f))
        rt.dc_flush()
        rt.dc_acquire(h, dc.DC_R)
        # read on torch's own stream, which the runtime's stream does not order
        got = x.cpu()
        rt.dc_release(h)
        rt.dc_unregister(h)
    assert torch.equal(got, (2 * x0).cpu())
