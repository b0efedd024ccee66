"""GPU parity of the batched path: many independent factorisations and
solves in one graph.

Each matrix is checked against the oracle (backward error <= 1e-13 and the
solution within 16 n u cond(A) of the oracle's); a matrix gives bit-identical
results alone and inside the batch; a non-SPD matrix in the batch reports its
own breakdown column and leaves the others bit-identical.
"""
import numpy as np
import pytest

from oracle import core
from paper_1304_0878_amd import inputs

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


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


@pytest.fixture()
def rt(dc, torch_dev):
    r = dc.Runtime(device=0)
    yield r
    r.close()


def _batch(count, seed, nmax=300):
    ns, rs = inputs.batch_shapes(count, seed, nmin=16, nmax=nmax)
    mats = [inputs.spd_uniform(n, seed * 100000 + i) for i, n in enumerate(ns)]
    rhs = [inputs.rhs(n, r, seed * 100000 + 50000 + i) for i, (n, r) in enumerate(zip(ns, rs))]
    return ns, mats, rhs


def _tile_rule(n):
    return 0 if n <= 128 else 128


def _run(dc, rt, torch_dev, mats, rhs, tiles):
    torch, dev = torch_dev
    ta = [torch.from_numpy(m).to(dev) for m in mats]
    tb = [torch.from_numpy(b).to(dev) for b in rhs]
    infos = dc.potrf_batched(rt, ta, tb, tiles)
    return infos, [np.tril(t.cpu().numpy()) for t in ta], [t.cpu().numpy() for t in tb]


def test_batched_matches_oracle(dc, rt, torch_dev):
    ns, mats, rhs = _batch(120, 1)
    tiles = [_tile_rule(n) for n in ns]
    infos, ls, xs = _run(dc, rt, torch_dev, mats, rhs, tiles)
    assert infos == [0] * len(ns)
    for a, b, l, x, t in zip(mats, rhs, ls, xs, tiles):
        n = a.shape[0]
        assert core.backward_error_fro(a, l) <= 1e-13
        lr = np.tril(core.potrf_tiled(a, t or n)[0])
        xr = core.potrs_tiled(lr, b, t or n)
        assert np.abs(x - xr).max() / np.abs(xr).max() <= 16 * n * U * np.linalg.cond(a)


def test_batched_alone_equals_in_batch(dc, rt, torch_dev):
    ns, mats, rhs = _batch(40, 2)
    tiles = [_tile_rule(n) for n in ns]
    _, ls, xs = _run(dc, rt, torch_dev, mats, rhs, tiles)
    for i in (0, 7, 19, 39):
        _, l1, x1 = _run(dc, rt, torch_dev, [mats[i]], [rhs[i]], [tiles[i]])
        assert np.array_equal(l1[0], ls[i]) and np.array_equal(x1[0], xs[i])


def test_batched_failure_is_isolated(dc, rt, torch_dev):
    ns, mats, rhs = _batch(30, 3)
    tiles = [_tile_rule(n) for n in ns]
    _, ls, xs = _run(dc, rt, torch_dev, mats, rhs, tiles)
    bad = [m.copy() for m in mats]
    j = 11
    k = ns[j] // 2
    bad[j][k, k] = -1.0
    infos, ls2, xs2 = _run(dc, rt, torch_dev, bad, rhs, tiles)
    assert infos[j] == core.potrf_tiled(bad[j], tiles[j] or ns[j])[1] > 0
    for i in range(len(ns)):
        if i != j:
            assert infos[i] == 0
            assert np.array_equal(ls2[i], ls[i]) and np.array_equal(xs2[i], xs[i])


def test_batched_integer_exact(dc, rt, torch_dev):
    mats, rhs, sols = [], [], []
    for i, n in enumerate((20, 64, 130, 257)):
        a, l0 = inputs.integer_factor(n, 40 + i, diag_choices=(1.0, 2.0))
        x0 = inputs.integer_solution(n, 2, 60 + i)
        mats.append(a)
        rhs.append(a @ x0)
        sols.append((l0, x0))
    infos, ls, xs = _run(dc, rt, torch_dev, mats, rhs, [0, 32, 64, 128])
    assert infos == [0, 0, 0, 0]
    for (l0, x0), l, x in zip(sols, ls, xs):
        assert np.array_equal(l, l0) and np.array_equal(x, x0)


def test_batched_at_tuner_tiles_matches_oracle(dc, rt, torch_dev):
    """The configuration the benchmark times: orders drawn from [16, 512] and
    the tile sizes the committed autotuner cache picks for them (for every
    bucket up to 512 the whole matrix, so the solves run the substitution
    TRSM_L / TRSM_LT units on diagonal tiles of order up to 512)."""
    from paper_1304_0878_amd import tune
    cache = tune.load()
    assert cache is not None
    ns, mats, rhs = _batch(64, 5, nmax=512)
    tiles = tune.tiles_for(ns, cache)
    assert sum(1 for n, t in zip(ns, tiles) if (t or n) > 128) >= 20
    infos, ls, xs = _run(dc, rt, torch_dev, mats, rhs, tiles)
    assert infos == [0] * len(ns)
    for a, b, l, x, t in zip(mats, rhs, ls, xs, tiles):
        n = a.shape[0]
        assert core.backward_error_fro(a, l) <= 1e-13
        lr = np.tril(core.potrf_tiled(a, t or n)[0])
        xr = core.potrs_tiled(lr, b, t or n)
        assert np.abs(x - xr).max() / np.abs(xr).max() <= 16 * n * U * np.linalg.cond(a)


def test_batched_fp32_and_fp64_in_one_graph(dc, rt, torch_dev):
    """FP32 matrices (factored as one tile: FP64 arithmetic, the factor
    rounded to FP32) next to FP64 ones in one call.  FP32 bars: backward
    error of the stored factor ||A32 - L L^T||_F / ||A32||_F <= 4 n u32
    (u32 = 2^-24: one rounding per stored entry, amplified by the
    recurrence) and the solution (FP64 arithmetic on the FP32 factor) within
    8 n u32 cond(A) of the oracle's FP64 solution of the same matrix; the
    FP64 matrices as in the FP64-only batches, and bit-identical to their
    factor in an FP64-only batch."""
    torch, dev = torch_dev
    ns, mats, rhs = _batch(48, 6, nmax=512)
    is32 = [i % 2 == 0 for i in range(len(ns))]
    ta = [torch.from_numpy(m).to(dev).to(torch.float32) if f else torch.from_numpy(m).to(dev)
          for m, f in zip(mats, is32)]
    tb = [torch.from_numpy(b).to(dev) for b in rhs]
    infos = dc.potrf_batched(rt, ta, tb, [0] * len(ns))
    assert infos == [0] * len(ns)
    U32 = 2.0 ** -24
    for i, (n, a, b) in enumerate(zip(ns, mats, rhs)):
        l = np.tril(ta[i].cpu().numpy().astype(np.float64))
        x = tb[i].cpu().numpy()
        if is32[i]:
            a32 = a.astype(np.float32).astype(np.float64)
            assert core.backward_error_fro(a32, l) <= 4 * n * U32
            assert np.array_equal(l, l.astype(np.float32).astype(np.float64))
            lr = np.tril(core.potrf_tiled(a32, n)[0])
            xr = core.potrs_tiled(lr, b, n)
            cond = np.linalg.cond(a32)
            assert np.abs(x - xr).max() / np.abs(xr).max() <= 8 * n * U32 * cond
        else:
            assert core.backward_error_fro(a, l) <= 1e-13
    # the FP64 matrices are unchanged by their FP32 neighbours
    idx = [i for i in range(len(ns)) if not is32[i]]
    _, l64, x64 = _run(dc, rt, torch_dev, [mats[i] for i in idx], [rhs[i] for i in idx],
                       [0] * len(idx))
    for k, i in enumerate(idx):
        assert np.array_equal(np.tril(ta[i].cpu().numpy()), l64[k])


def test_batched_fp32_integer_exact(dc, rt, torch_dev):
    """Integer factors with entries and partial sums exact in FP32: the FP32
    factor is L0 bit for bit and the solution the integer one."""
    torch, dev = torch_dev
    mats, rhs, sols = [], [], []
    for i, n in enumerate((24, 100, 300)):
        a, l0 = inputs.integer_factor(n, 70 + i, diag_choices=(1.0, 2.0))
        x0 = inputs.integer_solution(n, 2, 80 + i)
        mats.append(torch.from_numpy(a).to(dev).to(torch.float32))
        rhs.append(torch.from_numpy(a @ x0).to(dev))
        sols.append((l0, x0))
    assert dc.potrf_batched(rt, mats, rhs, [0, 0, 0]) == [0, 0, 0]
    for (l0, x0), m, b in zip(sols, mats, rhs):
        assert np.array_equal(np.tril(m.cpu().numpy().astype(np.float64)), l0)
        assert np.array_equal(b.cpu().numpy(), x0)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_whole_tile_large_orders(dc, torch_dev, dt):
    """Orders above 256 factored as one tile in a graph without GEMM units
    (the left-looking POTRF's instance of its own), next to smaller ones:
    each factor meets the oracle's bars, a matrix gives the same bits alone
    and in the batch, and a non-SPD one reports the oracle's breakdown
    column and leaves the others bit-identical.  The runtime is capped at
    one CU: an FP64 POTRF is then never its level's long pole, so none is
    split into sub-block tasks (as in a batch of thousands of matrices)."""
    torch, dev = torch_dev
    rt = dc.Runtime(device=0, workers=1)
    try:
        _whole_tile_large_orders(dc, rt, torch, dev, dt)
    finally:
        rt.close()


def _whole_tile_large_orders(dc, rt, torch, dev, dt):
    ns = [260, 100, 300, 384, 200, 450, 512, 257]
    mats = [inputs.spd_uniform(n, 9100 + i) for i, n in enumerate(ns)]
    rhs = [inputs.rhs(n, 2, 9200 + i) for i, n in enumerate(ns)]
    tt = torch.float64 if dt == "f64" else torch.float32

    def run(ms):
        ta = [torch.from_numpy(m).to(dev).to(tt) for m in ms]
        tb = [torch.from_numpy(b).to(dev) for b in rhs[:len(ms)]]
        infos = dc.potrf_batched(rt, ta, tb, [0] * len(ms))
        return (infos, [np.tril(t.cpu().numpy().astype(np.float64)) for t in ta],
                [t.cpu().numpy() for t in tb])

    infos, ls, xs = run(mats)
    assert infos == [0] * len(ns)
    U32 = 2.0 ** -24
    for n, a, b, l, x in zip(ns, mats, rhs, ls, xs):
        if dt == "f64":
            assert core.backward_error_fro(a, l) <= 1e-13
            ar, bound = a, 16 * n * U
        else:
            ar = a.astype(np.float32).astype(np.float64)
            assert core.backward_error_fro(ar, l) <= 4 * n * U32
            bound = 8 * n * U32
        lr = np.tril(core.potrf_tiled(ar, n)[0])
        xr = core.potrs_tiled(lr, b, n)
        assert np.abs(x - xr).max() / np.abs(xr).max() <= bound * np.linalg.cond(ar)
    for i in (2, 6):
        ta = [torch.from_numpy(mats[i]).to(dev).to(tt)]
        tb = [torch.from_numpy(rhs[i]).to(dev)]
        assert dc.potrf_batched(rt, ta, tb, [0]) == [0]
        assert np.array_equal(np.tril(ta[0].cpu().numpy().astype(np.float64)), ls[i])
        assert np.array_equal(tb[0].cpu().numpy(), xs[i])
    bad = [m.copy() for m in mats]
    j, k = 3, 200
    bad[j][k, k] = -1.0
    infos2, ls2, xs2 = run(bad)
    ref = bad[j] if dt == "f64" else bad[j].astype(np.float32).astype(np.float64)
    assert infos2[j] == core.potrf_tiled(ref, ns[j])[1] == k + 1
    for i in range(len(ns)):
        if i != j:
            assert infos2[i] == 0
            assert np.array_equal(ls2[i], ls[i]) and np.array_equal(xs2[i], xs[i])
