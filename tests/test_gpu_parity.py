"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Inputs are seeded (paper_1304_0878_amd.inputs) and fed as the same bytes to
both sides.  Tolerances:
  * FP64 factor: backward error ||A - L L^T||_F / ||A||_F <= 1e-13 (the
    stated bound for the FP64 path) and a normwise difference to the oracle's
    factor within 8 n u cond(A) (first-order perturbation of two backward
    stable factors);
  * exact-integer inputs: bitwise equality (every partial sum is an integer
    below 2^53, square roots of perfect squares and divisions by powers of two
    are exact, so any summation order gives the same bits);
  * solve: relative difference to the oracle's solution within
    16 n u cond(A).
"""
import numpy as np
import pytest

from oracle import core
from bounds import assert_factor_elementwise
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


def _gpu(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _factor(dc, rt, torch_dev, a, tile):
    ta = _gpu(torch_dev, a)
    info = dc.potrf(rt, ta, tile)
    torch_dev[0].cuda.synchronize()
    return np.tril(ta.cpu().numpy()), info, ta


# ---------------------------------------------- the paper's worked example

def test_scale_vector_bitwise(dc, rt, torch_dev):
    torch, dev = torch_dev
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    tx = torch.from_numpy(x).to(dev)
    h = rt.register_tensor(tx)
    import struct
    rt.dc_task_submit(dc.DC_SCAL, [h], [dc.DC_RW], cl_args=struct.pack("f", 3.14))
    rt.dc_wait_all()
    rt.dc_unregister(h)
    assert np.array_equal(tx.cpu().numpy(), core.scale_vector(x, 3.14))


# ---------------------------------------------------------- single tasks

def _single(dc, rt, kind, arrays, modes, torch_dev):
    ts = [_gpu(torch_dev, a) for a in arrays]
    hs = [rt.register_tensor(t) for t in ts]
    rt.dc_task_submit(kind, hs, modes)
    rt.dc_wait_all()
    out = [t.cpu().numpy() for t in ts]
    for h in hs:
        rt.dc_unregister(h)
    return out


@pytest.mark.parametrize("m,n,k", [(128, 128, 128), (300, 200, 256), (7, 5, 3), (512, 512, 512)])
def test_gemm_task(dc, rt, torch_dev, m, n, k):
    g = np.random.default_rng(m + n + k)
    x, y, c = g.standard_normal((m, k)), g.standard_normal((n, k)), g.standard_normal((m, n))
    got = _single(dc, rt, dc.DC_GEMM, [x, y, c], [dc.DC_R, dc.DC_R, dc.DC_RW], torch_dev)[2]
    ref = core.gemm_tile(c, x, y)
    assert np.abs(got - ref).max() <= 4 * k * U * (np.abs(x) @ np.abs(y).T + np.abs(c)).max()


@pytest.mark.parametrize("m,k", [(128, 128), (300, 256), (5, 3), (512, 512)])
def test_syrk_task(dc, rt, torch_dev, m, k):
    g = np.random.default_rng(m + k)
    x, c = g.standard_normal((m, k)), g.standard_normal((m, m))
    got = _single(dc, rt, dc.DC_SYRK, [x, c], [dc.DC_R, dc.DC_RW], torch_dev)[1]
    ref = core.syrk_tile(c, x)
    lo, up = np.tril_indices(m), np.triu_indices(m, 1)
    assert np.abs(got[lo] - ref[lo]).max() <= 4 * k * U * (np.abs(x) @ np.abs(x).T + np.abs(c)).max()
    assert np.array_equal(got[up], c[up])


@pytest.mark.parametrize("m,nb", [(128, 128), (100, 37), (512, 512), (33, 256)])
def test_trsm_task(dc, rt, torch_dev, m, nb):
    g = np.random.default_rng(m + nb)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb))
    x = g.standard_normal((m, nb))
    got = _single(dc, rt, dc.DC_TRSM, [l, x], [dc.DC_R, dc.DC_RW], torch_dev)[1]
    ref = core.trsm_tile(l, x)
    assert np.abs(got - ref).max() <= 64 * nb * U * np.abs(ref).max() * np.linalg.cond(l)


def _amp(l):
    """max |L| * max |L^{-1}|: the error growth of a solve through the inverse."""
    l = np.tril(l)
    return np.abs(l).max() * np.abs(core.trtri_tile(l)).max()


@pytest.mark.parametrize("nb", [16, 37, 128, 512])
def test_trtri_task(dc, rt, torch_dev, nb):
    l = np.linalg.cholesky(inputs.spd_uniform(nb, 7 * nb))
    w0 = np.full((nb, nb), np.nan)
    got = _single(dc, rt, dc.DC_TRTRI, [l, w0], [dc.DC_R, dc.DC_W], torch_dev)[1]
    ref = core.trtri_tile(l)
    lo = np.tril_indices(nb)
    assert np.abs(got[lo] - ref[lo]).max() <= 64 * nb * U * np.abs(ref).max() * np.linalg.cond(l)
    # the strictly upper part holds the two kinds of slots and nothing else
    nb16 = (nb + 15) // 16
    wl = np.tril(got)
    for u in range(nb16):
        assert got[0, 1 + u] == np.abs(wl[:, 16 * u:16 * u + 16]).max()
    assert got[1, 2] == np.abs(np.tril(l)).max()
    up = np.triu(np.ones((nb, nb), bool), 1)
    up[0, 1:1 + nb16] = False
    up[1, 2] = False
    assert np.all(np.isnan(got[up]))


@pytest.mark.parametrize("m,nb,x32", [(128, 128, False), (100, 37, False), (512, 512, False),
                                      (33, 256, False), (77, 512, True), (16, 16, False)])
def test_trsm_inv_task(dc, rt, torch_dev, m, nb, x32):
    g = np.random.default_rng(m + nb)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb))
    assert _amp(l) <= 1024   # the inverse product path, not the fallback
    x = g.standard_normal((m, nb))
    if x32:
        x = x.astype(np.float32)
    torch, dev = torch_dev
    tl, tx = _gpu(torch_dev, l), _gpu(torch_dev, x)
    tw = torch.zeros((nb, nb), dtype=torch.float64, device=dev)
    hl, hw, hx = rt.register_tensor(tl), rt.register_tensor(tw), rt.register_tensor(tx)
    rt.dc_task_submit(dc.DC_TRTRI, [hl, hw], [dc.DC_R, dc.DC_W])
    rt.dc_task_submit(dc.DC_TRSM_INV, [hl, hw, hx], [dc.DC_R, dc.DC_R, dc.DC_RW])
    rt.dc_wait_all()
    for h in (hl, hw, hx):
        rt.dc_unregister(h)
    got = tx.cpu().numpy().astype(np.float64)
    ref = core.trsm_inv_tile(core.trtri_tile(l), x.astype(np.float64))
    tol = 64 * nb * U * np.abs(ref).max() * np.linalg.cond(l)
    if x32:
        tol += 2.0 ** -24 * np.abs(ref).max()
    assert np.abs(got - ref).max() <= tol
    # the same operation as the substitution (different rounding)
    sub = core.trsm_tile(l, x.astype(np.float64))
    assert np.abs(got - sub).max() <= tol + 64 * nb * U * np.abs(sub).max() * np.linalg.cond(l)


@pytest.mark.parametrize("m,nb", [(64, 64), (40, 100)])
def test_trsm_inv_falls_back_to_substitution(dc, rt, torch_dev, m, nb):
    # integer L with entries up to 3 and power-of-two diagonal: its inverse
    # grows like 4^nb, far past the limit, so TRSM_INV must solve by
    # substitution and give the TRSM task's bits
    _, l0 = inputs.integer_factor(nb, 11)
    assert _amp(l0) > 1024
    g = np.random.default_rng(m * nb)
    x = (g.integers(-3, 4, (m, nb)).astype(np.float64)) @ l0.T
    torch, dev = torch_dev
    tl, tx = _gpu(torch_dev, l0), _gpu(torch_dev, x)
    tw = torch.zeros((nb, nb), dtype=torch.float64, device=dev)
    hl, hw, hx = rt.register_tensor(tl), rt.register_tensor(tw), rt.register_tensor(tx)
    rt.dc_task_submit(dc.DC_TRTRI, [hl, hw], [dc.DC_R, dc.DC_W])
    rt.dc_task_submit(dc.DC_TRSM_INV, [hl, hw, hx], [dc.DC_R, dc.DC_R, dc.DC_RW])
    rt.dc_wait_all()
    for h in (hl, hw, hx):
        rt.dc_unregister(h)
    sub = _single(dc, rt, dc.DC_TRSM, [l0, x], [dc.DC_R, dc.DC_RW], torch_dev)[1]
    assert np.array_equal(tx.cpu().numpy(), sub)
    assert np.array_equal(sub, core.trsm_tile(l0, x))


def _with_inverse(dc, rt, torch_dev, l, b, kind):
    """TRTRI, then one out-of-place task of `kind` (L, W, S = b, D); returns D
    and checks that S was only read."""
    torch, dev = torch_dev
    nb = l.shape[0]
    tl, tb = _gpu(torch_dev, l), _gpu(torch_dev, b)
    tw = torch.zeros((nb, nb), dtype=torch.float64, device=dev)
    td = torch.full(b.shape, float("nan"), dtype=torch.float64, device=dev)
    hs = [rt.register_tensor(t) for t in (tl, tw, tb, td)]
    rt.dc_task_submit(dc.DC_TRTRI, hs[:2], [dc.DC_R, dc.DC_W])
    rt.dc_task_submit(kind, hs, [dc.DC_R, dc.DC_R, dc.DC_R, dc.DC_W])
    rt.dc_wait_all()
    for h in hs:
        rt.dc_unregister(h)
    assert np.array_equal(tb.cpu().numpy(), b)
    return td.cpu().numpy()


@pytest.mark.parametrize("nb,r", [(512, 1), (512, 16), (100, 3), (16, 1), (256, 20), (37, 40),
                                  (200, 70)])
def test_solve_steps_through_inverse(dc, rt, torch_dev, nb, r):
    l = np.linalg.cholesky(inputs.spd_uniform(nb, 2 * nb + r))
    assert _amp(l) <= 1024
    bm = np.random.default_rng(nb * r).standard_normal((nb, r))
    tol = 64 * nb * U * np.linalg.cond(l)
    got = _with_inverse(dc, rt, torch_dev, l, bm, dc.DC_TRSM_L_INV)
    ref = core.trsm_left_tile(l, bm)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    got = _with_inverse(dc, rt, torch_dev, l, bm, dc.DC_TRSM_LT_INV)
    ref = core.trsm_left_t_tile(l, bm)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_solve_steps_through_inverse_fall_back(dc, rt, torch_dev):
    nb, r = 96, 5
    _, l0 = inputs.integer_factor(nb, 12)
    assert _amp(l0) > 1024
    x = np.random.default_rng(3).integers(-3, 4, (nb, r)).astype(np.float64)
    got = _with_inverse(dc, rt, torch_dev, l0, l0 @ x, dc.DC_TRSM_L_INV)
    assert np.array_equal(got, x)
    got = _with_inverse(dc, rt, torch_dev, l0, l0.T @ x, dc.DC_TRSM_LT_INV)
    assert np.array_equal(got, x)


def test_trsm_inv_cast_writes_bf16_copy(dc, rt, torch_dev):
    import torch
    m, nb = 70, 256
    l = np.linalg.cholesky(inputs.spd_uniform(nb, 5))
    x = np.random.default_rng(9).standard_normal((m, nb)).astype(np.float32)
    _, dev = torch_dev
    tl, tx = _gpu(torch_dev, l), _gpu(torch_dev, x)
    tw = torch.zeros((nb, nb), dtype=torch.float64, device=dev)
    ts = torch.zeros((m, nb), dtype=torch.bfloat16, device=dev)
    hs = [rt.register_tensor(t) for t in (tl, tw, tx, ts)]
    rt.dc_task_submit(dc.DC_TRTRI, hs[:2], [dc.DC_R, dc.DC_W])
    rt.dc_task_submit(dc.DC_TRSM_INV_CAST, hs, [dc.DC_R, dc.DC_R, dc.DC_RW, dc.DC_W])
    rt.dc_wait_all()
    for h in hs:
        rt.dc_unregister(h)
    got = tx.cpu()
    assert torch.equal(ts.cpu(), got.to(torch.bfloat16))
    ref = core.trsm_tile(l, x.astype(np.float64))
    tol = 64 * nb * U * np.linalg.cond(l) + 2.0 ** -24
    assert np.abs(got.numpy().astype(np.float64) - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("nb", [1, 16, 37, 100, 128, 200, 255, 256, 257, 512])
def test_potrf_task(dc, rt, torch_dev, nb):
    a = inputs.spd_normal(nb, nb, 0.1)
    got = _single(dc, rt, dc.DC_POTRF, [a], [dc.DC_RW], torch_dev)[0]
    ref, info = core.potrf_tile(a)
    assert info == 0
    lo, up = np.tril_indices(nb), np.triu_indices(nb, 1)
    assert np.abs(got[lo] - ref[lo]).max() <= 16 * nb * U * np.linalg.cond(a) * np.abs(ref).max()
    assert np.array_equal(got[up], a[up])


# ----------------------------------------------------------- whole factor

@pytest.mark.parametrize("n,tile", [(512, 128), (300, 128), (1000, 96), (2048, 256), (129, 64),
                                    (64, 64), (1, 16)])
def test_potrf_matches_oracle(dc, rt, torch_dev, n, tile):
    a = inputs.spd_uniform(n, n + tile)
    l, info, _ = _factor(dc, rt, torch_dev, a, tile)
    assert info == 0
    lr, info_r = core.potrf_tiled(a, tile)
    lr = np.tril(lr)
    assert info_r == 0
    eta = core.backward_error_fro(a, l) if n <= 1024 else None
    if eta is not None:
        assert eta <= 1e-13, eta
    cond = np.linalg.cond(a)
    assert np.linalg.norm(l - lr) / np.linalg.norm(lr) <= 8 * n * U * cond
    assert_factor_elementwise(l, lr, a, cond)


def test_potrf_ill_conditioned(dc, rt, torch_dev):
    n, tile = 1024, 128
    a = inputs.spd_cond(n, 3, 1e6)
    l, info, _ = _factor(dc, rt, torch_dev, a, tile)
    assert info == 0
    assert core.backward_error_fro(a, l) <= 1e-13


@pytest.mark.parametrize("n,tile", [(256, 64), (500, 128), (1024, 256), (333, 100)])
def test_potrf_integer_bitwise(dc, rt, torch_dev, n, tile):
    a, l0 = inputs.integer_factor(n, n)
    l, info, _ = _factor(dc, rt, torch_dev, a, tile)
    assert info == 0
    assert np.array_equal(l, l0)


def test_upper_triangle_untouched(dc, rt, torch_dev):
    n, tile = 400, 128
    a = inputs.spd_uniform(n, 5)
    a[np.triu_indices(n, 1)] = np.nan
    ta = _gpu(torch_dev, a)
    info = dc.potrf(rt, ta, tile)
    out = ta.cpu().numpy()
    assert info == 0
    assert np.all(np.isnan(out[np.triu_indices(n, 1)]))
    assert np.isfinite(out[np.tril_indices(n)]).all()


def test_breakdown_info(dc, rt, torch_dev):
    a, _ = inputs.integer_factor(300, 9)
    a[200, 200] -= 1e7
    _, info, _ = _factor(dc, rt, torch_dev, a, 64)
    assert info == 201
    assert core.potrf_tiled(a, 64)[1] == 201
    a2, _ = inputs.integer_factor(100, 1)
    a2[0, 0] = -1.0
    _, info2, _ = _factor(dc, rt, torch_dev, a2, 32)
    assert info2 == 1


@pytest.mark.parametrize("nb", [40, 200, 256, 300, 512])
def test_potrf_tile_breakdown_column(dc, rt, torch_dev, nb):
    """One tile (one POTRF task): a pivot made negative at column p gives
    info p + 1, at the first column, inside a 16-column block, at block
    edges and at the last column.  The finished 16-column blocks left of
    p's block are exact (integer factor) in the rows the failed factor
    owns: a tile of order above 256 is factored as 2 x 2 blocks, and after
    a failure in the leading 256 columns the tasks that would solve the
    rows below are skipped (the contract leaves the contents unspecified
    after a breakdown; only info is promised)."""
    a, l0 = inputs.integer_factor(nb, nb + 3)
    for p in sorted({0, 15, 16, 17, nb // 2 + 5, nb - 1}):
        a2 = a.copy()
        a2[p, p] -= 1e7
        l, info, _ = _factor(dc, rt, torch_dev, a2, nb)
        assert info == p + 1, (p, info)
        assert core.potrf_tiled(a2, nb)[1] == p + 1
        done = 16 * (p // 16)
        rows = 256 if nb > 256 and p < 256 else nb
        assert np.array_equal(l[:rows, :done], l0[:rows, :done]), p


def test_deterministic_across_runs_and_workers(dc, torch_dev):
    n, tile = 1536, 128
    a = inputs.spd_normal(n, 4, 1e-2)
    outs = []
    for workers in (0, 1, 7, 64, 0):
        with dc.Runtime(device=0, workers=workers) as rt:
            l, info, _ = _factor(dc, rt, torch_dev, a, tile)
            assert info == 0
            outs.append(l)
    for l in outs[1:]:
        assert np.array_equal(l, outs[0])


def test_lookahead_changes_no_bit(dc, torch_dev):
    """The lookahead depth only moves tasks between levels: the factor is
    bit-identical for every depth.  At 4096, tile 512, every diagonal factor
    outweighs its level's other work spread over the CUs, so the POTRF
    splitting is taken too."""
    for n, tile in ((1536, 128), (4096, 512)):
        a = inputs.spd_normal(n, 6, 1e-2)
        ref = None
        for depth in (0, 2, 48, 1000):
            with dc.Runtime(device=0, lookahead=depth) as rt:
                l, info, _ = _factor(dc, rt, torch_dev, a, tile)
            assert info == 0
            if ref is None:
                ref = l
                assert core.backward_error_fro(a, l) <= 1e-13
            assert np.array_equal(l, ref), (n, depth)


# ------------------------------------------------------------------ solve

@pytest.mark.parametrize("n,r,tile", [(512, 1, 128), (700, 3, 128), (1024, 16, 256), (50, 2, 16)])
def test_potrs_matches_oracle(dc, rt, torch_dev, n, r, tile):
    a = inputs.spd_uniform(n, n)
    bm = inputs.rhs(n, r, n + 1)
    lr = np.tril(core.potrf_tiled(a, tile)[0])
    tl = _gpu(torch_dev, lr)
    tb = _gpu(torch_dev, bm)
    dc.potrs(rt, tl, tb, tile)
    x = tb.cpu().numpy()
    xr = core.potrs_tiled(lr, bm, tile)
    assert np.abs(x - xr).max() / np.abs(xr).max() <= 16 * n * U * np.linalg.cond(a)


def test_potrs_integer_exact(dc, rt, torch_dev):
    n, r, tile = 400, 4, 64
    a, l0 = inputs.integer_factor(n, 3, diag_choices=(1.0, 2.0, 4.0))
    x0 = inputs.integer_solution(n, r, 4)
    bm = a @ x0
    tl, tb = _gpu(torch_dev, l0), _gpu(torch_dev, bm)
    dc.potrs(rt, tl, tb, tile)
    assert np.array_equal(tb.cpu().numpy(), x0)


def test_factor_then_solve_config0(dc, rt, torch_dev):
    """n=512, tile 128 (4x4 tiles, 20 tasks), one RHS."""
    n, tile = 512, 128
    a = inputs.spd_uniform(n, 0)
    bm = inputs.rhs(n, 1, 1)
    l, info, ta = _factor(dc, rt, torch_dev, a, tile)
    assert info == 0
    tb = _gpu(torch_dev, bm)
    dc.potrs(rt, ta, tb, tile)
    x = tb.cpu().numpy()
    lr = np.tril(core.potrf_tiled(a, tile)[0])
    xr = core.potrs_tiled(lr, bm, tile)
    assert core.backward_error_fro(a, l) <= 1e-13
    assert np.abs(x - xr).max() / np.abs(xr).max() <= 1e-12
