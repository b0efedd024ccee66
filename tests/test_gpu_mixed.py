"""GPU parity of the mixed-precision path: FP32/BF16 update kernels and the
FP64-residual iterative refinement solver (dc_posv_ir).

Bars:
  * FP32-input SYRK/GEMM tasks: |got - ref| <= 2 k u32 (|X||Y|^T + |C|)
    against the exact products of the FP32 inputs (numpy in FP64), FP32
    accumulation being the only rounding beyond the inputs;
  * BF16-input tasks: the same against products of the BF16-rounded inputs
    (oracle/mixed.round_bf16), plus the rounding of the FP32 result;
  * TRSM on FP32 tiles: FP64 arithmetic rounded to FP32 on store, so within
    one FP32 ulp-scale of the FP64 oracle; its BF16 copy is the RNE rounding
    of the stored FP32 values, bit for bit;
  * refined solutions: ||x - x_ref||_inf / ||x_ref||_inf <= 1e-10 for cond(A)
    <= 1e6 (the stated accuracy target), x_ref from the oracle's FP64 solve
    refined with a long-double residual;
  * exact-integer systems: x equals the integer solution bit for bit.
"""
import numpy as np
import pytest

from oracle import core, mixed
from paper_1304_0878_amd import inputs

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


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


def _t(torch_dev, a, dtype=None):
    torch, dev = torch_dev
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t.to(dtype) if dtype is not None else t


def _run(rt, dc, kind, tensors, modes):
    hs = [rt.register_tensor(t) for t in tensors]
    rt.dc_task_submit(kind, hs, modes)
    rt.dc_wait_all()
    for h in hs:
        rt.dc_unregister(h)


@pytest.mark.parametrize("cdt", ["f32", "f64"])
@pytest.mark.parametrize("m,n,k", [(128, 128, 128), (300, 200, 256), (512, 384, 512)])
def test_gemm_f32_inputs(dc, rt, torch_dev, m, n, k, cdt):
    torch = torch_dev[0]
    g = np.random.default_rng(m + n + k)
    x = g.standard_normal((m, k)).astype(np.float32)
    y = g.standard_normal((n, k)).astype(np.float32)
    c = g.standard_normal((m, n)).astype(np.float32 if cdt == "f32" else np.float64)
    tc = _t(torch_dev, c)
    _run(rt, dc, dc.DC_GEMM, [_t(torch_dev, x), _t(torch_dev, y), tc], [dc.DC_R, dc.DC_R, dc.DC_RW])
    got = tc.cpu().numpy().astype(np.float64)
    ref = c.astype(np.float64) - x.astype(np.float64) @ y.astype(np.float64).T
    bound = 2 * k * U32 * (np.abs(x.astype(np.float64)) @ np.abs(y.astype(np.float64)).T + np.abs(c))
    assert np.all(np.abs(got - ref) <= bound + 1e-30)


@pytest.mark.parametrize("cdt", ["f32", "f64"])
@pytest.mark.parametrize("m,k", [(128, 128), (300, 256), (512, 512)])
def test_syrk_bf16_inputs(dc, rt, torch_dev, m, k, cdt):
    torch = torch_dev[0]
    g = np.random.default_rng(m * 7 + k)
    x32 = g.standard_normal((m, k)).astype(np.float32)
    xb = mixed.round_bf16(x32)
    c = g.standard_normal((m, m)).astype(np.float32 if cdt == "f32" else np.float64)
    tc = _t(torch_dev, c)
    tx = _t(torch_dev, x32, torch.bfloat16)
    _run(rt, dc, dc.DC_SYRK, [tx, tc], [dc.DC_R, dc.DC_RW])
    got = tc.cpu().numpy().astype(np.float64)
    xd = xb.astype(np.float64)
    ref = c.astype(np.float64) - xd @ xd.T
    lo, up = np.tril_indices(m), np.triu_indices(m, 1)
    bound = 2 * k * U32 * (np.abs(xd) @ np.abs(xd).T + np.abs(c))
    assert np.all(np.abs(got[lo] - ref[lo]) <= bound[lo] + 1e-30)
    assert np.array_equal(got[up], c.astype(np.float64)[up])


def test_syrk_gemm_f32_integer_exact(dc, rt, torch_dev):
    """Small integers: FP32 accumulation is exact, so any order is bitwise."""
    torch = torch_dev[0]
    g = np.random.default_rng(3)
    x = g.integers(-3, 4, (256, 256)).astype(np.float32)
    y = g.integers(-3, 4, (256, 256)).astype(np.float32)
    c = g.integers(-50, 50, (256, 256)).astype(np.float64)
    tc = _t(torch_dev, c)
    _run(rt, dc, dc.DC_GEMM, [_t(torch_dev, x), _t(torch_dev, y), tc], [dc.DC_R, dc.DC_R, dc.DC_RW])
    assert np.array_equal(tc.cpu().numpy(), c - x.astype(np.float64) @ y.astype(np.float64).T)
    tb = _t(torch_dev, x, torch.bfloat16)
    tc2 = _t(torch_dev, c)
    _run(rt, dc, dc.DC_SYRK, [tb, tc2], [dc.DC_R, dc.DC_RW])
    ref = c - x.astype(np.float64) @ x.astype(np.float64).T
    lo = np.tril_indices(256)
    assert np.array_equal(tc2.cpu().numpy()[lo], ref[lo])


@pytest.mark.parametrize("m,nb", [(128, 128), (100, 37), (512, 512)])
def test_trsm_f32_tile_and_bf16_copy(dc, rt, torch_dev, m, nb):
    torch = torch_dev[0]
    g = np.random.default_rng(m + nb)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb))
    x = g.standard_normal((m, nb)).astype(np.float32)
    tx = _t(torch_dev, x)
    ts = torch.zeros(m, nb, dtype=torch.bfloat16, device=torch_dev[1])
    _run(rt, dc, dc.DC_TRSM_CAST, [_t(torch_dev, l), tx, ts], [dc.DC_R, dc.DC_RW, dc.DC_W])
    got = tx.cpu().numpy()
    ref = core.trsm_tile(l, x.astype(np.float64))
    assert np.all(np.abs(got.astype(np.float64) - ref) <= 2 * U32 * np.abs(ref) + 1e-12 * np.abs(ref).max())
    assert np.array_equal(ts.cpu().float().numpy(), mixed.round_bf16(got))


def _ir(dc, rt, torch_dev, a, bm, tile, upd, maxit=30):
    torch = torch_dev[0]
    ta, tb = _t(torch_dev, a), _t(torch_dev, bm)
    tx = torch.zeros_like(tb)
    rep = dc.posv_ir(rt, ta, tb, tx, tile, upd=upd, tol=1e-12, maxit=maxit)
    return tx.cpu().numpy(), rep, ta.cpu().numpy()


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("upd", ["f32", "bf16", "f64"])
def test_posv_ir_accuracy(dc, rt, torch_dev, kappa, upd):
    n, tile, r = 1000, 128, 2
    a = inputs.spd_cond(n, 11, kappa)
    bm = inputs.rhs(n, r, 12)
    code = {"f32": dc.DC_F32, "bf16": dc.DC_BF16, "f64": dc.DC_F64}[upd]
    x, rep, a_after = _ir(dc, rt, torch_dev, a, bm, tile, code)
    xref = mixed.reference_solution(a, bm, tile)
    err = np.abs(x - xref).max() / np.abs(xref).max()
    assert rep["converged"] == 1, rep
    assert err <= 1e-10, (err, rep)
    assert np.array_equal(a_after, a)   # A is never modified


def test_posv_ir_ragged_multi_rhs(dc, rt, torch_dev):
    n, tile, r = 777, 96, 5
    a = inputs.spd_cond(n, 5, 1e3)
    bm = inputs.rhs(n, r, 6)
    x, rep, _ = _ir(dc, rt, torch_dev, a, bm, tile, dc.DC_F32)
    xref = mixed.reference_solution(a, bm, tile)
    assert np.abs(x - xref).max() / np.abs(xref).max() <= 1e-10
    assert rep["final_prec"] == dc.DC_F32 and rep["fallbacks"] == 0


@pytest.mark.parametrize("upd", ["f32", "bf16"])
def test_posv_ir_integer_exact(dc, rt, torch_dev, upd):
    n, tile, r = 512, 128, 3
    a, l0 = inputs.integer_factor(n, 21, diag_choices=(1.0, 2.0, 4.0))
    x0 = inputs.integer_solution(n, r, 22)
    bm = a @ x0
    code = dc.DC_F32 if upd == "f32" else dc.DC_BF16
    x, rep, _ = _ir(dc, rt, torch_dev, a, bm, tile, code)
    assert np.array_equal(x, x0), rep
    assert rep["iterations"] == 0 and rep["converged"] == 1 and rep["fallbacks"] == 0


def test_posv_ir_not_spd_reports_info(dc, rt, torch_dev):
    torch = torch_dev[0]
    a, _ = inputs.integer_factor(256, 2)
    a[100, 100] = -5.0
    ta, tb = _t(torch_dev, a), _t(torch_dev, np.ones((256, 1)))
    tx = torch.zeros_like(tb)
    ha, hb, hx = rt.register_tensor(ta), rt.register_tensor(tb), rt.register_tensor(tx)
    rep = rt.dc_posv_ir(ha, hb, hx, 64, dc.DC_F32)
    assert rt.dc_get_info(ha) == 101
    assert rep["final_prec"] == dc.DC_F64 and rep["fallbacks"] == 1
    for h in (hx, hb, ha):
        rt.dc_unregister(h)


def test_posv_ir_many_tiles(dc, rt, torch_dev):
    """Thousands of tile handles are created during the call (the handle
    table grows while the call runs); the solution must still be right."""
    n, tile, r = 1024, 16, 1
    a = inputs.spd_cond(n, 41, 1e3)
    bm = inputs.rhs(n, r, 42)
    x, rep, _ = _ir(dc, rt, torch_dev, a, bm, tile, dc.DC_F32)
    xref = mixed.reference_solution(a, bm, 64)
    assert rep["converged"] == 1, rep
    assert np.abs(x - xref).max() / np.abs(xref).max() <= 1e-10


# ------------------------------------------- the mixed factor on its own

# Backward errors of the GPU's mixed factor, filled in by the test below and
# printed at the end of the module (pytest -s shows them).
MIXED_ETA = {}


@pytest.mark.parametrize("upd", ["f32", "bf16"])
@pytest.mark.parametrize("n,tile", [(256, 128), (1024, 256), (2048, 256)])
def test_mixed_factor_backward_error_within_4x_of_emulation(dc, rt, torch_dev, upd, n, tile):
    """dc_potrf with FP32/BF16 updates: the factor's backward error
    ||A - L L^T||_F / ||A||_F (long double) is at most 4 times that of the
    oracle's numpy emulation of the same mixed scheme (FP32 off-diagonal
    storage, BF16-rounded inputs for BF16, FP32 accumulation)."""
    a = inputs.spd_normal(n, 21, 1e-2)
    ta = _t(torch_dev, a)
    u = dc.DC_F32 if upd == "f32" else dc.DC_BF16
    assert dc.potrf(rt, ta, tile, upd=u) == 0
    l = np.tril(ta.cpu().numpy())
    eta_gpu = core.backward_error_fro(a, l)
    l_emu, info = mixed.mixed_factor(a, tile, upd)
    assert info == 0
    eta_emu = core.backward_error_fro(a, l_emu)
    MIXED_ETA[(upd, n)] = (eta_gpu, eta_emu)
    print(f"mixed factor {upd} n={n} tile={tile}: eta_gpu={eta_gpu:.3e} eta_emulation={eta_emu:.3e}")
    assert eta_gpu <= 4 * eta_emu
    # the off-diagonal part holds FP32 values
    off = np.tril(l, -tile)
    assert np.array_equal(off, off.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("upd", ["f32", "bf16"])
def test_mixed_factor_exact_on_integer_factor(dc, rt, torch_dev, upd):
    """A = L0 L0^T with integer L0 (entries within BF16 and FP32 exactness):
    the mixed factor returns L0 bit for bit."""
    a, l0 = inputs.integer_factor(300, 8)
    ta = _t(torch_dev, a)
    u = dc.DC_F32 if upd == "f32" else dc.DC_BF16
    assert dc.potrf(rt, ta, 64, upd=u) == 0
    assert np.array_equal(np.tril(ta.cpu().numpy()), l0)


def test_mixed_factor_breakdown_reports_column(dc, rt, torch_dev):
    a = inputs.spd_uniform(300, 4)
    a[200, 200] = -1.0
    ta = _t(torch_dev, a)
    info = dc.potrf(rt, ta, 64, upd=dc.DC_F32)
    _, info_ref = core.potrf_tiled(a, 64)
    assert info == info_ref > 0
