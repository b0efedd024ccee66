"""GPU parity at the workloads' full sizes, in the configuration bench.py runs.

* n = 8192, tiles 256 / 384 / 512, 16 right-hand sides (A = B B^T/n +
  1e-2 I): the whole factor and solution against the oracle's tiled
  factorisation and solve (normwise, first-order perturbation bounds), and
  sampled entries of A - L L^T computed by the oracle in long double.
* n = 32768, tile 512, the bench's matrix (generated on the device the same
  way): the oracle cannot factor it within a test, so the checks are
  properties that hold at any size: sampled entries of A - L L^T (oracle,
  long double) within the FP64 bound, the backward error probe, and for
  the mixed-precision solves at cond ~1e2 / 1e4 / 1e6 the normwise backward
  error of the refined solution from the oracle's long-double residual,
  whose product with the condition bound must stay below 1e-10.
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


def _samples(n, count, seed):
    g = np.random.default_rng(seed)
    rows = g.integers(0, n, count)
    cols = np.minimum(rows, g.integers(0, n, count))
    # the last rows and the diagonal, where the most updates accumulate
    rows = np.concatenate([rows, np.full(8, n - 1), np.arange(n - 8, n)])
    cols = np.concatenate([cols, np.arange(0, n, n // 8)[:8], np.arange(n - 8, n)])
    return rows.astype(np.int64), cols.astype(np.int64)


@pytest.fixture(scope="module")
def a8192():
    return inputs.spd_normal(8192, 11, 1e-2)


@pytest.mark.parametrize("tile", [256, 384, 512])
def test_n8192_factor_and_solve_vs_oracle(dc, torch_dev, a8192, tile):
    torch, dev = torch_dev
    n, r = 8192, 16
    a = a8192
    b = inputs.rhs(n, r, 12)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    with dc.Runtime(device=0) as rt:
        assert dc.potrf(rt, ta, tile) == 0
        dc.potrs(rt, ta, tb, tile)
    torch.cuda.synchronize()
    l = np.tril(ta.cpu().numpy())
    x = tb.cpu().numpy()
    lr = np.tril(core.potrf_tiled(a, tile)[0])
    xr = core.potrs_tiled(lr, b, tile)
    cond = 1.0 + 4.0 / 1e-2        # (lambda_max + 1e-2) / 1e-2 bound, lambda_max <= 4
    assert np.linalg.norm(l - lr) / np.linalg.norm(lr) <= 8 * n * U * cond
    assert_factor_elementwise(l, lr, a, cond)
    assert np.abs(x - xr).max() / np.abs(xr).max() <= 16 * n * U * cond
    rows, cols = _samples(n, 400, tile)
    res = core.sampled_residual(a, l, rows, cols)
    assert np.abs(res).max() / np.abs(a).max() <= 1e-13


@pytest.fixture(scope="module")
def big(torch_dev):
    """The bench's n = 32768 matrix (cond ~1e2) on the device and on the host."""
    import sys, os
    torch, dev = torch_dev
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    a, lam, delta = bench.make_spd(torch, 32768, 0, 1e2, dev)
    torch.cuda.synchronize()
    return a, a.cpu().numpy(), lam, delta


def test_n32768_fp64_factor_sampled_residual(dc, torch_dev, big):
    torch, dev = torch_dev
    a_dev, a_host, _, _ = big
    n, tile = 32768, 512
    l_dev = a_dev.clone()
    with dc.Runtime(device=0) as rt:
        assert dc.potrf(rt, l_dev, tile) == 0
    torch.cuda.synchronize()
    # backward error probe on the device (properties at any size)
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    z = torch.randn(n, 4, dtype=torch.float64, device=dev, generator=g)
    low = torch.tril(l_dev)
    az = a_dev @ z
    eta = float(torch.linalg.matrix_norm(az - low @ (low.T @ z)) / torch.linalg.matrix_norm(az))
    del low
    assert eta <= 1e-13
    l_host = np.tril(l_dev.cpu().numpy())
    del l_dev
    rows, cols = _samples(n, 300, 3)
    res = core.sampled_residual(a_host, l_host, rows, cols)
    assert np.abs(res).max() / np.abs(a_host).max() <= 1e-13


@pytest.mark.parametrize("kappa,upd", [(1e2, "f32"), (1e4, "f32"), (1e6, "f32"), (1e2, "bf16"),
                                       (1e4, "bf16"), (1e6, "bf16")])
def test_n32768_mixed_refinement_accuracy(dc, torch_dev, big, kappa, upd):
    torch, dev = torch_dev
    a_dev, a_host, lam, delta = big
    n = 32768
    shift = lam / (kappa - 1.0) - delta          # move from cond 1e2 to cond kappa
    a = a_dev.clone()
    a.diagonal().add_(shift)
    b = torch.from_numpy(inputs.rhs(n, 1, 21)).to(dev)
    x = torch.zeros_like(b)
    code = {"f32": dc.DC_F32, "bf16": dc.DC_BF16}[upd]
    with dc.Runtime(device=0) as rt:
        rep = dc.posv_ir(rt, a, b, x, 512, code)
    torch.cuda.synchronize()
    # BF16 updates at cond 1e4 and 1e6 may fall back to FP32 (or FP64)
    # updates: the result must still have converged, with the fallback stated
    print(f"n=32768 cond {kappa:g} {upd}: converged={rep['converged']} "
          f"final_prec={rep['final_prec']} fallbacks={rep['fallbacks']} "
          f"iterations={rep['iterations']} last_update={rep['last_update']:.2e}")
    assert rep["converged"] == 1, rep
    anorm = float(a.abs().sum(dim=1).max())      # infinity norm (A is stored whole)
    del a
    xh, bh = x.cpu().numpy(), b.cpu().numpy()
    diag = np.diag_indices(n)
    d0 = a_host[diag].copy()
    a_host[diag] = d0 + shift                    # the same rounding as on the device
    try:
        r = core.residual_ld(a_host, xh, bh)
    finally:
        a_host[diag] = d0
    eta = np.abs(r).max() / (anorm * np.abs(xh).max() + np.abs(bh).max())
    cond_bound = 2.0 * kappa
    assert cond_bound * eta <= 1e-10, (eta, rep)
