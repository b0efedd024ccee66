"""dc_potrf_noalloc (the factorisation that allocates nothing, its graph
layout in a fixed device scratch array) against dc_potrf, through the C ABI.

Two calls in a row on one runtime, the second on a smaller matrix (the
scratch keeps the first call's contents; the second must not depend on
them), each compared element by element with dc_potrf's factor of the same
matrix within the first-order bound 16 n u cond(A) sqrt(a_ii) (the two use
different panel solves: substitution here, inverse products in dc_potrf),
and by its backward error (<= 1e-13).  A non-positive-definite matrix gives
dc_potrf's breakdown column; a graph too large for the scratch is refused
before anything runs.
"""
import ctypes

import numpy as np
import pytest

from oracle import core
from bounds import assert_factor_elementwise
from paper_1304_0878_amd import inputs

pytestmark = pytest.mark.gpu


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


def _noalloc(dc, rt, t, tile):
    h = rt.register_tensor(t)
    try:
        code = dc._lib.dc_potrf_noalloc(rt._ptr, ctypes.c_int64(h), ctypes.c_int64(tile))
        info = rt.dc_get_info(h) if code == 0 else None
    finally:
        rt.dc_unregister(h)
    return code, info


def test_noalloc_matches_potrf_on_two_calls(dc, torch_dev):
    torch, dev = torch_dev
    with dc.Runtime(device=0) as rt:
        for n, tile, seed in ((2048, 256, 31), (700, 128, 32)):
            a = inputs.spd_normal(n, seed, 1e-2)
            t_ref = torch.from_numpy(a).to(dev)
            t_na = torch.from_numpy(a).to(dev)
            assert dc.potrf(rt, t_ref, tile) == 0
            code, info = _noalloc(dc, rt, t_na, tile)
            assert code == 0 and info == 0, (code, info)
            torch.cuda.synchronize()
            l_ref = np.tril(t_ref.cpu().numpy())
            l_na = np.tril(t_na.cpu().numpy())
            assert_factor_elementwise(l_na, l_ref, a, np.linalg.cond(a))
            assert core.backward_error_fro(a, l_na) <= 1e-13
            # the strictly upper triangle is never touched
            iu = np.triu_indices(n, 1)
            assert np.array_equal(t_na.cpu().numpy()[iu], a[iu])


def test_noalloc_breakdown_column(dc, torch_dev):
    torch, dev = torch_dev
    a = inputs.spd_uniform(600, 7)
    a[400, 400] = -1.0
    with dc.Runtime(device=0) as rt:
        code, info = _noalloc(dc, rt, torch.from_numpy(a).to(dev), 128)
        assert code == 0
        ref = dc.potrf(rt, torch.from_numpy(a).to(dev), 128)
    assert info == ref == core.potrf_tiled(a, 128)[1] > 0


def test_noalloc_refuses_a_graph_beyond_the_scratch(dc, torch_dev):
    """n = 4096 with tile 32 is 357,760 tasks: their 128-byte descriptors
    alone (45.8 MB) exceed the 16 MiB scratch, so the call returns -ENOMEM
    before anything is uploaded or launched (the buffer is real memory all
    the same), and the runtime keeps working."""
    torch, dev = torch_dev
    n = 4096
    t = torch.zeros((n, n), dtype=torch.float64, device=dev)
    with dc.Runtime(device=0) as rt:
        code, _ = _noalloc(dc, rt, t, 32)
        assert code == -12
        a = inputs.spd_uniform(256, 3)
        code, info = _noalloc(dc, rt, torch.from_numpy(a).to(dev), 64)
        assert code == 0 and info == 0
