"""Error bounds shared by the GPU parity tests."""
import numpy as np

U = 2.0 ** -53


def assert_factor_elementwise(l, lr, a, cond, c=16):
    """Element by element: two backward-stable factors of A differ, to first
    order, by dL = L Phi with ||Phi||_2 <~ n u cond(A) (Phi is built from
    L^-1 E L^-T), so row i of dL is at most ||L(i,:)||_2 n u cond(A) =
    sqrt(a_ii) n u cond(A) in norm, and so is each of its entries; c covers
    both factors and the constant."""
    n = a.shape[0]
    bound = c * n * U * cond * np.sqrt(np.diag(a))[:, None]
    diff = np.abs(l - lr)
    bad = diff > bound
    assert not bad.any(), (np.argwhere(bad)[:5], diff[bad][:5], bound.max())
