"""ctypes bindings of the plain C oracle (``oracle.c``), taking numpy arrays.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.

Every array argument is a C-contiguous float64 numpy array in row-major
order; functions that update a matrix work on a copy and return it, so
callers never see their inputs modified.
"""
import ctypes
import numpy as np

from .build_oracle import ensure_built

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64

# kind codes of or_run_task (tile tasks of the factor and of the solve)
POTRF, TRSM, SYRK, GEMM, TRSM_L, GEMM_RHS_N, TRSM_LT, GEMM_RHS_T = range(8)


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        l = ctypes.CDLL(path)
        sig = {
            "or_potrf_tile": (_I64, [_I64, _D, _I64]),
            "or_trsm_tile": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_gemm_tile": (None, [_I64, _I64, _I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_trtri_tile": (None, [_I64, _D, _I64, _D, _I64]),
            "or_trsm_inv_tile": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_syrk_tile": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_trsm_left_tile": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_trsm_left_t_tile": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_gemm_rhs_n": (None, [_I64, _I64, _I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_gemm_rhs_t": (None, [_I64, _I64, _I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_run_task": (_I64, [ctypes.c_int, _I64, _I64, _D, _I64, _I64, _I64, _I64,
                                   _D, _I64, _I64]),
            "or_potrf_tiled": (_I64, [_I64, _D, _I64, _I64]),
            "or_potrf_unblocked": (_I64, [_I64, _D, _I64]),
            "or_potrs_tiled": (None, [_I64, _I64, _D, _I64, _D, _I64, _I64]),
            "or_potrs_unblocked": (None, [_I64, _I64, _D, _I64, _D, _I64]),
            "or_backward_error_fro": (ctypes.c_double, [_I64, _D, _I64, _D, _I64]),
            "or_backward_error_est": (ctypes.c_double, [_I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_sampled_residual": (None, [_I64, _D, _I64, _D, _I64, _I64,
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64), _D]),
            "or_residual_ld": (None, [_I64, _I64, _D, _I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_residual_f64": (None, [_I64, _I64, _D, _I64, _D, _I64, _D, _I64, _D, _I64]),
            "or_num_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mat(a):
    a = _f64(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return a


# ---------------------------------------------------------------- tile tasks

def potrf_tile(d):
    """POTRF of one tile; returns (L in the lower triangle, info)."""
    d = _f64(d).copy()
    info = lib().or_potrf_tile(d.shape[0], _p(d), d.shape[1])
    return d, int(info)


def trsm_tile(l, x):
    """X <- X L^{-T} (right, lower, transposed, non-unit)."""
    l, x = _f64(l), _f64(x).copy()
    lib().or_trsm_tile(x.shape[0], x.shape[1], _p(l), l.shape[1], _p(x), x.shape[1])
    return x


def trtri_tile(l):
    """W = L^{-1} for lower-triangular L (non-unit); W's upper part is zero."""
    l = _f64(l)
    w = np.zeros_like(l)
    lib().or_trtri_tile(l.shape[0], _p(l), l.shape[1], _p(w), w.shape[1])
    return w


def trsm_inv_tile(w, x):
    """X <- X W^T with W lower triangular (only W's lower part is read)."""
    w, x = _f64(w), _f64(x).copy()
    lib().or_trsm_inv_tile(x.shape[0], x.shape[1], _p(w), w.shape[1], _p(x), x.shape[1])
    return x


def gemm_tile(c, x, y):
    """C <- C - X Y^T."""
    c, x, y = _f64(c).copy(), _f64(x), _f64(y)
    lib().or_gemm_tile(c.shape[0], c.shape[1], x.shape[1], _p(x), x.shape[1],
                       _p(y), y.shape[1], _p(c), c.shape[1])
    return c


def syrk_tile(c, x):
    """Lower half of C <- C - X X^T; the strictly upper part is untouched."""
    c, x = _f64(c).copy(), _f64(x)
    lib().or_syrk_tile(c.shape[0], x.shape[1], _p(x), x.shape[1], _p(c), c.shape[1])
    return c


def trsm_left_tile(l, bm):
    """B <- L^{-1} B (forward substitution)."""
    l, bm = _f64(l), _mat(bm).copy()
    lib().or_trsm_left_tile(bm.shape[0], bm.shape[1], _p(l), l.shape[1], _p(bm), bm.shape[1])
    return bm


def trsm_left_t_tile(l, bm):
    """B <- L^{-T} B (backward substitution)."""
    l, bm = _f64(l), _mat(bm).copy()
    lib().or_trsm_left_t_tile(bm.shape[0], bm.shape[1], _p(l), l.shape[1], _p(bm), bm.shape[1])
    return bm


def gemm_rhs_n(bi, l_ik, bk):
    """B_I <- B_I - L_IK B_K."""
    bi, l_ik, bk = _mat(bi).copy(), _f64(l_ik), _mat(bk)
    lib().or_gemm_rhs_n(bi.shape[0], bi.shape[1], bk.shape[0], _p(l_ik), l_ik.shape[1],
                        _p(bk), bk.shape[1], _p(bi), bi.shape[1])
    return bi


def gemm_rhs_t(bi, l_ki, xk):
    """B_I <- B_I - L_KI^T X_K."""
    bi, l_ki, xk = _mat(bi).copy(), _f64(l_ki), _mat(xk)
    lib().or_gemm_rhs_t(bi.shape[0], bi.shape[1], xk.shape[0], _p(l_ki), l_ki.shape[1],
                        _p(xk), xk.shape[1], _p(bi), bi.shape[1])
    return bi


# --------------------------------------------------------- whole algorithms

def potrf_tiled(a, b, inplace=False):
    """Tiled Cholesky in submission order.  Returns (L lower, info).

    Only the lower triangle of ``a`` is read; the strictly upper part of the
    result is the input's upper part, unchanged (use numpy.tril for L)."""
    a = _f64(a)
    if not inplace:
        a = a.copy()
    n = a.shape[0]
    info = lib().or_potrf_tiled(n, _p(a), a.shape[1], b)
    return a, int(info)


def potrf_unblocked(a):
    a = _f64(a).copy()
    info = lib().or_potrf_unblocked(a.shape[0], _p(a), a.shape[1])
    return a, int(info)


def potrs_tiled(l, bm, b):
    """Solve L L^T X = B with the tiled forward and backward tasks."""
    l = _f64(l)
    squeeze = np.ndim(bm) == 1
    x = _mat(bm).copy()
    lib().or_potrs_tiled(l.shape[0], x.shape[1], _p(l), l.shape[1], _p(x), x.shape[1], b)
    return x[:, 0] if squeeze else x


def potrs_unblocked(l, bm):
    l = _f64(l)
    squeeze = np.ndim(bm) == 1
    x = _mat(bm).copy()
    lib().or_potrs_unblocked(l.shape[0], x.shape[1], _p(l), l.shape[1], _p(x), x.shape[1])
    return x[:, 0] if squeeze else x


def run_task(kind, a, b, ti, tj=0, tk=0, bm=None):
    """Run one tile task in place on ``a`` (and ``bm`` for solve tasks)."""
    n = a.shape[0]
    if bm is None:
        return int(lib().or_run_task(kind, n, b, _p(a), a.shape[1], ti, tj, tk, None, 0, 0))
    return int(lib().or_run_task(kind, n, b, _p(a), a.shape[1], ti, tj, tk,
                                 _p(bm), bm.shape[1], bm.shape[1]))


# ----------------------------------------------------------------- checkers

def backward_error_fro(a, l):
    """||A - L L^T||_F / ||A||_F in long double (A symmetric, lower read)."""
    a, l = _f64(a), _f64(np.tril(l))
    return float(lib().or_backward_error_fro(a.shape[0], _p(a), a.shape[1], _p(l), l.shape[1]))


def backward_error_est(a, l, z):
    """||(A - L L^T) Z||_F / ||A Z||_F in long double."""
    a, l, z = _f64(a), _f64(np.tril(l)), _mat(z)
    return float(lib().or_backward_error_est(a.shape[0], _p(a), a.shape[1], _p(l), l.shape[1],
                                             _p(z), z.shape[1]))


def sampled_residual(a, l, rows, cols):
    """Entries (A - L L^T)_{ij} at the sampled positions, long double."""
    a, l = _f64(a), _f64(l)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(len(rows), dtype=np.float64)
    lib().or_sampled_residual(a.shape[0], _p(a), a.shape[1], _p(l), l.shape[1], len(rows),
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    return out


def residual_ld(a, x, bm):
    """B - A X with A symmetric (lower read), long double accumulation."""
    a = _f64(a)
    squeeze = np.ndim(x) == 1
    x, bm = _mat(x), _mat(bm)
    r = np.empty_like(bm)
    lib().or_residual_ld(a.shape[0], x.shape[1], _p(a), a.shape[1], _p(x), x.shape[1],
                         _p(bm), bm.shape[1], _p(r), r.shape[1])
    return r[:, 0] if squeeze else r


def residual_f64(a, x, bm):
    a = _f64(a)
    squeeze = np.ndim(x) == 1
    x, bm = _mat(x), _mat(bm)
    r = np.empty_like(bm)
    lib().or_residual_f64(a.shape[0], x.shape[1], _p(a), a.shape[1], _p(x), x.shape[1],
                          _p(bm), bm.shape[1], _p(r), r.shape[1])
    return r[:, 0] if squeeze else r


def num_threads():
    return int(lib().or_num_threads())


# ------------------------------------------- the paper's worked example task

def scale_vector(x, factor):
    """The scale_vector task of the paper's Section 2: every element of a
    float vector multiplied in place by a float scalar (one correctly
    rounded binary32 product per element)."""
    x = np.asarray(x, dtype=np.float32)
    return x * np.float32(factor)
