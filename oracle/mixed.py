"""Mixed-precision factor emulation and iterative refinement in numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/core.py``).

The mixed-precision variant of the tiled Cholesky keeps FP64 for the diagonal
tiles (POTRF stays FP64) and stores the off-diagonal tiles in FP32.  TRSM
runs in FP32 with the diagonal factor rounded to FP32; the SYRK and GEMM
updates multiply FP32 (or BF16-rounded) inputs with FP32 accumulation, the
SYRK result being subtracted in FP64 from the FP64 diagonal tile and the GEMM
result in FP32 from the FP32 tile.  Solves read that factor and compute in
FP64; iterative refinement forms the residual b - A x in FP64 from the
original A.

The accumulation order of a numpy float32 product is the BLAS library's
own, so this emulation is a statistical reference for the size of the mixed
factor's backward error, not a bitwise one.
"""
import numpy as np

from . import core


def round_bf16(x):
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32 holding the rounded values."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def mixed_factor(a, b, upd="f32"):
    """Tiled right-looking factor with FP64 diagonal tiles and FP32
    off-diagonal tiles.  Returns (L as float64 lower triangle, info)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    t = (n + b - 1) // b
    spans = [(k * b, min(n, (k + 1) * b)) for k in range(t)]
    diag = [a[s:e, s:e].copy() for s, e in spans]
    off = {}
    for i in range(t):
        for j in range(i):
            (si, ei), (sj, ej) = spans[i], spans[j]
            off[(i, j)] = a[si:ei, sj:ej].astype(np.float32)

    def operand(x):
        return round_bf16(x) if upd == "bf16" else x

    for k in range(t):
        lkk, info = core.potrf_tile(diag[k])
        if info:
            return None, spans[k][0] + info
        diag[k] = np.tril(lkk)
        l32 = diag[k].astype(np.float32)
        for i in range(k + 1, t):
            x = off[(i, k)]
            for j in range(x.shape[1]):
                x[:, j] = (x[:, j] - x[:, :j] @ l32[j, :j]) / l32[j, j]
        for i in range(k + 1, t):
            xi = operand(off[(i, k)])
            upd_ii = (xi @ xi.T).astype(np.float64)
            diag[i] = diag[i] - np.tril(upd_ii)
            for j in range(k + 1, i):
                xj = operand(off[(j, k)])
                off[(i, j)] = (off[(i, j)] - xi @ xj.T).astype(np.float32)

    l = np.zeros_like(a)
    for i in range(t):
        si, ei = spans[i]
        l[si:ei, si:ei] = np.tril(diag[i])
        for j in range(i):
            sj, ej = spans[j]
            l[si:ei, sj:ej] = off[(i, j)].astype(np.float64)
    return l, 0


def refine(a, bm, l, b, tol=1e-12, maxit=30):
    """Iterative refinement with a given factor ``l`` and an accurate
    residual.

    x0 = solve(b); repeat r = b - A x evaluated in extended precision and
    rounded to FP64 (an FP64 residual accumulated plainly carries errors of
    about u |A| |x|, which limit the refined solution to about cond(A) u
    relative error: 2.4e-10 measured at cond 1e6), d = solve(r), x += d,
    until ||d||_inf <= tol ||x||_inf for every column (converged), or
    ||d_i||_inf > 0.5 ||d_{i-1}||_inf in some column (stagnation: d_i is not
    added), or maxit steps.  From the second correction on, the corrections
    are taken to contract geometrically with the observed ratio
    rho = ||d_i|| / ||d_{i-1}||, so the error left after adding d_i is
    estimated as rho ||d_i|| / (1 - rho) = ||d_i||^2 / (||d_{i-1}|| - ||d_i||)
    (the estimate of extra-precise refinement, Demmel et al., ACM TOMS
    2006); when that is <= tol ||x||_inf in every column the step converges
    too, which saves the solve whose only use would be to confirm it.
    Returns (x, steps, status) with steps the refinement steps before the
    converging one and status in {"converged", "stagnated", "maxit"}."""
    x = core.potrs_tiled(l, bm, b)
    prev = None
    it = 0

    def colmax(v):
        return np.max(np.abs(v), axis=0) if v.ndim > 1 else np.max(np.abs(v))

    while True:
        r = core.residual_ld(a, x, bm)
        d = core.potrs_tiled(l, r, b)
        dn, xn = colmax(d), colmax(x)
        small = np.all(dn <= tol * xn)
        if not small and prev is not None and np.any(dn > 0.5 * prev):
            return x, it, "stagnated"
        x = x + d
        if small:
            return x, it, "converged"
        if prev is not None:
            # no stagnation here: every column has dn <= prev / 2, so the
            # denominator is positive wherever dn is
            left = np.where(dn > 0, dn * dn / np.where(dn > 0, prev - dn, 1.0), 0.0)
            if np.all(left <= tol * xn):
                return x, it, "converged"
        it += 1
        if it >= maxit:
            return x, it, "maxit"
        prev = dn


def reference_solution(a, bm, b=None, steps=2):
    """x_ref: FP64 tiled factor and solve, then ``steps`` refinement steps
    with a long-double residual, so its own error is far below the
    condition-number-limited error of a plain FP64 solve."""
    n = a.shape[0]
    b = b or min(n, 256)
    l, info = core.potrf_tiled(a, b)
    if info:
        raise np.linalg.LinAlgError(f"matrix not positive definite (info={info})")
    l = np.tril(l)
    x = core.potrs_tiled(l, bm, b)
    for _ in range(steps):
        r = core.residual_ld(a, x, bm)
        x = x + core.potrs_tiled(l, r, b)
    return x
