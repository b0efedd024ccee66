"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no Cholesky arithmetic: it only draws random numbers and
forms symmetric positive definite matrices from them, so that the oracle and
the HIP path can be fed the same bytes.  Every generator uses numpy's PCG64
(``numpy.random.default_rng``).

Recipes (the workloads the library is measured on):

* ``spd_uniform(n, seed)``: B iid uniform[-1, 1], A = B B^T + n I;
* ``spd_normal(n, seed, delta)``: B iid N(0, 1), A = B B^T / n + delta I;
* ``delta_for_cond``: the shift delta that gives A = B B^T / n + delta I a
  target 2-norm condition number kappa, delta = (l_max - kappa l_min) /
  (kappa - 1) from the extreme eigenvalues of B B^T / n;
* ``integer_factor(n, seed)``: an integer lower-triangular L0 (off-diagonal
  in [-3, 3], diagonal in {1, 2, 4, 8}) and A = L0 L0^T, exact in binary64;
* ``batch_shapes``: orders n ~ U{16..512} and 1-4 right-hand sides;
* ``serving_trace``: Poisson arrivals, n log-uniform in [32, 16384],
  cond 10^U(2, 6), 1-8 right-hand sides.

Every A is explicitly symmetrised (lower triangle mirrored) after it is
formed.
"""
import numpy as np


def _sym(a):
    low = np.tril(a)
    return low + np.tril(a, -1).T


def rng(seed):
    return np.random.default_rng(seed)


def spd_uniform(n, seed):
    g = rng(seed)
    b = g.uniform(-1.0, 1.0, (n, n))
    a = b @ b.T
    a[np.diag_indices(n)] += n
    return np.ascontiguousarray(_sym(a))


def normal_gram(n, seed):
    """B B^T / n with B iid N(0, 1) (symmetrised)."""
    g = rng(seed)
    b = g.standard_normal((n, n))
    a = (b @ b.T) / n
    return np.ascontiguousarray(_sym(a))


def spd_normal(n, seed, delta):
    a = normal_gram(n, seed)
    a[np.diag_indices(n)] += delta
    return a


def extreme_eigs(a):
    w = np.linalg.eigvalsh(a)
    return float(w[0]), float(w[-1])


def delta_for_cond(gram, kappa):
    """Shift that makes gram + delta I have condition number kappa."""
    lmin, lmax = extreme_eigs(gram)
    return (lmax - kappa * lmin) / (kappa - 1.0)


def spd_cond(n, seed, kappa):
    """A = B B^T / n + delta I with cond_2(A) = kappa (exact eigenvalues)."""
    a = normal_gram(n, seed)
    d = delta_for_cond(a, kappa)
    a[np.diag_indices(n)] += d
    return a


def rhs(n, r, seed):
    g = rng(seed)
    return np.ascontiguousarray(g.standard_normal((n, r)))


def integer_factor(n, seed, diag_choices=(1.0, 2.0, 4.0, 8.0), offmax=3):
    """(A, L0) with L0 integer lower triangular and A = L0 L0^T exactly."""
    g = rng(seed)
    l0 = np.tril(g.integers(-offmax, offmax + 1, (n, n)).astype(np.float64), -1)
    l0[np.diag_indices(n)] = g.choice(np.asarray(diag_choices), n)
    a = l0 @ l0.T
    return np.ascontiguousarray(_sym(a)), l0


def integer_solution(n, r, seed, lim=4):
    g = rng(seed)
    return g.integers(-lim, lim + 1, (n, r)).astype(np.float64)


def batch_shapes(count, seed, nmin=16, nmax=512, rmin=1, rmax=4):
    g = rng(seed)
    ns = g.integers(nmin, nmax + 1, count)
    rs = g.integers(rmin, rmax + 1, count)
    return [int(v) for v in ns], [int(v) for v in rs]


def serving_trace(count, rate, seed, nmin=32, nmax=16384, kmin=2.0, kmax=6.0,
                  rmin=1, rmax=8):
    """Open-loop request stream: arrival times (s), orders, condition
    numbers and RHS counts."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(g.uniform(np.log(nmin), np.log(nmax), count))).astype(np.int64)
    kappas = 10.0 ** g.uniform(kmin, kmax, count)
    rs = g.integers(rmin, rmax + 1, count)
    return arrivals, ns, kappas, rs
