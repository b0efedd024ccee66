"""Pins of the CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: closed
forms, exact-integer cases, library routines (LAPACK via numpy/scipy), the
unblocked textbook definition, brute force on tiny inputs, and the paper's
worked example.  Runs on the CPU only.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import core, dag, mixed
from paper_1304_0878_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def _read_golden_matrix(path, tag):
    rows, on = [], False
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("A", "L"):
            on = line == tag
            continue
        if on:
            rows.append([float(v) for v in line.split()])
    return np.array(rows)


# ------------------------------------------------------------ tile kernels

@pytest.mark.parametrize("nb", [1, 7, 33, 64])
def test_potrf_tile_matches_lapack(nb):
    a = inputs.spd_uniform(nb, 10 + nb)
    l, info = core.potrf_tile(a)
    assert info == 0
    ref = np.linalg.cholesky(a)
    err = np.abs(np.tril(l) - ref).max() / np.abs(ref).max()
    assert err < 16 * nb * U


@pytest.mark.parametrize("m,nb", [(1, 1), (5, 9), (40, 32)])
def test_trsm_tile_matches_scipy(m, nb):
    g = np.random.default_rng(m * 100 + nb)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb))
    x = g.standard_normal((m, nb))
    got = core.trsm_tile(l, x)
    # X L^{-T} = (L^{-1} X^T)^T
    ref = sla.solve_triangular(l, x.T, lower=True).T
    assert np.allclose(got, ref, rtol=0, atol=64 * nb * U * np.abs(ref).max())
    # and the definition itself: X_new L^T == X_old
    assert np.allclose(got @ l.T, x, atol=64 * nb * U * np.abs(x).max())


def test_trtri_bidiagonal_closed_form():
    # L = I - s * subdiagonal has the inverse W_ij = s^(i-j) (i >= j); with
    # s = 1/2 every entry and every partial sum is exact
    n, s = 12, 0.5
    l = np.eye(n) - s * np.eye(n, k=-1)
    ref = np.tril(np.fromfunction(lambda i, j: s ** (i - j), (n, n)))
    assert np.array_equal(core.trtri_tile(l), ref)


def test_trtri_diagonal_and_upper_zero():
    d = np.array([1.0, 2.0, 0.25, 8.0, 4.0])
    w = core.trtri_tile(np.diag(d))
    assert np.array_equal(w, np.diag(1.0 / d))


def test_trtri_integer_unit_lower_is_exact_inverse():
    # an integer unit lower-triangular matrix has an integer inverse; small
    # entries keep every partial sum exact
    g = np.random.default_rng(5)
    n = 10
    l = np.tril(g.integers(-1, 2, (n, n)).astype(np.float64), -1) + np.eye(n)
    w = core.trtri_tile(l)
    assert np.array_equal(w, np.round(w))
    assert np.array_equal(w @ l, np.eye(n))
    assert np.array_equal(l @ w, np.eye(n))


@pytest.mark.parametrize("nb", [1, 7, 48])
def test_trtri_matches_scipy(nb):
    l = np.linalg.cholesky(inputs.spd_uniform(nb, 3 * nb))
    w = core.trtri_tile(l)
    ref = sla.solve_triangular(l, np.eye(nb), lower=True)
    assert np.abs(w - ref).max() <= 64 * nb * U * np.abs(ref).max() * np.linalg.cond(l)
    assert np.abs(w @ l - np.eye(nb)).max() <= 64 * nb * U * np.linalg.cond(l)


@pytest.mark.parametrize("m,nb", [(1, 1), (6, 9), (40, 32)])
def test_trsm_inv_tile_is_product_with_inverse(m, nb):
    g = np.random.default_rng(m + 7 * nb)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb))
    x = g.standard_normal((m, nb))
    w = core.trtri_tile(l)
    got = core.trsm_inv_tile(w, x)
    assert np.allclose(got, x @ w.T, rtol=0, atol=4 * nb * U * (np.abs(x) @ np.abs(w).T).max())
    # the same operation as the substitution TRSM
    ref = core.trsm_tile(l, x)
    assert np.abs(got - ref).max() <= 64 * nb * U * np.abs(ref).max() * np.linalg.cond(l)
    # only the lower part of W is read
    wn = w.copy()
    wn[np.triu_indices(nb, 1)] = np.nan
    assert np.array_equal(core.trsm_inv_tile(wn, x), got)


def test_trsm_inv_tile_exact_on_dyadic_case():
    n, s = 8, 0.5
    l = np.eye(n) - s * np.eye(n, k=-1)
    x = np.random.default_rng(2).integers(-4, 5, (5, n)).astype(np.float64)
    got = core.trsm_inv_tile(core.trtri_tile(l), x)
    assert np.array_equal(got, core.trsm_tile(l, x))
    assert np.array_equal(got @ l.T, x)


@pytest.mark.parametrize("m,nn,kb", [(1, 1, 1), (7, 5, 3), (33, 17, 64)])
def test_gemm_tile_matches_numpy(m, nn, kb):
    g = np.random.default_rng(m + 7 * nn + 31 * kb)
    c, x, y = g.standard_normal((m, nn)), g.standard_normal((m, kb)), g.standard_normal((nn, kb))
    got = core.gemm_tile(c, x, y)
    ref = c - x @ y.T
    assert np.allclose(got, ref, rtol=0, atol=4 * kb * U * (1 + np.abs(x).max() * np.abs(y).max() * kb))


def test_gemm_tile_brute_force_order():
    """Brute force on a tiny tile: exactly one rounded product and one
    rounded subtraction per p, p increasing."""
    g = np.random.default_rng(3)
    c, x, y = g.standard_normal((3, 4)), g.standard_normal((3, 5)), g.standard_normal((4, 5))
    ref = c.copy()
    for i in range(3):
        for j in range(4):
            t = ref[i, j]
            for p in range(5):
                t = t - float(np.float64(x[i, p]) * np.float64(y[j, p]))
            ref[i, j] = t
    assert np.array_equal(core.gemm_tile(c, x, y), ref)


def test_syrk_tile_lower_only():
    g = np.random.default_rng(4)
    c, x = g.standard_normal((9, 9)), g.standard_normal((9, 6))
    got = core.syrk_tile(c, x)
    ref = c - x @ x.T
    low = np.tril_indices(9)
    up = np.triu_indices(9, 1)
    assert np.allclose(got[low], ref[low], atol=1e-13)
    assert np.array_equal(got[up], c[up])  # strictly upper never touched


@pytest.mark.parametrize("nb,r", [(1, 1), (6, 3), (50, 2)])
def test_solve_tiles_match_scipy(nb, r):
    g = np.random.default_rng(nb + r)
    l = np.linalg.cholesky(inputs.spd_uniform(nb, nb + 1))
    bm = g.standard_normal((nb, r))
    fw = core.trsm_left_tile(l, bm)
    assert np.allclose(fw, sla.solve_triangular(l, bm, lower=True), atol=1e-12)
    bw = core.trsm_left_t_tile(l, bm)
    assert np.allclose(bw, sla.solve_triangular(l.T, bm, lower=False), atol=1e-12)
    lk = g.standard_normal((nb + 3, nb))
    bi = g.standard_normal((nb + 3, r))
    assert np.allclose(core.gemm_rhs_n(bi, lk, bm), bi - lk @ bm, atol=1e-12)
    lki = g.standard_normal((nb, nb + 3))
    assert np.allclose(core.gemm_rhs_t(bi, lki, bm), bi - lki.T @ bm, atol=1e-12)


# ---------------------------------------------- tiled factor: definitions

@pytest.mark.parametrize("n", [1, 2, 13, 29])
def test_tiled_equals_unblocked_for_every_tile_size(n):
    """Every element sees the unblocked operation sequence, so the tiled
    factor is bit-identical to the textbook algorithm for all b in 1..n."""
    a = inputs.spd_normal(n, 100 + n, 0.05)
    ref, info = core.potrf_unblocked(a)
    assert info == 0
    for b in range(1, n + 1):
        got, info = core.potrf_tiled(a, b)
        assert info == 0
        assert np.array_equal(np.tril(got), np.tril(ref)), f"b={b}"


def test_tiled_equals_unblocked_ragged_large():
    n = 150
    a = inputs.spd_uniform(n, 7)
    ref, _ = core.potrf_unblocked(a)
    for b in (16, 37, 64, 100, 149):
        got, info = core.potrf_tiled(a, b)
        assert info == 0 and np.array_equal(np.tril(got), np.tril(ref))


@pytest.mark.parametrize("n,b", [(64, 16), (200, 48), (256, 128)])
def test_tiled_matches_lapack(n, b):
    a = inputs.spd_normal(n, n, 1e-2)
    got, info = core.potrf_tiled(a, b)
    assert info == 0
    ref = np.linalg.cholesky(a)
    err = np.linalg.norm(np.tril(got) - ref) / np.linalg.norm(ref)
    assert err < 10 * n * U * np.linalg.cond(a)
    assert core.backward_error_fro(a, got) < 1e-15 * n


def test_upper_triangle_untouched():
    a = inputs.spd_uniform(40, 1)
    a_marked = a.copy()
    a_marked[np.triu_indices(40, 1)] = np.nan  # strictly upper is never read
    got, info = core.potrf_tiled(a_marked, 16)
    assert info == 0
    assert np.all(np.isnan(got[np.triu_indices(40, 1)]))
    ref, _ = core.potrf_tiled(a, 16)
    assert np.array_equal(np.tril(got), np.tril(ref))


# ---------------------------------------------------------- closed forms

def test_min_matrix_gives_ones():
    n = 30
    idx = np.arange(1, n + 1, dtype=np.float64)
    a = np.minimum.outer(idx, idx)
    for b in (1, 4, 7, 30):
        got, info = core.potrf_tiled(a, b)
        assert info == 0
        assert np.array_equal(np.tril(got), np.tril(np.ones((n, n))))


def test_pascal_closed_form():
    n = 20
    a = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    want = np.array([[math.comb(i, j) for j in range(n)] for i in range(n)], dtype=np.float64)
    for b in (1, 3, 8, 20):
        got, info = core.potrf_tiled(a, b)
        assert info == 0
        assert np.array_equal(np.tril(got), want)


def test_identity_and_diagonal():
    n = 17
    got, info = core.potrf_tiled(np.eye(n), 5)
    assert info == 0 and np.array_equal(np.tril(got), np.eye(n))
    d = np.arange(1, n + 1, dtype=np.float64)
    got, info = core.potrf_tiled(np.diag(d * d), 4)
    assert info == 0 and np.array_equal(np.tril(got), np.diag(d))


def test_two_by_two_formula():
    a = np.array([[9.0, 6.0], [6.0, 20.0]])
    got, _ = core.potrf_tiled(a, 1)
    l11 = math.sqrt(9.0)
    l21 = 6.0 / l11
    l22 = math.sqrt(20.0 - l21 * l21)
    assert np.array_equal(np.tril(got), np.array([[l11, 0.0], [l21, l22]]))


def test_textbook_3x3_golden():
    path = os.path.join(GOLDEN, "textbook_3x3.txt")
    a, want = _read_golden_matrix(path, "A"), _read_golden_matrix(path, "L")
    for b in (1, 2, 3):
        got, info = core.potrf_tiled(a, b)
        assert info == 0 and np.array_equal(np.tril(got), want)


@pytest.mark.parametrize("n,b", [(16, 4), (45, 8), (128, 32), (97, 96)])
def test_integer_factor_uniqueness_bitwise(n, b):
    """A = L0 L0^T with positive integer diagonal returns L0 exactly."""
    a, l0 = inputs.integer_factor(n, n + b)
    got, info = core.potrf_tiled(a, b)
    assert info == 0
    assert np.array_equal(np.tril(got), l0)


def test_random_factor_uniqueness_bound():
    n = 120
    g = np.random.default_rng(5)
    l0 = np.tril(g.standard_normal((n, n)), -1) / np.sqrt(n) + np.diag(1.0 + g.uniform(0, 1, n))
    a = l0 @ l0.T
    a = np.tril(a) + np.tril(a, -1).T
    got, info = core.potrf_tiled(a, 32)
    assert info == 0
    kappa = np.linalg.cond(a)
    assert np.linalg.norm(np.tril(got) - l0) / np.linalg.norm(l0) < 10 * kappa * U


# ----------------------------------------------------------- breakdown

def test_breakdown_info_column():
    a, _ = inputs.integer_factor(20, 9)
    a2 = a.copy()
    # make the pivot of column 11 (0-based) negative: subtract more than it has
    a2[11, 11] -= 1e6
    for b in (1, 4, 5, 20):
        _, info = core.potrf_tiled(a2, b)
        assert info == 12
    _, info = core.potrf_unblocked(a2)
    assert info == 12
    a3 = a.copy()
    a3[0, 0] = 0.0
    assert core.potrf_tiled(a3, 7)[1] == 1
    a4 = a.copy()
    a4[5, 5] = np.nan
    assert core.potrf_tiled(a4, 3)[1] == 6


# ---------------------------------------------------------------- solve

@pytest.mark.parametrize("n,r", [(1, 1), (23, 3), (64, 1)])
def test_tiled_solve_equals_unblocked(n, r):
    a = inputs.spd_normal(n, n, 0.1)
    l = np.tril(core.potrf_tiled(a, n)[0])
    bm = inputs.rhs(n, r, n)
    ref = core.potrs_unblocked(l, bm)
    for b in range(1, n + 1, max(1, n // 9)):
        assert np.array_equal(core.potrs_tiled(l, bm, b), ref), f"b={b}"


def test_solve_integer_exact():
    n, r = 60, 3
    a, l0 = inputs.integer_factor(n, 2, diag_choices=(1.0, 2.0, 4.0))
    x0 = inputs.integer_solution(n, r, 3)
    bm = a @ x0  # integers well below 2^53: exact
    l, info = core.potrf_tiled(a, 16)
    assert info == 0
    assert np.array_equal(core.potrs_tiled(np.tril(l), bm, 16), x0)


def test_solve_matches_scipy():
    n = 90
    a = inputs.spd_uniform(n, 11)
    bm = inputs.rhs(n, 4, 12)
    l = np.tril(core.potrf_tiled(a, 32)[0])
    x = core.potrs_tiled(l, bm, 32)
    ref = sla.cho_solve((np.linalg.cholesky(a), True), bm)
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------ DAG (Section 2)

@pytest.mark.parametrize("t", [1, 2, 4, 7])
def test_dag_closed_forms(t):
    tasks = dag.cholesky_tasks(t)
    kinds = [k for k, _, _ in tasks]
    assert kinds.count(dag.POTRF) == t
    assert kinds.count(dag.TRSM) == t * (t - 1) // 2
    assert kinds.count(dag.SYRK) == t * (t - 1) // 2
    assert kinds.count(dag.GEMM) == t * (t - 1) * (t - 2) // 6
    preds, succs, war = dag.infer_dag(tasks)
    assert not war  # the factor DAG has no write-after-read edge
    for (kind, (i, j, k), _), p in zip(tasks, preds):
        want = {dag.POTRF: 0, dag.TRSM: 1, dag.SYRK: 1, dag.GEMM: 2}[kind] + (k > 0)
        if kind == dag.POTRF:
            want = 1 if i > 0 else 0
        assert len(p) == want, (kind, i, j, k)
    assert dag.critical_path_length(preds) == 3 * t - 2


def test_dag_t4_has_20_tasks():
    assert len(dag.cholesky_tasks(4)) == 20


def test_dag_t2_by_hand():
    tasks = dag.cholesky_tasks(2)
    # POTRF(0) -> TRSM(1,0) -> SYRK(1,0) -> POTRF(1)
    assert [(k, c) for k, c, _ in tasks] == [
        (dag.POTRF, (0, 0, 0)), (dag.TRSM, (1, 0, 0)), (dag.SYRK, (1, 0, 0)), (dag.POTRF, (1, 0, 0))]
    preds, _, _ = dag.infer_dag(tasks)
    assert preds == [set(), {0}, {1}, {2}]


def test_dag_mode_rules_on_synthetic_tasks():
    x, y = ("x",), ("y",)
    tasks = [
        (0, (0, 0, 0), [(x, dag.W)]),             # 0 writes x
        (0, (0, 0, 0), [(x, dag.R)]),             # 1 RAW on 0
        (0, (0, 0, 0), [(x, dag.R), (y, dag.W)]),  # 2 RAW on 0
        (0, (0, 0, 0), [(x, dag.RW)]),            # 3 WAW on 0, WAR on 1 and 2
        (0, (0, 0, 0), [(y, dag.R)]),             # 4 RAW on 2
        (0, (0, 0, 0), [(x, dag.W)]),             # 5 WAW on 3
    ]
    preds, _, war = dag.infer_dag(tasks)
    assert preds == [set(), {0}, {0}, {0, 1, 2}, {2}, {3}]
    assert war == {(1, 3), (2, 3)}


def test_solve_dag_has_war_edges():
    _, _, war = dag.infer_dag(dag.solve_tasks(4))
    assert war


@pytest.mark.parametrize("n,b", [(40, 8), (37, 10)])
def test_random_topological_orders_bitwise(n, b):
    """Any order allowed by the access-mode graph gives the sequential
    (submission-order) result, bit for bit: the factor and the solve."""
    t = -(-n // b)
    a = inputs.spd_normal(n, 77, 0.05)
    bm0 = inputs.rhs(n, 2, 78)
    seq = a.copy()
    for kind, (i, j, k), _ in dag.cholesky_tasks(t):
        assert core.run_task(kind, seq, b, i, j, k) == 0
    seq_b = bm0.copy()
    for kind, (i, j, k), _ in dag.solve_tasks(t):
        core.run_task(kind, seq, b, i, j, k, bm=seq_b)
    ft, st = dag.cholesky_tasks(t), dag.solve_tasks(t)
    fp, fs, _ = dag.infer_dag(ft)
    sp, ss, _ = dag.infer_dag(st)
    for seed in range(20):
        g = dag.make_rng(seed)
        order = dag.random_topological_order(fp, fs, g)
        assert dag.is_valid_order(order, fp)
        m = a.copy()
        for idx in order:
            kind, (i, j, k), _ = ft[idx]
            core.run_task(kind, m, b, i, j, k)
        assert np.array_equal(np.tril(m), np.tril(seq))
        bm = bm0.copy()
        for idx in dag.random_topological_order(sp, ss, g):
            kind, (i, j, k), _ = st[idx]
            core.run_task(kind, m, b, i, j, k, bm=bm)
        assert np.array_equal(bm, seq_b)


def test_submission_order_solve_equals_potrs():
    n, b = 33, 8
    a = inputs.spd_uniform(n, 1)
    l, _ = core.potrf_tiled(a, b)
    bm = inputs.rhs(n, 2, 2)
    m = l.copy()
    x = bm.copy()
    for kind, (i, j, k), _ in dag.solve_tasks(-(-n // b)):
        core.run_task(kind, m, b, i, j, k, bm=x)
    assert np.array_equal(x, core.potrs_tiled(np.tril(l), bm, b))


# -------------------------------------------------------------- checkers

def test_backward_error_exact_zero_for_integer_case():
    a, l0 = inputs.integer_factor(50, 1)
    assert core.backward_error_fro(a, l0) == 0.0


def test_backward_error_known_perturbation():
    a, l0 = inputs.integer_factor(30, 2)
    e = np.zeros_like(a)
    e[3, 1] = e[1, 3] = 0.5
    e[7, 7] = -0.25
    got = core.backward_error_fro(a + e, l0)
    want = np.linalg.norm(e) / np.linalg.norm(a + e)
    assert abs(got - want) < 1e-15 * want
    z = np.random.default_rng(0).standard_normal((30, 8))
    est = core.backward_error_est(a + e, l0, z)
    az = (a + e) @ z
    assert abs(est - np.linalg.norm(e @ z) / np.linalg.norm(az)) < 1e-12 * est


def test_sampled_residual_and_residual_ld():
    a, l0 = inputs.integer_factor(25, 3)
    rows = np.array([0, 5, 24, 10])
    cols = np.array([0, 2, 24, 17])
    assert np.array_equal(core.sampled_residual(a, l0, rows, cols), np.zeros(4))
    x0 = inputs.integer_solution(25, 2, 4)
    bm = a @ x0
    assert np.array_equal(core.residual_ld(a, x0, bm), np.zeros((25, 2)))
    assert np.array_equal(core.residual_f64(a, x0, bm), np.zeros((25, 2)))


def test_sampled_residual_planted_perturbations():
    """A = L0 L0^T + E with integer L0 and dyadic E: every sampled entry of
    A - L L^T is E_ij exactly (both index orders), and a dyadic change d of
    one factor entry L_{i0,p0} shows up exactly where it must: at
    (i0, i0) as -(2 d L0[i0,p0] + d^2), at (i0, j) and (j, i0) for j >= p0 as
    -d L0[j,p0], and nowhere else."""
    n = 40
    a, l0 = inputs.integer_factor(n, 5)
    e = np.zeros_like(a)
    pts = [(3, 1, 0.5), (17, 17, -0.25), (39, 0, 2.0), (25, 24, 1.75), (10, 9, -3.0)]
    for i, j, v in pts:
        e[i, j] = e[j, i] = v
    rows = np.array([i for i, _, _ in pts] + [j for _, j, _ in pts] + [10, 39, 5])
    cols = np.array([j for _, j, _ in pts] + [i for i, _, _ in pts] + [5, 38, 30])
    got = core.sampled_residual(a + e, l0, rows, cols)
    assert np.array_equal(got, np.array([e[r, c] for r, c in zip(rows, cols)]))

    d, i0, p0 = 0.5, 20, 7
    l = l0.copy()
    l[i0, p0] += d
    rows2 = np.array([20, 20, 30, 7, 20, 6, 20, 33])
    cols2 = np.array([20, 7, 20, 20, 6, 20, 12, 31])
    want = []
    for r, c in zip(rows2, cols2):
        if r == i0 and c == i0:
            want.append(-(2 * d * l0[i0, p0] + d * d))
        elif i0 in (r, c):
            j = c if r == i0 else r
            want.append(-d * l0[j, p0] if j >= p0 else 0.0)
        else:
            want.append(0.0)
    got2 = core.sampled_residual(a, l, rows2, cols2)
    assert np.array_equal(got2, np.array(want))
    assert np.count_nonzero(want) == 5


# -------------------------------------------------- mixed precision, IR

def test_round_bf16_ties_to_even_against_torch():
    import torch
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 3.14159, 1e-3, -7.5e4,
                     0.0, 2 ** -130], dtype=np.float32)
    assert mixed.round_bf16(np.array([1 + 2 ** -8], dtype=np.float32))[0] == 1.0
    assert mixed.round_bf16(np.array([1 + 3 * 2 ** -8], dtype=np.float32))[0] == 1 + 2 ** -6
    g = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    for v in (vals, g):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
        assert np.array_equal(mixed.round_bf16(v), want)


@pytest.mark.parametrize("upd", ["f32", "bf16"])
def test_mixed_factor_integer_exact(upd):
    a, l0 = inputs.integer_factor(96, 8)
    l, info = mixed.mixed_factor(a, 32, upd)
    assert info == 0
    assert np.array_equal(l, l0)


def test_mixed_factor_error_size():
    n = 256
    a = inputs.spd_normal(n, 1, 1e-2)
    l32, info = mixed.mixed_factor(a, 64, "f32")
    assert info == 0
    eta = core.backward_error_fro(a, l32)
    assert 1e-9 < eta < 64 * n * 2.0 ** -24  # FP32-sized, not FP64-sized
    l16, info = mixed.mixed_factor(a, 64, "bf16")
    assert info == 0
    assert core.backward_error_fro(a, l16) > eta


def test_refine_integer_stops_at_zero():
    a, _ = inputs.integer_factor(40, 4, diag_choices=(1.0, 2.0))
    x0 = inputs.integer_solution(40, 2, 5)
    bm = a @ x0
    l = np.tril(core.potrf_tiled(a, 8)[0])
    x, it, status = mixed.refine(a, bm, l, 8)
    assert status == "converged" and it == 0 and np.array_equal(x, x0)


def test_refine_mixed_reaches_reference():
    n = 200
    gram = inputs.normal_gram(n, 21)
    a = gram + inputs.delta_for_cond(gram, 1e4) * np.eye(n)
    bm = inputs.rhs(n, 1, 22)
    xref = mixed.reference_solution(a, bm, 64)
    l, _ = mixed.mixed_factor(a, 64, "f32")
    x, it, status = mixed.refine(a, bm, l, 64)
    assert status in ("converged", "stagnated")
    err = np.abs(x - xref).max() / np.abs(xref).max()
    assert err < 1e-10
    # the reference itself: long-double residual is tiny relative to b
    r = core.residual_ld(a, xref, bm)
    assert np.abs(r).max() <= 4 * U * (np.abs(a).sum(1).max() * np.abs(xref).max())


def test_refine_stops_on_predicted_contraction():
    """Closed form: with the factor c L of c^2 A (L the FP64 factor of A),
    refinement contracts by exactly rho = 1 - 1/c^2 per step, so
    ||d_k|| = rho^(k+1) ||x*|| / c^2.  With c = 1 + 2^-9 and tol = 1e-11
    the correction test alone is met first at k = 4 (rho^5 = 9e-13); the
    contraction estimate ||d_k||^2 / (||d_{k-1}|| - ||d_k||), which here
    equals the sum of the corrections still to come, is met at k = 3
    (2.3e-10 at k = 2), so the refinement ends after 3 steps with x within
    the estimate of x*."""
    n = 64
    a = inputs.spd_cond(n, 41, 10.0)
    bm = inputs.rhs(n, 2, 42)
    l = np.tril(core.potrf_tiled(a, 16)[0])
    c = 1.0 + 2.0 ** -9
    rho = 1.0 - 1.0 / (c * c)
    x, it, status = mixed.refine(a, bm, c * l, 16, tol=1e-11)
    assert status == "converged" and it == 3
    xref = mixed.reference_solution(a, bm, 16)
    err = np.abs(x - xref).max(axis=0) / np.abs(xref).max(axis=0)
    assert np.all(err <= 2 * rho ** 5 / (1 - rho)) and np.all(err > 1e-14)
    # rho = 0.4 (c^2 = 5/3), tol = 5.1e-4: the estimate rho^(k+2) ||x*|| is
    # first met at k = 7 (rho^8 = 6.6e-4 at k = 6); without its 1 / (1 - rho)
    # it would be met at k = 6 (0.6 rho^8 = 3.9e-4)
    x, it, status = mixed.refine(a, bm, np.sqrt(5.0 / 3.0) * l, 16, tol=5.1e-4)
    assert status == "converged" and it == 7


def test_delta_for_cond_hits_target():
    gram = inputs.normal_gram(300, 5)
    for kappa in (1e2, 1e4, 1e6):
        a = gram + inputs.delta_for_cond(gram, kappa) * np.eye(300)
        assert abs(np.linalg.cond(a) / kappa - 1) < 1e-6


# ------------------------------------------ the paper's worked example

def test_scale_vector_golden():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "scale_vector.txt"))
             if l.strip() and not l.startswith("#")]
    factor = float(lines[0][1])
    xs = np.array([float(v[0]) for v in lines[1:]], dtype=np.float32)
    want = np.array([float(v[1]) for v in lines[1:]], dtype=np.float64)
    got = core.scale_vector(xs, factor).astype(np.float64)
    assert np.array_equal(got, want)


def test_oracle_threads_do_not_change_results():
    """OpenMP only splits independent rows: results are thread-count-free."""
    import subprocess
    import sys
    code = ("import numpy as np, oracle; from paper_1304_0878_amd import inputs;"
            "a=inputs.spd_normal(300,3,0.01); l,_=oracle.core.potrf_tiled(a,64);"
            "import hashlib; print(hashlib.sha256(np.tril(l).tobytes()).hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for th in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=th, PYTHONPATH=root)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, cwd=root,
                                   capture_output=True, text=True, check=True).stdout)
    assert outs[0] == outs[1]


def test_refine_cond_1e6_reaches_reference():
    """With the extended-precision residual, refinement at cond 1e6 ends on
    the correction test and reaches the long-double-refined reference far
    inside 1e-10 (a plainly accumulated FP64 residual stalls near
    cond * u = 1.1e-10 and does not)."""
    n = 300
    a = inputs.spd_cond(n, 31, 1e6)
    bm = inputs.rhs(n, 2, 32)
    xref = mixed.reference_solution(a, bm, 64)
    for upd in ("f32", "f64"):
        l, _ = mixed.mixed_factor(a, 64, upd)
        x, it, status = mixed.refine(a, bm, l, 64)
        assert status == "converged", (upd, it, status)
        assert np.abs(x - xref).max() / np.abs(xref).max() <= 1e-12


def test_refine_bf16_factor_at_cond_1e6_does_not_converge():
    """A BF16-update factor at cond 1e6 is too poor for refinement to
    contract (cond * u_bf16 >> 1): the oracle reports it unconverged, which
    is what triggers the fallback to a wider precision."""
    n = 200
    a = inputs.spd_cond(n, 33, 1e6)
    bm = inputs.rhs(n, 1, 34)
    l, info = mixed.mixed_factor(a, 64, "bf16")
    if info:
        return   # breakdown also triggers the fallback
    _, _, status = mixed.refine(a, bm, l, 64, maxit=10)
    assert status != "converged"
