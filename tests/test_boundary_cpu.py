"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-side graph building (a host-only runtime) matches the oracle's
access-mode inference and the closed forms.  No GPU work is issued."""
import os
import re
import ctypes

import pytest

from oracle import dag as odag

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dc():
    from paper_1304_0878_amd import dagchol
    return dagchol


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(dc_[a-z0-9_]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol(dc):
    lib = ctypes.CDLL(dc.LIB_PATH)
    names = _declared()
    assert len(names) > 20
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names <= set(dc.EXPORTED) | set(), names - set(dc.EXPORTED)


def _host_rt(dc):
    return dc.Runtime(device=-1)


FAKE = 0x10000


def _tiles(dc, rt, n, tile, ptr=FAKE):
    a = rt.dc_matrix_register(ptr, n, n, n, dc.DC_F64)
    return a, rt.dc_matrix_partition(a, tile)


def _submit_cholesky(dc, rt, tiles):
    T = len(tiles)
    for k in range(T):
        rt.dc_task_submit(dc.DC_POTRF, [tiles[k][k]], [dc.DC_RW])
        for i in range(k + 1, T):
            rt.dc_task_submit(dc.DC_TRSM, [tiles[k][k], tiles[i][k]], [dc.DC_R, dc.DC_RW])
        for i in range(k + 1, T):
            rt.dc_task_submit(dc.DC_SYRK, [tiles[i][k], tiles[i][i]], [dc.DC_R, dc.DC_RW])
            for j in range(k + 1, i):
                rt.dc_task_submit(dc.DC_GEMM, [tiles[i][k], tiles[j][k], tiles[i][j]],
                                  [dc.DC_R, dc.DC_R, dc.DC_RW])


@pytest.mark.parametrize("n,tile", [(512, 128), (1000, 128), (8192, 512), (300, 7)])
def test_factor_graph_matches_oracle(dc, n, tile):
    with _host_rt(dc) as rt:
        _, tiles = _tiles(dc, rt, n, tile)
        T = len(tiles)
        _submit_cholesky(dc, rt, tiles)
        st = rt.dc_graph_stats_get()
        assert st["ntasks"] == T + T * (T - 1) + T * (T - 1) * (T - 2) // 6
        assert st["critical_path"] == 3 * T - 2
        assert st["nwar_edges"] == 0
        if T <= 40:
            preds, _, _ = odag.infer_dag(odag.cholesky_tasks(T))
            for t in range(st["ntasks"]):
                assert rt.dc_graph_preds(t) == sorted(preds[t])
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_wait_all()
        assert e.value.code == -19  # host-only: -ENODEV


def test_solve_graph_matches_oracle(dc):
    n, tile, T = 640, 128, 5
    with _host_rt(dc) as rt:
        _, L = _tiles(dc, rt, n, tile)
        b = rt.dc_matrix_register(FAKE * 7, n, 2, 2, dc.DC_F64)
        B = [row[0] for row in rt.dc_matrix_partition(b, tile)]
        tasks = odag.solve_tasks(T)
        for kind, (i, j, k), _ in tasks:
            if kind == odag.TRSM_L:
                rt.dc_task_submit(dc.DC_TRSM_L, [L[i][i], B[i]], [dc.DC_R, dc.DC_RW])
            elif kind == odag.TRSM_LT:
                rt.dc_task_submit(dc.DC_TRSM_LT, [L[i][i], B[i]], [dc.DC_R, dc.DC_RW])
            elif kind == odag.GEMM_RHS_N:
                rt.dc_task_submit(dc.DC_GEMM_RHS_N, [L[i][k], B[k], B[i]],
                                  [dc.DC_R, dc.DC_R, dc.DC_RW])
            else:
                rt.dc_task_submit(dc.DC_GEMM_RHS_T, [L[k][i], B[k], B[i]],
                                  [dc.DC_R, dc.DC_R, dc.DC_RW])
        preds, _, war = odag.infer_dag(tasks)
        st = rt.dc_graph_stats_get()
        assert st["nwar_edges"] > 0 and war
        for t in range(len(tasks)):
            assert rt.dc_graph_preds(t) == sorted(preds[t])


def test_mode_rules_synthetic(dc):
    with _host_rt(dc) as rt:
        x = rt.dc_matrix_register(FAKE, 4, 4, 4, dc.DC_F64)
        y = rt.dc_matrix_register(FAKE * 2, 4, 4, 4, dc.DC_F64)
        z = rt.dc_matrix_register(FAKE * 3, 4, 4, 4, dc.DC_F64)
        R, RW = dc.DC_R, dc.DC_RW
        # TRSM (L:R, X:RW) used as a generic (read one, write one) task
        rt.dc_task_submit(dc.DC_TRSM, [y, x], [R, RW])   # 0 writes x
        rt.dc_task_submit(dc.DC_TRSM, [x, y], [R, RW])   # 1 reads x (RAW 0), writes y (WAR 0)
        rt.dc_task_submit(dc.DC_TRSM, [x, z], [R, RW])   # 2 reads x (RAW 0)
        rt.dc_task_submit(dc.DC_TRSM, [z, x], [R, RW])   # 3 writes x: WAW 0, WAR 1, 2; RAW z 2
        assert rt.dc_graph_preds(0) == []
        assert rt.dc_graph_preds(1) == [0]
        assert rt.dc_graph_preds(2) == [0]
        assert rt.dc_graph_preds(3) == [0, 1, 2]


def test_error_codes(dc):
    with _host_rt(dc) as rt:
        a = rt.dc_matrix_register(FAKE, 64, 64, 64, dc.DC_F64)
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_matrix_register(FAKE, 8, 8, 8, dc.DC_F64)
        assert e.value.code == -16  # -EBUSY: pointer already registered
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_task_submit(dc.DC_POTRF, [999], [dc.DC_RW])
        assert e.value.code == -2   # -ENOENT
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_task_submit(dc.DC_POTRF, [a], [dc.DC_R])
        assert e.value.code == -22  # mode does not match the signature
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_task_submit(dc.DC_GEMM, [a, a], [dc.DC_R, dc.DC_RW])
        assert e.value.code == -22  # arity
        tiles = rt.dc_matrix_partition(a, 16)
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_task_submit(dc.DC_POTRF, [a], [dc.DC_RW])
        assert e.value.code == -16  # parent used while partitioned
        assert rt.dc_handle_lookup(FAKE) == a
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_handle_lookup(FAKE + 8)
        assert e.value.code == -2
        rt.dc_matrix_unpartition(a)
        rt.dc_unregister(a)
        with pytest.raises(dc.DagcholError):
            rt.dc_task_submit(dc.DC_POTRF, [a], [dc.DC_RW])
        b = rt.dc_matrix_register(FAKE * 5, 10, 10, 10, dc.DC_BF16)
        with pytest.raises(dc.DagcholError) as e:
            rt.dc_task_submit(dc.DC_POTRF, [b], [dc.DC_RW])
        assert e.value.code == -22  # POTRF needs FP64 or FP32 storage


def test_lookahead_config(dc):
    """The lookahead depth defaults to 48 levels, 0 is accepted (every task
    at its earliest level), a negative depth is rejected."""
    cfg = dc.dc_config()
    dc._lib.dc_config_default(dc.ctypes.byref(cfg))
    assert cfg.lookahead == 48
    for depth in (0, 3):
        with dc.Runtime(device=-1, lookahead=depth):
            pass
    with pytest.raises(dc.DagcholError) as e:
        dc.Runtime(device=-1, lookahead=-1)
    assert e.value.code == -22


def test_ragged_partition_shapes(dc):
    with _host_rt(dc) as rt:
        a = rt.dc_matrix_register(FAKE, 1000, 1000, 1024, dc.DC_F64)
        tiles = rt.dc_matrix_partition(a, 384)
        assert len(tiles) == 3 and len(tiles[0]) == 3
        # a TRSM between the ragged tile (232 rows) and a full diagonal tile
        rt.dc_task_submit(dc.DC_TRSM, [tiles[0][0], tiles[2][0]], [dc.DC_R, dc.DC_RW])
        # shape mismatch: a 384-wide diagonal tile against a ragged 232-wide one
        with pytest.raises(dc.DagcholError):
            rt.dc_task_submit(dc.DC_TRSM, [tiles[2][2], tiles[2][0]], [dc.DC_R, dc.DC_RW])
        st = rt.dc_graph_stats_get()
        assert st["ntasks"] == 1 and st["nunits"] == -(-232 // 16)


def test_strerror(dc):
    assert "unregistered" in dc.dc_strerror(-2)
    assert dc.dc_strerror(0) == "success"


def test_server_config_validation(dc):
    """dc_server_create checks its configuration before touching a device:
    defaults, then each out-of-range field rejected with -EINVAL."""
    lib = dc._lib
    cfg = dc.dc_server_config()
    lib.dc_server_config_default(ctypes.byref(cfg))
    assert (cfg.slots, cfg.tile, cfg.whole_max, cfg.upd, cfg.maxit) == (4, 256, 512, dc.DC_F32, 30)
    assert cfg.tol == 1e-12 and cfg.pool_bytes == 64 << 30
    assert (cfg.tile_large, cfg.large_min, cfg.mixed_min) == (512, 4096, 0)
    for field, bad in (("whole_max", 513), ("whole_max", -1), ("tile", 0), ("tile", 513),
                       ("slots", 0), ("slots", 65), ("tol", 0.0), ("maxit", -1), ("upd", 7),
                       ("pool_bytes", 0), ("tile_large", 0), ("tile_large", 513),
                       ("large_min", -1), ("mixed_min", -1)):
        c = dc.dc_server_config()
        lib.dc_server_config_default(ctypes.byref(c))
        setattr(c, field, bad)
        out = ctypes.c_void_p()
        assert lib.dc_server_create(ctypes.byref(out), ctypes.byref(c)) == -22, (field, bad)
        assert not out.value
