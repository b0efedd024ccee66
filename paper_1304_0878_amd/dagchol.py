"""Thin Python binding of the dagchol C ABI (include/dagchol.h).

Argument marshalling only: every operation runs in the HIP library
``libdagchol.so``.  If the library is missing this module raises on import;
there is no fallback.  PyTorch provides device memory and the stream.
"""
import ctypes
import os

# PyTorch is imported first so that the library binds to the HIP runtime
# PyTorch already loaded (one HIP runtime per process: two copies would each
# try to own the device).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdagchol.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1304_0878_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ C types

dc_handle = ctypes.c_int64
DC_R, DC_W, DC_RW = 1, 2, 3
DC_F64, DC_F32, DC_BF16 = 0, 1, 2
DC_EXEC_LEVELS, DC_EXEC_QUEUE = 0, 1
(DC_POTRF, DC_TRSM, DC_SYRK, DC_GEMM, DC_TRSM_L, DC_GEMM_RHS_N, DC_TRSM_LT, DC_GEMM_RHS_T,
 DC_SCAL, DC_CAST, DC_RESID, DC_AXPY, DC_TRSM_CAST, DC_TRTRI, DC_TRSM_INV,
 DC_TRSM_INV_CAST, DC_TRSM_L_INV, DC_TRSM_LT_INV) = range(18)

ERRNO = {22: "EINVAL", 2: "ENOENT", 16: "EBUSY", 12: "ENOMEM", 19: "ENODEV", 110: "ETIMEDOUT",
         5: "EIO", 38: "ENOSYS"}


class dc_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("workers", ctypes.c_int),
                ("watchdog_ms", ctypes.c_int64), ("trace", ctypes.c_int),
                ("executor", ctypes.c_int), ("lookahead", ctypes.c_int)]


class dc_graph_stats(ctypes.Structure):
    _fields_ = [("ntasks", ctypes.c_int64), ("nedges", ctypes.c_int64),
                ("nwar_edges", ctypes.c_int64), ("critical_path", ctypes.c_int64),
                ("nunits", ctypes.c_int64)]


class dc_ir_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("final_prec", ctypes.c_int), ("fallbacks", ctypes.c_int),
                ("last_update", ctypes.c_double), ("factor_ms", ctypes.c_double),
                ("refine_ms", ctypes.c_double)]


class dc_kernel_stat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class dc_kernel_stats(ctypes.Structure):
    _fields_ = [("panel", dc_kernel_stat), ("gemm", dc_kernel_stat)]


class dc_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("slots", ctypes.c_int), ("pool_bytes", ctypes.c_size_t),
                ("tile", ctypes.c_int64), ("upd", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("whole_max", ctypes.c_int64),
                ("mixed_min", ctypes.c_int64), ("tile_large", ctypes.c_int64),
                ("large_min", ctypes.c_int64)]


class dc_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("r", ctypes.c_int64), ("A", ctypes.c_void_p),
                ("B", ctypes.c_void_p), ("X", ctypes.c_void_p), ("arrival", ctypes.c_double)]


class dc_request_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("info", ctypes.c_int64),
                ("converged", ctypes.c_int), ("iterations", ctypes.c_int),
                ("final_prec", ctypes.c_int), ("restarts", ctypes.c_int),
                ("last_update", ctypes.c_double), ("arrival", ctypes.c_double),
                ("admitted", ctypes.c_double), ("completed", ctypes.c_double)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_H = dc_handle
_PH = ctypes.POINTER(dc_handle)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "dc_config_default": (None, [ctypes.POINTER(dc_config)]),
    "dc_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(dc_config)]),
    "dc_shutdown": (ctypes.c_int, [_P]),
    "dc_vector_register": (ctypes.c_int, [_P, _PH, _P, _I64, ctypes.c_int]),
    "dc_matrix_register": (ctypes.c_int, [_P, _PH, _P, _I64, _I64, _I64, ctypes.c_int]),
    "dc_matrix_partition": (ctypes.c_int, [_P, _H, _I64, _PH]),
    "dc_matrix_unpartition": (ctypes.c_int, [_P, _H]),
    "dc_matrix_tiles": (ctypes.c_int, [_P, _H, _PI64, _PI64]),
    "dc_handle_lookup": (ctypes.c_int, [_P, _P, _PH]),
    "dc_task_submit": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _PH,
                                      ctypes.POINTER(ctypes.c_int), _P, ctypes.c_size_t,
                                      ctypes.c_int]),
    "dc_flush": (ctypes.c_int, [_P]),
    "dc_wait_all": (ctypes.c_int, [_P]),
    "dc_acquire": (ctypes.c_int, [_P, _H, ctypes.c_int]),
    "dc_release": (ctypes.c_int, [_P, _H]),
    "dc_unregister": (ctypes.c_int, [_P, _H]),
    "dc_get_info": (ctypes.c_int, [_P, _H, _PI64]),
    "dc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dc_last_error": (ctypes.c_char_p, []),
    "dc_selftest": (ctypes.c_int, [_P, _I64, _P]),
    "dc_graph_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(dc_graph_stats)]),
    "dc_graph_preds": (ctypes.c_int, [_P, _I64, _PI64, _I64, _PI64]),
    "dc_trace_get": (ctypes.c_int, [_P, _I64, _PI64, _PI64, _PI32, _PI32]),
    "dc_potrf": (ctypes.c_int, [_P, _H, _I64, ctypes.c_int]),
    "dc_potrs": (ctypes.c_int, [_P, _H, _H, _I64]),
    "dc_potrf_noalloc": (ctypes.c_int, [_P, _H, _I64]),
    "dc_posv_ir": (ctypes.c_int, [_P, _H, _H, _H, _I64, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.POINTER(dc_ir_report)]),
    "dc_last_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), _PI64, _PI32]),
    "dc_potrf_batched": (ctypes.c_int, [_P, _I64, _PH, _PH, _PI64, _PI64]),
    "dc_kernel_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "dc_kernel_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(dc_kernel_stats)]),
    "dc_server_config_default": (None, [ctypes.POINTER(dc_server_config)]),
    "dc_server_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(dc_server_config)]),
    "dc_server_destroy": (ctypes.c_int, [_P]),
    "dc_server_now": (ctypes.c_double, [_P]),
    "dc_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(dc_request), _PI64]),
    "dc_server_progress": (ctypes.c_int, [_P, ctypes.POINTER(dc_request_result), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int)]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_SIGS)


class DagcholError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.dc_strerror(code).decode()
        detail = _lib.dc_last_error().decode() if code == -5 else ""
        super().__init__(f"{where}: {msg} ({ERRNO.get(-code, code)}) {detail}".rstrip())


def _check(code, where):
    if code < 0:
        raise DagcholError(code, where)
    return code


def dc_strerror(code):
    return _lib.dc_strerror(code).decode()


# ------------------------------------------------------------------ runtime

def _dtype_code(t):
    import torch
    return {torch.float64: DC_F64, torch.float32: DC_F32, torch.bfloat16: DC_BF16}[t.dtype]


class Runtime:
    """One dc_runtime.  device=-1 makes a host-only runtime (graph building
    and inspection, no execution)."""

    def __init__(self, device=0, stream=None, workers=0, watchdog_ms=60000, trace=False,
                 executor=DC_EXEC_LEVELS, lookahead=None):
        cfg = dc_config()
        _lib.dc_config_default(ctypes.byref(cfg))
        cfg.device = device
        cfg.workers = workers
        cfg.watchdog_ms = watchdog_ms
        cfg.trace = 1 if trace else 0
        cfg.executor = executor
        if lookahead is not None:
            cfg.lookahead = lookahead
        if device >= 0:
            import torch
            s = stream if stream is not None else torch.cuda.current_stream(device)
            cfg.stream = ctypes.c_void_p(s.cuda_stream)
        self._ptr = ctypes.c_void_p()
        _check(_lib.dc_init(ctypes.byref(self._ptr), ctypes.byref(cfg)), "dc_init")

    # -- lifecycle
    def close(self):
        if self._ptr:
            code = _lib.dc_shutdown(self._ptr)
            self._ptr = ctypes.c_void_p()
            _check(code, "dc_shutdown")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._ptr:
                _lib.dc_shutdown(self._ptr)
        except Exception:
            pass

    # -- registration (the C calls of the same names)
    def dc_vector_register(self, ptr, nx, dtype):
        h = dc_handle()
        _check(_lib.dc_vector_register(self._ptr, ctypes.byref(h), ptr, nx, dtype),
               "dc_vector_register")
        return h.value

    def dc_matrix_register(self, ptr, rows, cols, ld, dtype):
        h = dc_handle()
        _check(_lib.dc_matrix_register(self._ptr, ctypes.byref(h), ptr, rows, cols, ld, dtype),
               "dc_matrix_register")
        return h.value

    def register_tensor(self, t):
        """Registers a CUDA tensor (1-D: vector, 2-D: row-major matrix)."""
        if t.dim() == 1:
            return self.dc_vector_register(t.data_ptr(), t.shape[0], _dtype_code(t))
        assert t.dim() == 2 and t.stride(1) == 1, "row-major 2-D tensor expected"
        return self.dc_matrix_register(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0),
                                       _dtype_code(t))

    def dc_matrix_partition(self, m, tile):
        tr = -(-self._rows(m) // tile)
        tc = -(-self._cols(m) // tile)
        arr = (dc_handle * (tr * tc))()
        _check(_lib.dc_matrix_partition(self._ptr, m, tile, arr), "dc_matrix_partition")
        return [[arr[i * tc + j] for j in range(tc)] for i in range(tr)]

    def _shape(self, m):
        self._shapes = getattr(self, "_shapes", {})
        return self._shapes[m]

    def _rows(self, m):
        return self._meta[m][0]

    def _cols(self, m):
        return self._meta[m][1]

    def dc_matrix_unpartition(self, m):
        _check(_lib.dc_matrix_unpartition(self._ptr, m), "dc_matrix_unpartition")

    def dc_handle_lookup(self, ptr):
        h = dc_handle()
        code = _lib.dc_handle_lookup(self._ptr, ptr, ctypes.byref(h))
        _check(code, "dc_handle_lookup")
        return h.value

    def dc_task_submit(self, kind, bufs, modes, cl_args=None, priority=0):
        n = len(bufs)
        hb = (dc_handle * n)(*bufs)
        mb = (ctypes.c_int * n)(*modes)
        if cl_args is None:
            p, size = None, 0
        else:
            buf = ctypes.create_string_buffer(bytes(cl_args), len(cl_args))
            p, size = ctypes.cast(buf, ctypes.c_void_p), len(cl_args)
        _check(_lib.dc_task_submit(self._ptr, kind, n, hb, mb, p, size, priority),
               "dc_task_submit")

    def dc_flush(self):
        _check(_lib.dc_flush(self._ptr), "dc_flush")

    def dc_wait_all(self):
        _check(_lib.dc_wait_all(self._ptr), "dc_wait_all")

    def dc_acquire(self, h, mode=DC_R):
        _check(_lib.dc_acquire(self._ptr, h, mode), "dc_acquire")

    def dc_release(self, h):
        _check(_lib.dc_release(self._ptr, h), "dc_release")

    def dc_unregister(self, h):
        _check(_lib.dc_unregister(self._ptr, h), "dc_unregister")

    def dc_get_info(self, h):
        v = ctypes.c_int64()
        _check(_lib.dc_get_info(self._ptr, h, ctypes.byref(v)), "dc_get_info")
        return v.value

    def dc_graph_stats_get(self):
        s = dc_graph_stats()
        _check(_lib.dc_graph_stats_get(self._ptr, ctypes.byref(s)), "dc_graph_stats_get")
        return {f: getattr(s, f) for f, _ in dc_graph_stats._fields_}

    def dc_graph_preds(self, t):
        cnt = ctypes.c_int64()
        _check(_lib.dc_graph_preds(self._ptr, t, None, 0, ctypes.byref(cnt)), "dc_graph_preds")
        arr = (ctypes.c_int64 * max(cnt.value, 1))()
        _check(_lib.dc_graph_preds(self._ptr, t, arr, cnt.value, ctypes.byref(cnt)),
               "dc_graph_preds")
        return sorted(arr[i] for i in range(cnt.value))

    def dc_trace_get(self, t):
        s, e = ctypes.c_int64(), ctypes.c_int64()
        w, k = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.dc_trace_get(self._ptr, t, ctypes.byref(s), ctypes.byref(e), ctypes.byref(w),
                                 ctypes.byref(k)), "dc_trace_get")
        return s.value, e.value, w.value, k.value

    def dc_last_launch(self):
        b, u, w = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.dc_last_launch(self._ptr, ctypes.byref(b), ctypes.byref(u), ctypes.byref(w)),
               "dc_last_launch")
        return {"build_ms": b.value, "units": u.value, "workers": w.value}

    def dc_kernel_timing(self, enable=True):
        _check(_lib.dc_kernel_timing(self._ptr, 1 if enable else 0), "dc_kernel_timing")

    def dc_kernel_stats_get(self):
        st = dc_kernel_stats()
        _check(_lib.dc_kernel_stats_get(self._ptr, ctypes.byref(st)), "dc_kernel_stats_get")
        return {k: {f: getattr(getattr(st, k), f) for f, _ in dc_kernel_stat._fields_}
                for k in ("panel", "gemm")}

    # -- high level
    def dc_potrf(self, a, tile, upd=DC_F64):
        _check(_lib.dc_potrf(self._ptr, a, tile, upd), "dc_potrf")

    def dc_potrf_noalloc(self, a, tile):
        _check(_lib.dc_potrf_noalloc(self._ptr, a, tile), "dc_potrf_noalloc")

    def dc_potrs(self, l, b, tile):
        _check(_lib.dc_potrs(self._ptr, l, b, tile), "dc_potrs")

    def dc_potrf_batched(self, a_handles, b_handles, tiles):
        n = len(a_handles)
        ha = (dc_handle * max(n, 1))(*a_handles)
        hb = (dc_handle * max(n, 1))(*(b_handles or [0] * n))
        tl = (ctypes.c_int64 * max(n, 1))(*tiles)
        info = (ctypes.c_int64 * max(n, 1))()
        _check(_lib.dc_potrf_batched(self._ptr, n, ha, hb if b_handles is not None else None,
                                     tl, info), "dc_potrf_batched")
        return [info[i] for i in range(n)]

    def dc_posv_ir(self, a, b, x, tile, upd=DC_F32, tol=1e-12, maxit=30):
        rep = dc_ir_report()
        _check(_lib.dc_posv_ir(self._ptr, a, b, x, tile, upd, tol, maxit, ctypes.byref(rep)),
               "dc_posv_ir")
        return {f: getattr(rep, f) for f, _ in dc_ir_report._fields_}


# The shapes of registered handles are kept on the Python side only for
# dc_matrix_partition's output sizing.
def _track_meta():
    orig_m = Runtime.dc_matrix_register
    orig_v = Runtime.dc_vector_register

    def mreg(self, ptr, rows, cols, ld, dtype):
        h = orig_m(self, ptr, rows, cols, ld, dtype)
        self._meta = getattr(self, "_meta", {})
        self._meta[h] = (rows, cols)
        return h

    def vreg(self, ptr, nx, dtype):
        h = orig_v(self, ptr, nx, dtype)
        self._meta = getattr(self, "_meta", {})
        self._meta[h] = (nx, 1)
        return h

    Runtime.dc_matrix_register = mreg
    Runtime.dc_vector_register = vreg


_track_meta()


# ------------------------------------------------------ tensor-level helpers

def potrf(rt, a, tile, upd=DC_F64):
    """Factors the lower triangle of a CUDA float64 tensor in place (trailing
    updates at precision ``upd``); returns info."""
    h = rt.register_tensor(a)
    try:
        rt.dc_potrf(h, tile, upd)
        return rt.dc_get_info(h)
    finally:
        rt.dc_unregister(h)


def potrs(rt, l, b, tile):
    """Solves L L^T X = B in place in B (CUDA float64, n x r)."""
    hl = rt.register_tensor(l)
    hb = rt.register_tensor(b)
    try:
        rt.dc_potrs(hl, hb, tile)
    finally:
        rt.dc_unregister(hb)
        rt.dc_unregister(hl)


def posv_ir(rt, a, b, x, tile, upd=DC_F32, tol=1e-12, maxit=30):
    """Mixed-precision solve with FP64-residual refinement; x receives the solution."""
    ha, hb, hx = rt.register_tensor(a), rt.register_tensor(b), rt.register_tensor(x)
    try:
        return rt.dc_posv_ir(ha, hb, hx, tile, upd, tol, maxit)
    finally:
        for h in (hx, hb, ha):
            rt.dc_unregister(h)


def potrf_batched(rt, mats, rhs=None, tiles=None):
    """Factors every CUDA float64 or float32 matrix of ``mats`` in place (and
    solves the matching float64 ``rhs`` in place) in one graph; returns the
    per-matrix infos.  Float32 matrices are factored as one tile."""
    ha = [rt.register_tensor(m) for m in mats]
    hb = [rt.register_tensor(b) for b in rhs] if rhs is not None else None
    try:
        return rt.dc_potrf_batched(ha, hb, tiles if tiles is not None else [0] * len(mats))
    finally:
        for h in (hb or []) + ha:
            rt.dc_unregister(h)


# ------------------------------------------------------------------ serving

class Server:
    """Continuous-batching solve server (dc_server_*).  Tensors handed to
    submit() are kept alive here until their request completes."""

    def __init__(self, device=0, slots=4, pool_bytes=None, tile=256, upd=DC_F32, tol=1e-12,
                 maxit=30, whole_max=None, mixed_min=None, tile_large=None, large_min=None):
        cfg = dc_server_config()
        _lib.dc_server_config_default(ctypes.byref(cfg))
        cfg.device, cfg.slots, cfg.tile, cfg.upd = device, slots, tile, upd
        cfg.tol, cfg.maxit = tol, maxit
        if whole_max is not None:
            cfg.whole_max = whole_max
        if mixed_min is not None:
            cfg.mixed_min = mixed_min
        if tile_large is not None:
            cfg.tile_large = tile_large
        if large_min is not None:
            cfg.large_min = large_min
        if pool_bytes is not None:
            cfg.pool_bytes = pool_bytes
        p = _P()
        _check(_lib.dc_server_create(ctypes.byref(p), ctypes.byref(cfg)), "dc_server_create")
        self._ptr = p
        self._keep = {}
        self._res = (dc_request_result * 256)()

    def now(self):
        return _lib.dc_server_now(self._ptr)

    def submit(self, a, b, x, arrival=None):
        """A (n x n), B and X (n x r): contiguous CUDA float64 tensors whose
        values are complete when this is called (the server's slots run on
        their own streams: synchronise the producing stream first)."""
        for t in (a, b, x):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("server tensors must be contiguous CUDA float64")
        b2 = b if b.dim() == 2 else b.view(-1, 1)
        x2 = x if x.dim() == 2 else x.view(-1, 1)
        q = dc_request(n=a.shape[0], r=b2.shape[1], A=a.data_ptr(), B=b2.data_ptr(),
                       X=x2.data_ptr(), arrival=self.now() if arrival is None else arrival)
        rid = ctypes.c_int64()
        _check(_lib.dc_server_submit(self._ptr, ctypes.byref(q), ctypes.byref(rid)),
               "dc_server_submit")
        self._keep[rid.value] = (a, b, x)
        return rid.value

    def progress(self):
        """Returns (completed results as dicts, number still queued or running)."""
        nd, act = ctypes.c_int(), ctypes.c_int()
        _check(_lib.dc_server_progress(self._ptr, self._res, len(self._res), ctypes.byref(nd),
                                       ctypes.byref(act)), "dc_server_progress")
        out = []
        for i in range(nd.value):
            r = self._res[i]
            d = {f: getattr(r, f) for f, _ in dc_request_result._fields_}
            self._keep.pop(d["id"], None)
            out.append(d)
        return out, act.value

    def drain(self, sleep=0.0):
        import time
        done = []
        while True:
            got, act = self.progress()
            done += got
            if act == 0:
                return done
            if sleep:
                time.sleep(sleep)

    def close(self):
        if self._ptr:
            _check(_lib.dc_server_destroy(self._ptr), "dc_server_destroy")
            self._ptr = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
