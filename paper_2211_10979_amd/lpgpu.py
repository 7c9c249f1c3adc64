"""Python binding of liblpgpu (the C ABI in include/lpgpu.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. The functions keep the C names; arrays are numpy float64 / int32.

If PyTorch is importable it is imported before the library is loaded: torch
ships its own HIP runtime under the same soname, and loading it first makes
the process use a single runtime, so torch tensors can serve as device
buffers (`device_buffer=`) and torch streams as the solver stream.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: torch's, when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional
    torch = None

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblpgpu.so")

LP_OPTIMAL, LP_UNBOUNDED, LP_ITER_LIMIT, LP_NUMERICAL, LP_RUNNING, LP_STALLED, LP_INFEASIBLE = 0, 1, 2, 3, 4, 5, 6
STATUS_NAMES = {0: "OPTIMAL", 1: "UNBOUNDED", 2: "ITER_LIMIT", 3: "NUMERICAL", 4: "RUNNING", 5: "STALLED",
                6: "INFEASIBLE"}
LP_LE, LP_GE, LP_EQ = 0, 1, 2  # row senses of the general form
LP_OK, LP_E_INVAL, LP_E_NEG_RHS, LP_E_NOMEM, LP_E_DEVICE, LP_E_STATE, LP_E_PENDING, LP_E_BUDGET = 0, -1, -2, -3, -4, -5, -6, -7


class LPError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__(f"{func} failed with code {code}: {msg}")
        self.code = code


class lp_tuning(ctypes.Structure):
    """Execution and kernel-shape choices (none changes a result); all zero = automatic."""
    _fields_ = [
        ("chunk_pivots", ctypes.c_int32),
        ("cols_per_block", ctypes.c_int32),
        ("plain_launches", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32),
        ("batch_block", ctypes.c_int32),
        ("batch_unroll", ctypes.c_int32),
        ("update_hints", ctypes.c_int32),
        ("update_block", ctypes.c_int32),
        ("update_grid_stride", ctypes.c_int32),
        ("update_unroll", ctypes.c_int32),
        ("select_workgroups", ctypes.c_int32),
        ("fuse_pivots", ctypes.c_int32),
        ("decide_kernel", ctypes.c_int32),
        ("decide_spin", ctypes.c_int32),
        ("decide_block", ctypes.c_int32),
        ("eager_build", ctypes.c_int32),
        ("status_readback", ctypes.c_int32),
    ]


TUNING_FIELDS = frozenset(name for name, _ in lp_tuning._fields_)


class lp_options(ctypes.Structure):
    _fields_ = [
        ("eps_dual", ctypes.c_double),
        ("eps_pivot", ctypes.c_double),
        ("max_pivots", ctypes.c_int64),
        ("record_pivots", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("device_buffer", ctypes.c_void_p),
        ("device_buffer_bytes", ctypes.c_size_t),
        ("device", ctypes.c_int32),
        ("bland_after", ctypes.c_int32),
        ("tuning", ctypes.POINTER(lp_tuning)),
    ]


class lp_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pivots", ctypes.c_int64),
        ("objective", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
    ]


class lp_info(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("width", ctypes.c_int64),
        ("ld", ctypes.c_int64),
        ("tableau_bytes", ctypes.c_size_t),
        ("tableau", ctypes.c_void_p),
        ("update_block", ctypes.c_int32),
        ("update_cols", ctypes.c_int32),
        ("update_rows", ctypes.c_int32),
        ("update_hints", ctypes.c_int32),
        ("update_fuse", ctypes.c_int32),
        ("decide_workgroups", ctypes.c_int32),
        ("status_readback", ctypes.c_int32),
    ]


class lp_timing(ctypes.Structure):
    _fields_ = [
        ("solve_ms", ctypes.c_double),
        ("update_ms", ctypes.c_double),
        ("update_launches", ctypes.c_int64),
        ("pivots", ctypes.c_int64),
        ("updated_columns", ctypes.c_int64),
        ("update_ms_applied", ctypes.c_double),
        ("applied_launches", ctypes.c_int64),
        ("first_pass_ms", ctypes.c_double),
        ("first_pass_pivots", ctypes.c_int64),
        ("first_pass_changed", ctypes.c_int64),
        ("first_pass_columns", ctypes.c_int64),
    ]


class lp_server_stats_t(ctypes.Structure):
    """struct lp_server_stats."""
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("rejected", ctypes.c_int64),
        ("resident_now", ctypes.c_int64),
        ("bytes_in_use", ctypes.c_size_t),
        ("peak_bytes", ctypes.c_size_t),
        ("ticks", ctypes.c_int64),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.c_int64
_OPT = ctypes.POINTER(lp_options)
_RES = ctypes.POINTER(lp_result)

# name -> (restype, argtypes); the full exported surface of include/lpgpu.h
SIGNATURES = {
    "lp_version": (ctypes.c_char_p, []),
    "lp_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lp_last_error": (ctypes.c_char_p, []),
    "lp_options_default": (ctypes.c_int, [_OPT]),
    "lp_tuning_default": (ctypes.c_int, [ctypes.POINTER(lp_tuning)]),
    "lp_tableau_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "lp_create": (ctypes.c_int, [_PP, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _OPT]),
    "lp_create_device": (ctypes.c_int, [_PP, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _OPT]),
    "lp_create_general": (ctypes.c_int, [_PP, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _I32, _OPT]),
    "lp_reload_device": (ctypes.c_int, [_P, _P, _P, _P]),
    "lp_solve": (ctypes.c_int, [_P]),
    "lp_step": (ctypes.c_int, [_P, _I64]),
    "lp_get_solution": (ctypes.c_int, [_P, _RES, _D, _D]),
    "lp_get_pivots": (ctypes.c_int, [_P, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_int64)]),
    "lp_get_tableau": (ctypes.c_int, [_P, _D]),
    "lp_get_basis": (ctypes.c_int, [_P, _I32]),
    "lp_get_info": (ctypes.c_int, [_P, ctypes.POINTER(lp_info)]),
    "lp_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(lp_timing)]),
    "lp_destroy": (None, [_P]),
    "lp_solve_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_size_t, _OPT,
                                        _RES, _D, _D, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_int64)]),
    "lp_diag_arith": (ctypes.c_int, [ctypes.c_int32, _I64, _D, _D, _D, _D, _D]),
    "lp_diag_copy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32, _D]),
    "lp_batch_create": (ctypes.c_int, [_PP, ctypes.c_int32, _I32, _I32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                       ctypes.POINTER(_D), _OPT]),
    "lp_batch_solve": (ctypes.c_int, [_P]),
    "lp_batch_get_solution": (ctypes.c_int, [_P, ctypes.c_int32, _RES, _D, _D]),
    "lp_batch_get_pivots": (ctypes.c_int, [_P, ctypes.c_int32, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_int64)]),
    "lp_batch_solve_ms": (ctypes.c_double, [_P]),
    "lp_batch_reset": (ctypes.c_int, [_P]),
    "lp_batch_get_shape": (ctypes.c_int, [_P, _I32, _I32, _I32]),
    "lp_batch_get_split": (ctypes.c_int, [_P, _I32, _I32, _I32]),
    "lp_batch_set_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lp_batch_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int32, _D]),
    "lp_batch_destroy": (None, [_P]),
    "lp_server_create": (ctypes.c_int, [_PP, ctypes.c_size_t, ctypes.c_int32, _OPT]),
    "lp_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _D, _D, _D,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "lp_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _RES, _D, _D]),
    "lp_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, _RES, _D, _D]),
    "lp_server_get_pivots": (ctypes.c_int, [_P, ctypes.c_uint64, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_int64)]),
    "lp_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(lp_server_stats_t)]),
    "lp_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(lp_server_stats_t)]),
    "lp_server_destroy": (None, [_P]),
    "lp_hybrid_create": (ctypes.c_int, [_PP, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, ctypes.c_double,
                                        ctypes.c_int32, _OPT]),
    "lp_hybrid_solve": (ctypes.c_int, [_P]),
    "lp_hybrid_get_solution": (ctypes.c_int, [_P, _RES, _D, _D]),
    "lp_hybrid_get_pivots": (ctypes.c_int, [_P, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_int64)]),
    "lp_hybrid_get_tableau": (ctypes.c_int, [_P, _D]),
    "lp_hybrid_info": (ctypes.c_int, [_P, _I32, _I32, _I32, _D]),
    "lp_hybrid_destroy": (None, [_P]),
}

_lib = None


def library():
    """Loads liblpgpu.so (built in-tree by paper_2211_10979_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2211_10979_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code, func):
    if code != LP_OK:
        lib = library()
        raise LPError(code, func, lib.lp_last_error().decode() or lib.lp_error_string(code).decode())
    return code


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I32)


def lp_version() -> str:
    return library().lp_version().decode()


def lp_last_error() -> str:
    return library().lp_last_error().decode()


def lp_error_string(code: int) -> str:
    return library().lp_error_string(code).decode()


def lp_tableau_bytes(m: int, n: int) -> int:
    return library().lp_tableau_bytes(m, n)


def lp_tuning_default(**overrides) -> lp_tuning:
    t = lp_tuning()
    _check(library().lp_tuning_default(ctypes.byref(t)), "lp_tuning_default")
    for k, v in overrides.items():
        setattr(t, k, v)
    return t


def lp_options_default(**overrides) -> lp_options:
    """Default options with keyword overrides. `stream` and `device_buffer`
    may be torch objects (a torch.cuda.Stream, a CUDA tensor). Names of
    lp_tuning fields go into a tuning record that the options point to (kept
    alive by the returned object)."""
    o = lp_options()
    _check(library().lp_options_default(ctypes.byref(o)), "lp_options_default")
    tun = {k: v for k, v in overrides.items() if k in TUNING_FIELDS and v is not None}
    if tun:
        o._tuning = lp_tuning_default(**tun)
        o.tuning = ctypes.pointer(o._tuning)
    for k, v in overrides.items():
        if v is None or k in TUNING_FIELDS:
            continue
        if k == "stream" and hasattr(v, "cuda_stream"):
            v = v.cuda_stream
        if k == "device_buffer" and hasattr(v, "data_ptr"):
            o.device_buffer_bytes = v.numel() * v.element_size()
            v = v.data_ptr()
        setattr(o, k, v)
    return o


def _opts(options, kw):
    if options is None:
        return lp_options_default(**kw)
    return options


def lp_create(A, b, c, options: lp_options | None = None, **kw):
    """Creates a context from host arrays; returns the handle (c_void_p)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    m, n = A.shape
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_create(ctypes.byref(h), m, n, _dp(A), _dp(b), _dp(c), ctypes.byref(o)), "lp_create")
    return h


def lp_create_general(A, b, c, sense, options: lp_options | None = None, **kw):
    """Creates a general-form context (rows <=, >= or = per `sense`: LP_LE,
    LP_GE, LP_EQ; any sign of b) from host arrays; returns the handle."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    sense = np.ascontiguousarray(sense, dtype=np.int32)
    m, n = A.shape
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_create_general(ctypes.byref(h), m, n, _dp(A), _dp(b), _dp(c), _ip(sense), ctypes.byref(o)),
           "lp_create_general")
    return h


def lp_create_device(m, n, dA, db, dc, options: lp_options | None = None, **kw):
    """Creates a context from device pointers (ints or torch tensors)."""
    ptr = lambda t: t.data_ptr() if hasattr(t, "data_ptr") else int(t)
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_create_device(ctypes.byref(h), m, n, ptr(dA), ptr(db), ptr(dc), ctypes.byref(o)),
           "lp_create_device")
    return h


def lp_reload_device(h, dA, db, dc):
    ptr = lambda t: t.data_ptr() if hasattr(t, "data_ptr") else int(t)
    _check(library().lp_reload_device(h, ptr(dA), ptr(db), ptr(dc)), "lp_reload_device")


def lp_solve(h):
    _check(library().lp_solve(h), "lp_solve")


def lp_step(h, pivots: int):
    _check(library().lp_step(h, int(pivots)), "lp_step")


def lp_get_info(h) -> lp_info:
    info = lp_info()
    _check(library().lp_get_info(h, ctypes.byref(info)), "lp_get_info")
    return info


def lp_get_timing(h) -> dict:
    t = lp_timing()
    _check(library().lp_get_timing(h, ctypes.byref(t)), "lp_get_timing")
    return {name: getattr(t, name) for name, _ in lp_timing._fields_}


def lp_get_solution(h, want_x=True, want_y=True, m=None, n=None):
    """Returns (result dict, x or None, y or None). For a general-form
    context pass the caller's m and n (lp_get_info reports the tableau's)."""
    info = lp_get_info(h)
    x = np.empty(info.n if n is None else n, dtype=np.float64) if want_x else None
    y = np.empty(info.m if m is None else m, dtype=np.float64) if want_y else None
    res = lp_result()
    _check(library().lp_get_solution(h, ctypes.byref(res), _dp(x) if want_x else None, _dp(y) if want_y else None),
           "lp_get_solution")
    return _res_dict(res), x, y


def _res_dict(res):
    return dict(status=res.status, pivots=res.pivots, objective=res.objective, solve_ms=res.solve_ms)


def lp_get_pivots(h, cap=None):
    count = ctypes.c_int64()
    _check(library().lp_get_pivots(h, None, None, 0, ctypes.byref(count)), "lp_get_pivots")
    k = count.value if cap is None else min(cap, count.value)
    rows = np.empty(max(k, 1), dtype=np.int32)
    cols = np.empty(max(k, 1), dtype=np.int32)
    _check(library().lp_get_pivots(h, _ip(rows), _ip(cols), k, ctypes.byref(count)), "lp_get_pivots")
    return rows[:k].copy(), cols[:k].copy()


def lp_get_tableau(h):
    """The tableau as a row-major (m+1) x W array (a transposed view of the copy)."""
    info = lp_get_info(h)
    out = np.empty((info.width, info.m + 1), dtype=np.float64)
    _check(library().lp_get_tableau(h, _dp(out)), "lp_get_tableau")
    return out.T


def lp_get_basis(h):
    info = lp_get_info(h)
    out = np.empty(info.m, dtype=np.int32)
    _check(library().lp_get_basis(h, _ip(out)), "lp_get_basis")
    return out


def lp_destroy(h):
    if h:
        library().lp_destroy(h)


NOALLOC_SCRATCH_BYTES = 8 << 20  # LP_NOALLOC_SCRATCH_BYTES


def lp_solve_noalloc(m, n, dA, db, dc, tableau, tableau_bytes=None, cap=None, options: lp_options | None = None,
                     **kw):
    """One solve through the entry point that allocates nothing: device inputs
    and a caller-owned device tableau buffer (ints or torch tensors). Returns
    (result dict, x, y, rows, cols, count); the log holds min(count, cap)
    pivots (cap defaults to the device log's length)."""
    ptr = lambda t: t.data_ptr() if hasattr(t, "data_ptr") else int(t)
    if tableau_bytes is None:
        tableau_bytes = tableau.numel() * tableau.element_size()
    o = _opts(options, kw)
    if cap is None:
        cap = min(o.max_pivots if o.max_pivots > 0 else 50 * (m + n), 4 * (m + n) + 64)
    x = np.empty(n, dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    rows = np.empty(max(cap, 1), dtype=np.int32)
    cols = np.empty(max(cap, 1), dtype=np.int32)
    res = lp_result()
    count = ctypes.c_int64()
    _check(library().lp_solve_noalloc(m, n, ptr(dA), ptr(db), ptr(dc), ptr(tableau), int(tableau_bytes),
                                      ctypes.byref(o), ctypes.byref(res), _dp(x), _dp(y), _ip(rows), _ip(cols),
                                      int(cap), ctypes.byref(count)), "lp_solve_noalloc")
    k = min(cap, count.value)
    return _res_dict(res), x, y, rows[:k].copy(), cols[:k].copy(), count.value


def lp_diag_copy(nbytes, reps=10, device=0) -> float:
    """Average device time (ms) of one plain copy of `nbytes` bytes."""
    ms = ctypes.c_double()
    _check(library().lp_diag_copy(device, int(nbytes), int(reps), ctypes.byref(ms)), "lp_diag_copy")
    return ms.value


def lp_diag_arith(a, b, c, device=0):
    """Device a/b and fma(a, b, c), element-wise; returns (quot, fma)."""
    a, b, c = _f64(a), _f64(b), _f64(c)
    q = np.empty_like(a)
    f = np.empty_like(a)
    _check(library().lp_diag_arith(device, a.size, _dp(a), _dp(b), _dp(c), _dp(q), _dp(f)), "lp_diag_arith")
    return q, f


# ------------------------------------------------------------------ batched


def lp_batch_create(lps, options: lp_options | None = None, **kw):
    """lps: sequence of (A, b, c). Returns (handle, keepalive)."""
    arrs = [(_f64(A), _f64(b), _f64(c)) for A, b, c in lps]
    count = len(arrs)
    m = np.array([a[0].shape[0] for a in arrs], dtype=np.int32)
    n = np.array([a[0].shape[1] for a in arrs], dtype=np.int32)
    PA = (_D * count)(*[_dp(a[0]) for a in arrs])
    Pb = (_D * count)(*[_dp(a[1]) for a in arrs])
    Pc = (_D * count)(*[_dp(a[2]) for a in arrs])
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_batch_create(ctypes.byref(h), count, _ip(m), _ip(n), PA, Pb, Pc, ctypes.byref(o)),
           "lp_batch_create")
    return h


def lp_batch_solve(h):
    _check(library().lp_batch_solve(h), "lp_batch_solve")


def lp_batch_solve_ms(h) -> float:
    return library().lp_batch_solve_ms(h)


def lp_batch_get_solution(h, k, m, n):
    x = np.empty(n, dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    res = lp_result()
    _check(library().lp_batch_get_solution(h, k, ctypes.byref(res), _dp(x), _dp(y)), "lp_batch_get_solution")
    return _res_dict(res), x, y


def lp_batch_get_pivots(h, k):
    count = ctypes.c_int64()
    _check(library().lp_batch_get_pivots(h, k, None, None, 0, ctypes.byref(count)), "lp_batch_get_pivots")
    kk = count.value
    rows = np.empty(max(kk, 1), dtype=np.int32)
    cols = np.empty(max(kk, 1), dtype=np.int32)
    _check(library().lp_batch_get_pivots(h, k, _ip(rows), _ip(cols), kk, ctypes.byref(count)),
           "lp_batch_get_pivots")
    return rows[:kk].copy(), cols[:kk].copy()


def lp_batch_reset(h):
    _check(library().lp_batch_reset(h), "lp_batch_reset")


def lp_batch_get_shape(h):
    b, u, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(library().lp_batch_get_shape(h, ctypes.byref(b), ctypes.byref(u), ctypes.byref(g)), "lp_batch_get_shape")
    return dict(block=b.value, unroll=u.value, grid_per_cu=g.value)


def lp_batch_get_split(h):
    w, k, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(library().lp_batch_get_split(h, ctypes.byref(w), ctypes.byref(k), ctypes.byref(e)), "lp_batch_get_split")
    return dict(max_parts=w.value, split_lps=k.value, queue_entries=e.value)


def lp_batch_set_shape(h, block, unroll, grid_per_cu, split=1):
    _check(library().lp_batch_set_shape(h, int(block), int(unroll), int(grid_per_cu), int(split)), "lp_batch_set_shape")


def lp_batch_autotune(h, cache_path=None, trials=2) -> float:
    ms = ctypes.c_double()
    path = cache_path.encode() if cache_path else None
    _check(library().lp_batch_autotune(h, path, int(trials), ctypes.byref(ms)), "lp_batch_autotune")
    return ms.value


def lp_batch_destroy(h):
    if h:
        library().lp_batch_destroy(h)


# ------------------------------------------------------------------ serving


def lp_server_create(budget_bytes: int, max_slots: int = 0, options: lp_options | None = None, **kw):
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_server_create(ctypes.byref(h), int(budget_bytes), int(max_slots), ctypes.byref(o)),
           "lp_server_create")
    return h


def lp_server_submit(h, A, b, c) -> int:
    A, b, c = _f64(A), _f64(b), _f64(c)
    m, n = A.shape
    t = ctypes.c_uint64()
    _check(library().lp_server_submit(h, m, n, _dp(A), _dp(b), _dp(c), ctypes.byref(t)), "lp_server_submit")
    return t.value


def lp_server_poll(h, ticket, m, n):
    """Returns None while pending, else (result dict, x, y)."""
    x = np.empty(n, dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    res = lp_result()
    code = library().lp_server_poll(h, ticket, ctypes.byref(res), _dp(x), _dp(y))
    if code == LP_E_PENDING:
        return None
    _check(code, "lp_server_poll")
    return _res_dict(res), x, y


def lp_server_wait(h, ticket, m, n):
    x = np.empty(n, dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    res = lp_result()
    _check(library().lp_server_wait(h, ticket, ctypes.byref(res), _dp(x), _dp(y)), "lp_server_wait")
    return _res_dict(res), x, y


def lp_server_get_pivots(h, ticket):
    """Pivot log of a finished, uncollected request (LPError LP_E_PENDING before)."""
    count = ctypes.c_int64()
    _check(library().lp_server_get_pivots(h, ticket, None, None, 0, ctypes.byref(count)), "lp_server_get_pivots")
    k = count.value
    rows = np.empty(max(k, 1), dtype=np.int32)
    cols = np.empty(max(k, 1), dtype=np.int32)
    _check(library().lp_server_get_pivots(h, ticket, _ip(rows), _ip(cols), k, ctypes.byref(count)),
           "lp_server_get_pivots")
    k = min(k, count.value)
    return rows[:k].copy(), cols[:k].copy()


def lp_server_stats(h) -> dict:
    st = lp_server_stats_t()
    _check(library().lp_server_stats(h, ctypes.byref(st)), "lp_server_stats")
    return {name: getattr(st, name) for name, _ in lp_server_stats_t._fields_}


lp_server_get_stats = lp_server_stats


def lp_server_destroy(h):
    if h:
        library().lp_server_destroy(h)


# ------------------------------------------------------------------ hybrid


def lp_hybrid_create(A, b, c, theta, host_threads=0, options: lp_options | None = None, **kw):
    """CPU + GPU column split: the GPU holds a share `theta` of the n+m
    columns, the host the rest (updated on `host_threads` threads)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    m, n = A.shape
    o = _opts(options, kw)
    h = ctypes.c_void_p()
    _check(library().lp_hybrid_create(ctypes.byref(h), m, n, _dp(A), _dp(b), _dp(c), float(theta), int(host_threads),
                                      ctypes.byref(o)), "lp_hybrid_create")
    return h


def lp_hybrid_solve(h):
    return _check(library().lp_hybrid_solve(h), "lp_hybrid_solve")


def lp_hybrid_info(h) -> dict:
    dc, hc, ht = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_double()
    _check(library().lp_hybrid_info(h, ctypes.byref(dc), ctypes.byref(hc), ctypes.byref(ht), ctypes.byref(ms)),
           "lp_hybrid_info")
    return dict(device_columns=dc.value, host_columns=hc.value, host_threads=ht.value, host_ms=ms.value)


def lp_hybrid_get_solution(h, m, n):
    """Returns (result dict, x, y) of a solved hybrid handle."""
    x = np.empty(n, dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    res = lp_result()
    _check(library().lp_hybrid_get_solution(h, ctypes.byref(res), _dp(x), _dp(y)), "lp_hybrid_get_solution")
    return _res_dict(res), x, y


def lp_hybrid_get_pivots(h, cap=None):
    count = ctypes.c_int64()
    _check(library().lp_hybrid_get_pivots(h, None, None, 0, ctypes.byref(count)), "lp_hybrid_get_pivots")
    k = count.value if cap is None else min(cap, count.value)
    rows = np.empty(max(k, 1), dtype=np.int32)
    cols = np.empty(max(k, 1), dtype=np.int32)
    _check(library().lp_hybrid_get_pivots(h, _ip(rows), _ip(cols), k, ctypes.byref(count)), "lp_hybrid_get_pivots")
    return rows[:k].copy(), cols[:k].copy()


def lp_hybrid_get_tableau(h, m, n):
    """The tableau as a row-major (m+1) x (n+m+1) array (a transposed view)."""
    out = np.empty((n + m + 1, m + 1), dtype=np.float64)
    _check(library().lp_hybrid_get_tableau(h, _dp(out)), "lp_hybrid_get_tableau")
    return out.T


def lp_hybrid_destroy(h):
    if h:
        library().lp_hybrid_destroy(h)


# ------------------------------------------------------------------ convenience


def solve(A, b, c, **kw):
    """One LP, start to finish: returns a dict with status, pivots, objective,
    x, y, rows, cols and solve_ms."""
    h = lp_create(A, b, c, **kw)
    try:
        lp_solve(h)
        res, x, y = lp_get_solution(h)
        rows, cols = lp_get_pivots(h)
        res.update(x=x, y=y, rows=rows, cols=cols)
        return res
    finally:
        lp_destroy(h)


def solve_hybrid(A, b, c, theta, host_threads=0, **kw):
    """One LP on the CPU + GPU split: as solve, plus the split's info."""
    m, n = np.shape(A)
    h = lp_hybrid_create(A, b, c, theta, host_threads, **kw)
    try:
        lp_hybrid_solve(h)
        res, x, y = lp_hybrid_get_solution(h, m, n)
        rows, cols = lp_hybrid_get_pivots(h)
        res.update(x=x, y=y, rows=rows, cols=cols, **lp_hybrid_info(h))
        return res
    finally:
        lp_hybrid_destroy(h)


def solve_general(A, b, c, sense, **kw):
    """One general-form LP, both phases: returns a dict with status, pivots,
    objective, x, y (the caller's rows), rows, cols and solve_ms."""
    m, n = np.shape(A)
    h = lp_create_general(A, b, c, sense, **kw)
    try:
        lp_solve(h)
        res, x, y = lp_get_solution(h, m=m, n=n)
        rows, cols = lp_get_pivots(h)
        res.update(x=x, y=y, rows=rows, cols=cols)
        return res
    finally:
        lp_destroy(h)
