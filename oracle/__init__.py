"""CPU reference for the full-tableau simplex method, and result certificates.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers. The GPU solver package neither
imports this module nor links its library, and this module imports nothing
from the solver package.

The arithmetic lives in `tableau_simplex.c` (plain C, binary64, explicit fma,
built with -ffp-contract=off); this file only loads it and checks results.

Parity status of each function (what pins it is in the test suite):
  solve / OracleLP       pinned: exact-rational Dantzig simplex (pivot
                         sequence), brute-force vertex enumeration (optimum),
                         closed forms, B^-1 [A I b] recomputation (tableau),
                         scipy HiGHS (objective), strong duality.
  certificates           pinned: hand-built feasible/infeasible points.
  solve_general          pinned: exact-rational run of the same two-phase
                         method (pivot sequence, statuses), brute-force vertex
                         enumeration of the equality form (optimum,
                         infeasibility), scipy HiGHS (status, objective),
                         closed forms, reduction to `solve` on <= rows with
                         b >= 0 (bit for bit), general certificates.
  certificates_general   pinned: hand-built points.
  bland_after (either)   pinned: the cycling example below ends at its
                         optimum; exact-rational run of the same switching
                         rule (pivot sequence); with Bland's rule forced from
                         the first pivot, Bland's theorem (no basis repeats)
                         on degenerate batteries; off, bit-identical to the
                         plain method.
  The pivot sequence at m = n = 8000 is "parity unpinned" beyond the oracle
  itself: no exact reference finishes at that size; only the certificates pin
  its optimum independently.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tableau_simplex.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OPTIMAL, UNBOUNDED, ITER_LIMIT, NUMERICAL, RUNNING, INFEASIBLE = 0, 1, 2, 3, 4, 6
STATUS_NAMES = {0: "OPTIMAL", 1: "UNBOUNDED", 2: "ITER_LIMIT", 3: "NUMERICAL", 4: "RUNNING", 6: "INFEASIBLE"}
LE, GE, EQ = 0, 1, 2  # row senses of the general form

CFLAGS = ["-O3", "-mfma", "-mavx2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(verbose: bool = False, src: str = _SRC, out: str = LIB_PATH) -> str:
    """Compile the C reference with gcc (by default to liboracle.so). Returns the path."""
    cmd = ["gcc", *CFLAGS, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def _load(path=None):
    """Loads the default library, or a library built from a variant at `path`."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    if path is None and not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(path or LIB_PATH)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i64 = ctypes.c_int64
    lib.oracle_create.restype = P
    lib.oracle_create.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                  i64, i64, ctypes.c_int]
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_step.argtypes = [P, i64]
    lib.oracle_status.restype = ctypes.c_int
    lib.oracle_status.argtypes = [P]
    lib.oracle_pivots.restype = i64
    lib.oracle_pivots.argtypes = [P]
    lib.oracle_width.restype = ctypes.c_int
    lib.oracle_width.argtypes = [P]
    lib.oracle_get_tableau.argtypes = [P, dp]
    lib.oracle_get_basis.argtypes = [P, ip]
    lib.oracle_get_log.restype = i64
    lib.oracle_get_log.argtypes = [P, ip, ip, i64]
    lib.oracle_extract.argtypes = [P, dp, dp, dp]
    lib.oracle_create_general.restype = P
    lib.oracle_create_general.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ip, ctypes.c_double,
                                          ctypes.c_double, i64, i64, ctypes.c_int]
    lib.oracle_solve_general.restype = ctypes.c_int
    lib.oracle_solve_general.argtypes = [P]
    lib.oracle_extract_general.argtypes = [P, dp, dp, dp]
    lib.oracle_general_layout.argtypes = [P, ip, ip, ip, ip, dp]
    lib.oracle_set_bland.argtypes = [P, ctypes.c_int]
    if path is None:
        _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_max_pivots(m: int, n: int) -> int:
    return 50 * (m + n)


class OracleLP:
    """A tableau held by the C reference, advanced pivot by pivot."""

    def __init__(self, A, b, c, eps_d=1e-9, eps_p=1e-9, max_pivots=None, log_cap=None, threads=None,
                 library=None, bland_after=0):
        lib = _load(library)
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        m, n = A.shape
        if b.shape != (m,) or c.shape != (n,):
            raise ValueError("shape mismatch")
        self.m, self.n, self.W = m, n, n + m + 1
        if max_pivots is None:
            max_pivots = default_max_pivots(m, n)
        if log_cap is None:
            log_cap = max_pivots
        if threads is None:
            threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        self.threads = threads
        self._h = lib.oracle_create(m, n, _dptr(A), _dptr(b), _dptr(c), eps_d, eps_p, int(max_pivots),
                                    int(log_cap), int(threads))
        if not self._h:
            raise ValueError("oracle_create rejected the LP (bad size, non-finite value or negative b)")
        self._lib = lib
        if bland_after:
            lib.oracle_set_bland(self._h, int(bland_after))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, k: int = -1) -> int:
        return self._lib.oracle_step(self._h, int(k))

    @property
    def status(self) -> int:
        return self._lib.oracle_status(self._h)

    @property
    def pivots(self) -> int:
        return self._lib.oracle_pivots(self._h)

    def tableau(self) -> np.ndarray:
        out = np.empty((self.m + 1, self.W), dtype=np.float64)
        self._lib.oracle_get_tableau(self._h, _dptr(out))
        return out

    def basis(self) -> np.ndarray:
        out = np.empty(self.m, dtype=np.int32)
        self._lib.oracle_get_basis(self._h, _iptr(out))
        return out

    def log(self):
        k = self.pivots
        rows = np.empty(max(k, 1), dtype=np.int32)
        cols = np.empty(max(k, 1), dtype=np.int32)
        got = self._lib.oracle_get_log(self._h, _iptr(rows), _iptr(cols), int(k))
        return rows[:got].copy(), cols[:got].copy()

    def extract(self):
        x = np.empty(self.n, dtype=np.float64)
        y = np.empty(self.m, dtype=np.float64)
        obj = np.empty(1, dtype=np.float64)
        self._lib.oracle_extract(self._h, _dptr(x), _dptr(y), _dptr(obj))
        return x, y, float(obj[0])


def solve(A, b, c, eps_d=1e-9, eps_p=1e-9, max_pivots=None, threads=None, library=None, bland_after=0):
    """Solves to the end. Returns a dict with status, pivots, objective, x, y, log.
    bland_after = k > 0: Bland's rule after k consecutive degenerate pivots."""
    o = OracleLP(A, b, c, eps_d=eps_d, eps_p=eps_p, max_pivots=max_pivots, threads=threads, library=library,
                 bland_after=bland_after)
    try:
        o.step(-1)
        x, y, obj = o.extract()
        rows, cols = o.log()
        return dict(status=o.status, pivots=o.pivots, objective=obj, x=x, y=y, rows=rows, cols=cols,
                    basis=o.basis())
    finally:
        o.close()


def solve_general(A, b, c, sense, eps_d=1e-9, eps_p=1e-9, max_pivots=None, threads=None, library=None,
                  bland_after=0):
    """The general form (rows <=, >= or = by `sense`: LE, GE, EQ; any sign of
    b; x >= 0) by the two-phase method. Returns a dict with status, pivots,
    objective, x, y (the caller's row order), the pivot log (tableau rows:
    the <= rows, then >=, then =, after sign normalisation; row m+1 carries
    the objective), the final tableau ((m+2) x (n'+m+2)), the basis, and the
    layout (nprime, n_le, perm, sign)."""
    lib = _load(library)
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    sense = np.ascontiguousarray(sense, dtype=np.int32)
    m, n = A.shape
    if b.shape != (m,) or c.shape != (n,) or sense.shape != (m,):
        raise ValueError("shape mismatch")
    if max_pivots is None:
        max_pivots = default_max_pivots(m, n)
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    h = lib.oracle_create_general(m, n, _dptr(A), _dptr(b), _dptr(c), _iptr(sense), eps_d, eps_p,
                                  int(max_pivots), int(max_pivots), int(threads))
    if not h:
        raise ValueError("oracle_create_general rejected the LP (bad size, non-finite value or sense)")
    try:
        if bland_after:
            lib.oracle_set_bland(h, int(bland_after))
        status = lib.oracle_solve_general(h)
        pivots = lib.oracle_pivots(h)
        x = np.empty(n)
        y = np.empty(m)
        obj = np.empty(1)
        lib.oracle_extract_general(h, _dptr(x), _dptr(y), _dptr(obj))
        W = lib.oracle_width(h)
        T = np.empty((m + 2, W))
        lib.oracle_get_tableau(h, _dptr(T))
        basis = np.empty(m + 1, dtype=np.int32)
        lib.oracle_get_basis(h, _iptr(basis))
        rows = np.empty(max(pivots, 1), dtype=np.int32)
        cols = np.empty(max(pivots, 1), dtype=np.int32)
        got = lib.oracle_get_log(h, _iptr(rows), _iptr(cols), int(pivots))
        npr = np.zeros(1, dtype=np.int32)
        nle = np.zeros(1, dtype=np.int32)
        ph = np.zeros(1, dtype=np.int32)
        perm = np.empty(m, dtype=np.int32)
        sign = np.empty(m)
        lib.oracle_general_layout(h, _iptr(npr), _iptr(nle), _iptr(ph), _iptr(perm), _dptr(sign))
        return dict(status=status, pivots=pivots, objective=float(obj[0]), x=x, y=y, rows=rows[:got].copy(),
                    cols=cols[:got].copy(), tableau=T, basis=basis, nprime=int(npr[0]), n_le=int(nle[0]),
                    perm=perm, sign=sign)
    finally:
        lib.oracle_destroy(h)


def certificates_general(A, b, c, sense, x, y, objective, tau=1e-9):
    """Optimality certificates of (x, y) for the general form: max c^T x with
    rows A_i x <= b_i (sense LE), >= b_i (GE) or = b_i (EQ), x >= 0. The dual
    is min b^T y with A^T y >= c, y_i >= 0 on <= rows, y_i <= 0 on >= rows,
    y_i free on = rows. Residuals scaled as in `certificates`."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    sense = np.asarray(sense)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    absA = np.abs(A)
    Ax = A @ x
    scale_p = np.maximum(1.0, np.maximum(np.abs(b), absA @ np.abs(x)))
    viol = np.where(sense == LE, np.maximum(Ax - b, 0.0),
                    np.where(sense == GE, np.maximum(b - Ax, 0.0), np.abs(Ax - b)))
    primal = float(np.max(viol / scale_p, initial=0.0))
    xneg = float(np.max(np.maximum(-x, 0.0), initial=0.0) / max(1.0, float(np.max(np.abs(x), initial=0.0))))
    ATy = A.T @ y
    scale_d = np.maximum(1.0, np.maximum(np.abs(c), absA.T @ np.abs(y)))
    dual = float(np.max(np.maximum(c - ATy, 0.0) / scale_d, initial=0.0))
    ysign = np.where(sense == LE, np.maximum(-y, 0.0), np.where(sense == GE, np.maximum(y, 0.0), 0.0))
    ybad = float(np.max(ysign, initial=0.0) / max(1.0, float(np.max(np.abs(y), initial=0.0))))
    cx = float(c @ x)
    by = float(b @ y)
    gap = abs(cx - by) / max(1.0, abs(cx))
    objerr = abs(objective - cx) / max(1.0, abs(cx))
    res = dict(primal=primal, x_nonneg=xneg, dual=dual, y_sign=ybad, gap=gap, objective=objerr)
    res["ok"] = all(v <= tau for v in res.values())
    return res


def certificates(A, b, c, x, y, objective, tau=1e-9):
    """Optimality certificates of (x, y) for max c^T x, Ax <= b, x >= 0.

    Each residual is scaled as stated; a check passes when its scaled residual
    is <= tau. Returns a dict of scaled residuals plus 'ok'.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    absA = np.abs(A)
    Ax = A @ x
    scale_p = np.maximum(1.0, np.maximum(np.abs(b), absA @ np.abs(x)))
    primal = float(np.max(np.maximum(Ax - b, 0.0) / scale_p, initial=0.0))
    xneg = float(np.max(np.maximum(-x, 0.0), initial=0.0) / max(1.0, float(np.max(np.abs(x), initial=0.0))))
    ATy = A.T @ y
    scale_d = np.maximum(1.0, np.maximum(np.abs(c), absA.T @ np.abs(y)))
    dual = float(np.max(np.maximum(c - ATy, 0.0) / scale_d, initial=0.0))
    yneg = float(np.max(np.maximum(-y, 0.0), initial=0.0) / max(1.0, float(np.max(np.abs(y), initial=0.0))))
    cx = float(c @ x)
    by = float(b @ y)
    gap = abs(cx - by) / max(1.0, abs(cx))
    objerr = abs(objective - cx) / max(1.0, abs(cx))
    res = dict(primal=primal, x_nonneg=xneg, dual=dual, y_nonneg=yneg, gap=gap, objective=objerr)
    res["ok"] = all(v <= tau for v in res.values())
    return res
