"""Seeded synthetic LP inputs for the dense-tableau simplex.

This module only draws numbers. It holds none of the simplex arithmetic, so
both the solver and the CPU reference may take their inputs from it.

The paper measures on randomly generated dense LPs whose generator it does not
specify (Section V.B). The stand-in used here: every entry of A, b and c is an
integer drawn uniformly from [1, 1000]. A > 0 and b > 0 make every instance
feasible at the origin and bounded.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014). Its state advances by the
golden-ratio increment and each output is the 64-bit finaliser of the state.
The t-th output (t = 1, 2, ...) of a stream whose state starts at s0 is
therefore mix64(s0 + t * GOLDEN); that closed form lets numpy draw a whole
block at once.

Streams:
  * LP number k of a run seeded with `seed` draws from the stream whose start
    state is mix64(seed * GOLDEN xor k), in the order A (row-major, m*n draws),
    then b (m draws), then c (n draws).
  * Batch and trace sizes draw from the stream starting at mix64(seed xor 0x5EED).

Integers on [lo, hi] use rejection: with span = hi - lo + 1, a draw u is
rejected when u >= floor(2^64 / span) * span, else the value is lo + u mod span.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

GENERATOR_VERSION = 1

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
SIZE_STREAM_SALT = 0x5EED

_CHUNK = 1 << 20
_POOL = None
_NATIVE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblpgen.so")
_NATIVE = None


def _native():
    """The C build of the same draws (lpgen_native.c), or None when it is not
    built (then numpy draws the same numbers, more slowly)."""
    global _NATIVE
    if _NATIVE is None:
        _NATIVE = False
        if os.path.exists(_NATIVE_PATH) and not os.environ.get("LPGEN_NUMPY"):
            import ctypes

            lib = ctypes.CDLL(_NATIVE_PATH)
            lib.lpgen_values.restype = ctypes.c_int64
            lib.lpgen_values.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_void_p]
            _NATIVE = lib
    return _NATIVE or None


def _pool():
    global _POOL
    if _POOL is None:
        workers = int(os.environ.get("LPGEN_THREADS", "0")) or min(16, len(os.sched_getaffinity(0)))
        _POOL = ThreadPoolExecutor(max_workers=max(1, workers))
    return _POOL


def mix64(z: int) -> int:
    """SplitMix64 output finaliser on one Python integer (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
    return z ^ (z >> np.uint64(31))


class Stream:
    """One SplitMix64 stream, drawn in blocks."""

    def __init__(self, start_state: int):
        self.state = start_state & MASK64
        self.drawn = 0  # number of outputs consumed so far

    def raw(self, count: int) -> np.ndarray:
        """The next `count` raw 64-bit outputs (blocks computed in parallel;
        each output depends only on its position, so the result does not
        depend on the number of threads)."""
        out = np.empty(count, dtype=np.uint64)
        first = self.drawn

        def block(lo):
            hi = min(count, lo + _CHUNK)
            with np.errstate(over="ignore"):
                t = np.arange(first + lo + 1, first + hi + 1, dtype=np.uint64)
                out[lo:hi] = _mix64_np(np.uint64(self.state) + t * np.uint64(GOLDEN))

        starts = range(0, count, _CHUNK)
        if count > 2 * _CHUNK:
            list(_pool().map(block, starts))
        else:
            for lo in starts:
                block(lo)
        self.drawn += count
        return out

    def integers(self, count: int, lo: int, hi: int) -> np.ndarray:
        """`count` integers uniform on [lo, hi], by rejection, as int64."""
        span = hi - lo + 1
        limit = ((1 << 64) // span) * span
        got = []
        need = count
        while need > 0:
            u = self.raw(need)
            keep = u[u < np.uint64(limit)] if limit < (1 << 64) else u
            if keep.size > need:  # cannot happen: at most `need` drawn
                keep = keep[:need]
            got.append(keep)
            need -= keep.size
        u = np.concatenate(got) if len(got) > 1 else got[0]
        return (u % np.uint64(span)).astype(np.int64) + lo

    def values(self, count: int, lo: int, hi: int) -> np.ndarray:
        """As integers(), as float64, computed block-parallel. When no draw
        of the range is rejected (each draw is rejected with probability
        below 2^-54), the k-th value is the k-th draw's; otherwise the exact
        sequential rejection path is taken."""
        span = hi - lo + 1
        lib = _native()
        if lib is not None and 1 <= span <= (1 << 62):
            out = np.empty(count, dtype=np.float64)
            self.drawn += lib.lpgen_values(self.state, self.drawn, count, lo, hi, out.ctypes.data)
            return out
        limit = np.uint64(((1 << 64) // span) * span)
        out = np.empty(count, dtype=np.float64)
        first = self.drawn
        rejected = [False]

        def block(b0):
            b1 = min(count, b0 + _CHUNK)
            with np.errstate(over="ignore"):
                t = np.arange(first + b0 + 1, first + b1 + 1, dtype=np.uint64)
                u = _mix64_np(np.uint64(self.state) + t * np.uint64(GOLDEN))
            if np.any(u >= limit):
                rejected[0] = True
            np.add(u % np.uint64(span), np.uint64(lo), out=u)
            out[b0:b1] = u

        starts = range(0, count, _CHUNK)
        if count > 2 * _CHUNK:
            list(_pool().map(block, starts))
        else:
            for b0 in starts:
                block(b0)
        if rejected[0]:
            return self.integers(count, lo, hi).astype(np.float64)
        self.drawn += count
        return out

    def unit(self, count: int) -> np.ndarray:
        """`count` doubles in [0, 1) from the top 53 bits of each draw."""
        u = self.raw(count) >> np.uint64(11)
        return u.astype(np.float64) * (1.0 / (1 << 53))


def lp_stream(seed: int, k: int) -> Stream:
    return Stream(mix64(((seed * GOLDEN) & MASK64) ^ k))


def size_stream(seed: int) -> Stream:
    return Stream(mix64(seed ^ SIZE_STREAM_SALT))


@dataclass
class LP:
    """max c^T x subject to A x <= b, x >= 0 (A row-major m x n, float64)."""

    A: np.ndarray
    b: np.ndarray
    c: np.ndarray

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def dense_lp(seed: int, m: int, n: int, k: int = 0, lo: int = 1, hi: int = 1000) -> LP:
    """LP number k of `seed`: A, b, c integer-valued uniform on [lo, hi]."""
    if m < 1 or n < 1:
        raise ValueError("m and n must be >= 1")
    s = lp_stream(seed, k)
    A = s.values(m * n, lo, hi).reshape(m, n)
    b = s.values(m, lo, hi)
    c = s.values(n, lo, hi)
    return LP(A, b, c)


def batch_sizes(seed: int, count: int, lo: int = 32, hi: int = 512):
    """Sizes (m_k, n_k), each uniform on {lo..hi}, drawn m then n per LP."""
    s = size_stream(seed)
    v = s.integers(2 * count, lo, hi).reshape(count, 2)
    return [(int(a), int(b)) for a, b in v]


def trace_sizes(seed: int, count: int, lo: int = 64, octaves: int = 6):
    """Sizes log-uniform on [lo, lo * 2^octaves] and unit-rate exponential gaps.

    Per LP three draws: u_m, u_n, u_gap. m = round(lo * 2^(octaves * u_m)),
    likewise n; the inter-arrival gap at rate lambda is gap / lambda with
    gap = -ln(1 - u_gap).
    """
    s = size_stream(seed)
    u = s.unit(3 * count).reshape(count, 3)
    sizes = []
    gaps = []
    for um, un, ug in u:
        sizes.append((int(round(lo * 2.0 ** (octaves * um))), int(round(lo * 2.0 ** (octaves * un)))))
        gaps.append(-math.log1p(-ug))
    return sizes, np.asarray(gaps, dtype=np.float64)


# Named workloads, by their sizes and seeds.
WORKLOADS = {
    "dense_200x200": dict(seed=1, m=200, n=200),
    "dense_2000x2000": dict(seed=2, m=2000, n=2000),
    "dense_8000x8000": dict(seed=3, m=8000, n=8000),
}
BATCH_SEED = 4
TRACE_SEED = 5


def workload(name: str) -> LP:
    w = WORKLOADS[name]
    return dense_lp(w["seed"], w["m"], w["n"])
