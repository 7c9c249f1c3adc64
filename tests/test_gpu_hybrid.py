"""GPU parity of the CPU + GPU column split (Section IV: the GPU holds a share
theta of the columns, the host the rest, the right-hand side on both) against
the CPU oracle, through the C ABI.

Bar: status, pivot count and log identical; the final tableau equal element
by element (the GPU's columns and its copy of the right-hand side, the host's
columns), x, y and the objective equal; over a sweep of theta that puts the
entering column on either side, several host thread counts, tied and
degenerate LPs, unbounded LPs, the iteration cap and the non-finite stops.
"""

import sys

import numpy as np
import pytest

import oracle
from goldens import read_fixture

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")

THETAS = [0.0, 0.02, 0.1, 0.5, 0.9, 1.0]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b), equal_nan=True)


def rand_lp(rng, m, n, lo=1, hi=1000, signed=False):
    A = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    if signed:
        A *= rng.choice([-1.0, 1.0], size=(m, n), p=[0.3, 0.7])
    b = rng.integers(lo, hi + 1, size=m).astype(np.float64)
    c = rng.integers(lo, hi + 1, size=n).astype(np.float64)
    return A, b, c


def split(theta, m, n):
    """The device's share: the first round(theta n) structural and
    round(theta m) slack columns (halves round up)."""
    return int(np.floor(theta * n + 0.5)), int(np.floor(theta * m + 0.5))


def compare(A, b, c, theta, host_threads=0, max_pivots=None):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    ot = oracle.OracleLP(A, b, c, max_pivots=max_pivots)
    kw = {} if max_pivots is None else dict(max_pivots=max_pivots)
    h = lpgpu.lp_hybrid_create(A, b, c, theta, host_threads, **kw)
    try:
        info = lpgpu.lp_hybrid_info(h)
        Jn, Jm = split(theta, m, n)
        assert info["device_columns"] == Jn + Jm
        assert info["device_columns"] + info["host_columns"] == n + m
        assert same(lpgpu.lp_hybrid_get_tableau(h, m, n), ot.tableau()), "initial tableau"
        ot.step(-1)
        lpgpu.lp_hybrid_solve(h)
        res, x, y = lpgpu.lp_hybrid_get_solution(h, m, n)
        rows, cols = lpgpu.lp_hybrid_get_pivots(h)
        ox, oy, oobj = ot.extract()
        orows, ocols = ot.log()
        assert lpgpu.STATUS_NAMES[res["status"]] == oracle.STATUS_NAMES[ot.status]
        assert res["pivots"] == ot.pivots
        assert rows.tolist() == orows.tolist() and cols.tolist() == ocols.tolist()
        assert same(lpgpu.lp_hybrid_get_tableau(h, m, n), ot.tableau())
        assert same(x, ox) and same(y, oy)
        assert (res["objective"] != res["objective"] and oobj != oobj) or res["objective"] == oobj
        on_dev = np.where(cols < n, cols < Jn, cols - n < Jm)
        return res, on_dev, info
    finally:
        lpgpu.lp_hybrid_destroy(h)
        ot.close()


@pytest.mark.parametrize("theta", THETAS)
def test_theta_sweep_matches_the_oracle(theta):
    rng = np.random.default_rng(int(theta * 1000) + 7)
    on_gpu = on_host = 0
    say(f"hybrid: theta {theta}, 12 LPs")
    for t in range(12):
        m, n = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        A, b, c = rand_lp(rng, m, n, hi=(5 if t % 3 == 0 else 1000))
        res, on_dev, info = compare(A, b, c, theta, host_threads=1 + t % 4)
        on_gpu += int(np.sum(on_dev))
        on_host += int(np.sum(~on_dev))
    if 0.0 < theta < 1.0:
        assert on_gpu > 0 and on_host > 0, (on_gpu, on_host)


def test_unbounded_and_degenerate():
    rng = np.random.default_rng(21)
    seen = set()
    for t in range(24):
        m, n = int(rng.integers(2, 120)), int(rng.integers(2, 120))
        A, b, c = rand_lp(rng, m, n, lo=1, hi=4, signed=True)
        if t % 2:
            b[: m // 2] = 0.0  # degenerate vertices
        res, _, _ = compare(A, b, c, theta=(0.3, 0.7)[t % 2], host_threads=4)
        seen.add(res["status"])
    assert lpgpu.LP_UNBOUNDED in seen and lpgpu.LP_OPTIMAL in seen, seen


def test_iteration_cap():
    rng = np.random.default_rng(22)
    A, b, c = rand_lp(rng, 80, 90, signed=True)
    o = oracle.solve(A, b, c)
    assert o["status"] == oracle.OPTIMAL and o["pivots"] > 6
    for cap in (1, 2, o["pivots"] // 2, o["pivots"] - 1, o["pivots"]):
        say(f"hybrid: cap {cap} of {o['pivots']}")
        res, _, _ = compare(A, b, c, theta=0.5, host_threads=2, max_pivots=cap)
        assert res["status"] == (lpgpu.LP_OPTIMAL if cap == o["pivots"] else lpgpu.LP_ITER_LIMIT)


@pytest.mark.parametrize("name", ["nonfinite_step2_nan_rhs.txt", "nonfinite_step1_neg_inf.txt",
                                  "nonfinite_step2_inf_column.txt", "nonfinite_step1_nan.txt"])
def test_nonfinite_fixtures(name):
    fx = read_fixture(name)
    m, n = fx["A"].shape
    for theta in (0.0, 0.5, 1.0):
        say(f"hybrid: fixture {name}, theta {theta}")
        res, _, _ = compare(fx["A"], fx["b"], fx["c"], theta=theta, host_threads=2)
        assert oracle.STATUS_NAMES[res["status"]] == fx["status"] and res["pivots"] == fx["pivots"]


def test_dense_1500_several_tiles():
    rng = np.random.default_rng(23)
    A, b, c = rand_lp(rng, 1500, 1700, signed=True)
    for theta in (0.05, 0.95):
        say(f"hybrid: 1500 x 1700, theta {theta}")
        res, _, _ = compare(A, b, c, theta=theta, host_threads=8)
        assert res["status"] == lpgpu.LP_OPTIMAL and res["pivots"] > 50


def test_same_as_the_single_gpu_solver():
    rng = np.random.default_rng(24)
    A, b, c = rand_lp(rng, 400, 500)
    s = lpgpu.solve(A, b, c)
    g = lpgpu.solve_hybrid(A, b, c, 0.8, host_threads=4)
    assert g["status"] == s["status"] and g["pivots"] == s["pivots"]
    assert g["rows"].tolist() == s["rows"].tolist() and g["cols"].tolist() == s["cols"].tolist()
    assert np.array_equal(g["x"], s["x"]) and np.array_equal(g["y"], s["y"]) and g["objective"] == s["objective"]
    assert g["host_ms"] > 0.0


def test_rejected_arguments():
    A, b, c = np.ones((2, 2)), np.ones(2), np.ones(2)
    for theta in (-0.1, 1.5, float("nan")):
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_hybrid_create(A, b, c, theta)
        assert e.value.code == lpgpu.LP_E_INVAL
    with pytest.raises(lpgpu.LPError) as e:
        lpgpu.lp_hybrid_create(A, -b, c, 0.5)
    assert e.value.code == lpgpu.LP_E_NEG_RHS
    with pytest.raises(lpgpu.LPError) as e:
        lpgpu.lp_hybrid_create(A, b, c, 0.5, bland_after=3)
    assert e.value.code == lpgpu.LP_E_INVAL
    h = lpgpu.lp_hybrid_create(A, b, c, 0.5)
    try:
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_hybrid_get_solution(h, 2, 2)
        assert e.value.code == lpgpu.LP_E_STATE
        lpgpu.lp_hybrid_solve(h)
        lpgpu.lp_hybrid_solve(h)  # solved already: nothing more happens
        res, _, _ = lpgpu.lp_hybrid_get_solution(h, 2, 2)
        assert res["status"] == lpgpu.LP_OPTIMAL
    finally:
        lpgpu.lp_hybrid_destroy(h)
