"""GPU parity of the general form (rows <=, >= or =, any sign of b; the
two-phase method on the one-pivot kernels) against the CPU oracle, through
the C ABI: status, pivot log (both phases and the drive-out), basis, the
final tableau element by element, x, y and the objective."""

import sys

import numpy as np
import pytest

import oracle
from test_oracle_general import feasible_general, random_general

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")

LE, GE, EQ = lpgpu.LP_LE, lpgpu.LP_GE, lpgpu.LP_EQ


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(A, b, c, sense, max_pivots=None, **opts):
    A = np.asarray(A, dtype=float)
    m, n = A.shape
    o = oracle.solve_general(A, b, c, sense, max_pivots=max_pivots)
    kw = dict(opts)
    if max_pivots is not None:
        kw["max_pivots"] = max_pivots
    h = lpgpu.lp_create_general(A, b, c, sense, **kw)
    try:
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h, m=m, n=n)
        rows, cols = lpgpu.lp_get_pivots(h)
        assert res["status"] == o["status"], (res["status"], o["status"])
        assert res["pivots"] == o["pivots"]
        assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist()
        assert lpgpu.lp_get_basis(h).tolist() == o["basis"].tolist()
        assert np.array_equal(lpgpu.lp_get_tableau(h), o["tableau"])
        if o["status"] == oracle.OPTIMAL:
            assert np.array_equal(x, o["x"]) and np.array_equal(y, o["y"])
            assert res["objective"] == o["objective"]
        return o
    finally:
        lpgpu.lp_destroy(h)


def test_mixed_rows_match_the_oracle():
    rng = np.random.default_rng(11)
    seen = {}
    say("general form: 150 mixed LPs")
    for t in range(150):
        m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        if t % 3 == 0:
            A, b, c, sense = random_general(rng, m, n)
        elif t % 3 == 1:
            A, b, c, sense = feasible_general(rng, m, n, bound=200.0)
        else:
            A, b, c, sense = feasible_general(rng, m, n)
        o = compare(A, b, c, sense)
        seen[o["status"]] = seen.get(o["status"], 0) + 1
    assert seen.get(oracle.OPTIMAL, 0) >= 40 and seen.get(oracle.INFEASIBLE, 0) >= 10, seen
    assert seen.get(oracle.UNBOUNDED, 0) >= 5, seen


def test_tile_shapes_and_options():
    rng = np.random.default_rng(12)
    for opts in (dict(cols_per_block=1), dict(cols_per_block=8), dict(rows_per_thread=2), dict(plain_launches=1),
                 dict(chunk_pivots=1), dict(fuse_pivots=1)):
        say(f"general form: options {opts}")
        for t in range(8):
            m, n = int(rng.integers(20, 300)), int(rng.integers(20, 300))
            A, b, c, sense = feasible_general(rng, m, n, bound=500.0)
            compare(A, b, c, sense, **opts)


def test_all_le_rows_equal_the_standard_path():
    rng = np.random.default_rng(13)
    for t in range(10):
        m, n = int(rng.integers(5, 200)), int(rng.integers(5, 200))
        A = rng.integers(1, 1000, size=(m, n)).astype(float)
        b = rng.integers(1, 1000, size=m).astype(float)
        c = rng.integers(1, 1000, size=n).astype(float)
        g = lpgpu.solve_general(A, b, c, np.full(m, LE))
        s = lpgpu.solve(A, b, c, fuse_pivots=1)
        assert g["status"] == s["status"] and g["rows"].tolist() == s["rows"].tolist()
        assert g["cols"].tolist() == s["cols"].tolist()
        assert np.array_equal(g["x"], s["x"]) and np.array_equal(g["y"], s["y"]) and g["objective"] == s["objective"]


def test_closed_forms():
    compare([[1.0], [1.0]], [1.0, 2.0], [1.0], [LE, GE])  # infeasible
    o = compare([[-1.0, -1.0], [1.0, 0.0]], [0.0, 5.0], [1.0, 1.0], [EQ, LE])  # drive-out on a negative entry
    assert o["status"] == oracle.OPTIMAL and (2, 0) in list(zip(o["rows"].tolist(), o["cols"].tolist()))
    A = np.array([[1.0, 2.0], [1.0, 2.0], [1.0, 0.0]])  # a redundant equality
    o = compare(A, [4.0, 4.0, 3.0], [1.0, 1.0], [EQ, EQ, LE])
    assert o["status"] == oracle.OPTIMAL
    o = compare([[1.0, -1.0]], [1.0], [1.0, 0.0], [GE])  # unbounded
    assert o["status"] == oracle.UNBOUNDED
    k = 9
    rng = np.random.default_rng(14)
    bb = rng.integers(0, 9, size=k).astype(float)
    cc = rng.integers(-4, 9, size=k).astype(float)
    o = compare(np.eye(k), bb, cc, np.full(k, EQ))  # x = b, y = c
    assert np.array_equal(o["x"], bb) and np.array_equal(o["y"], cc)


def test_iteration_cap_in_each_phase():
    rng = np.random.default_rng(15)
    A, b, c, sense = feasible_general(rng, 60, 50, bound=300.0)
    o = oracle.solve_general(A, b, c, sense)
    assert o["status"] == oracle.OPTIMAL and o["pivots"] > 4
    for cap in range(1, o["pivots"] + 1):  # 0 asks for the default cap
        say(f"general form: cap {cap} of {o['pivots']}")
        g = compare(A, b, c, sense, max_pivots=cap)
        assert g["status"] == (oracle.OPTIMAL if cap == o["pivots"] else oracle.ITER_LIMIT)


def test_dense_2000_general():
    rng = np.random.default_rng(16)
    say("general form: 2000 x 2000")
    A, b, c, sense = feasible_general(rng, 2000, 2000, bound=5000.0)
    o = compare(A, b, c, sense)
    assert o["status"] == oracle.OPTIMAL and o["pivots"] > 100
    cert = oracle.certificates_general(A, b, c, sense, o["x"], o["y"], o["objective"])
    assert cert["ok"], cert


def test_rejected_options_and_calls():
    A, b, c = np.ones((2, 2)), np.ones(2), np.ones(2)
    with pytest.raises(lpgpu.LPError) as e:
        lpgpu.lp_create_general(A, b, c, [LE, GE], fuse_pivots=4)
    assert e.value.code == lpgpu.LP_E_INVAL
    with pytest.raises(lpgpu.LPError):
        lpgpu.lp_create_general(A, b, c, [LE, 3])
    h = lpgpu.lp_create_general(A, b, c, [LE, GE])
    try:
        with pytest.raises(lpgpu.LPError):
            lpgpu.lp_step(h, 1)
        lpgpu.lp_solve(h)
        lpgpu.lp_solve(h)  # solved already: nothing more happens
        res, _, _ = lpgpu.lp_get_solution(h, m=2, n=2)
        assert res["status"] == lpgpu.LP_OPTIMAL
    finally:
        lpgpu.lp_destroy(h)
