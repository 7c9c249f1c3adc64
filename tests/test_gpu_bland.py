"""GPU parity of the anti-cycling fallback (bland_after = k: Bland's rule
after k degenerate pivots in a row; the one-pivot kernels) against the CPU
oracle, through the C ABI: status, pivot log, tableau, x, y."""

import sys

import numpy as np
import pytest

import oracle
from goldens import read_fixture
from test_oracle_bland import degenerate
from test_oracle_general import random_general

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(A, b, c, k, max_pivots=None, **opts):
    o = oracle.OracleLP(A, b, c, bland_after=k, max_pivots=max_pivots)
    o.step(-1)
    kw = dict(opts, bland_after=k)
    if max_pivots is not None:
        kw["max_pivots"] = max_pivots
    h = lpgpu.lp_create(A, b, c, **kw)
    try:
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        orow, ocol = o.log()
        assert res["status"] == o.status and res["pivots"] == o.pivots
        assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
        assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
        ox, oy, oobj = o.extract()
        assert np.array_equal(x, ox) and np.array_equal(y, oy) and res["objective"] == oobj
        return res["status"], rows, cols
    finally:
        lpgpu.lp_destroy(h)
        o.close()


def test_cycling_example_cycles_without_and_ends_with_the_fallback():
    fx = read_fixture("cycling_example.txt")
    A, b, c = fx["A"], fx["b"], fx["c"]
    st, rows, cols = compare(A, b, c, 0, max_pivots=60)
    assert st == lpgpu.LP_ITER_LIMIT and list(zip(rows.tolist(), cols.tolist()))[:6] == fx["pivot"]
    for k in range(1, 9):
        st, _, _ = compare(A, b, c, k, max_pivots=60)
        assert st == lpgpu.LP_OPTIMAL


def test_degenerate_battery():
    rng = np.random.default_rng(31)
    say("bland: 200 degenerate LPs")
    for t in range(200):
        m, n = int(rng.integers(2, 40)), int(rng.integers(2, 40))
        A, b, c = degenerate(rng, m, n)
        compare(A, b, c, 1 + t % 4)


@pytest.mark.parametrize("opts", [dict(), dict(cols_per_block=1), dict(plain_launches=1), dict(chunk_pivots=1),
                                  dict(update_grid_stride=2)])
def test_options(opts):
    rng = np.random.default_rng(32)
    for t in range(10):
        m, n = int(rng.integers(100, 600)), int(rng.integers(100, 600))
        A, b, c = degenerate(rng, m, n)
        compare(A, b, c, 2, **opts)


def test_general_form_with_the_fallback():
    rng = np.random.default_rng(33)
    say("bland: 60 general-form LPs")
    for t in range(60):
        m, n = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        A, b, c, sense = random_general(rng, m, n)
        b = np.where(rng.random(len(b)) < 0.5, 0.0, b)
        k = 1 + t % 2
        o = oracle.solve_general(A, b, c, sense, bland_after=k)
        h = lpgpu.lp_create_general(A, b, c, sense, bland_after=k)
        try:
            lpgpu.lp_solve(h)
            res, x, y = lpgpu.lp_get_solution(h, m=m, n=n)
            rows, cols = lpgpu.lp_get_pivots(h)
            assert res["status"] == o["status"], t
            assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist(), t
            assert np.array_equal(lpgpu.lp_get_tableau(h), o["tableau"]), t
            if o["status"] == oracle.OPTIMAL:
                assert np.array_equal(x, o["x"]) and np.array_equal(y, o["y"]), t
        finally:
            lpgpu.lp_destroy(h)


def test_off_by_default_and_rejected_forms():
    rng = np.random.default_rng(34)
    A, b, c = degenerate(rng, 30, 30)
    g0 = lpgpu.solve(A, b, c, fuse_pivots=1)
    g1 = lpgpu.solve(A, b, c, fuse_pivots=1, bland_after=0)
    assert g0["rows"].tolist() == g1["rows"].tolist()
    for bad in (dict(bland_after=1, fuse_pivots=4), dict(bland_after=1, select_workgroups=2), dict(bland_after=-1)):
        with pytest.raises(lpgpu.LPError):
            lpgpu.lp_create(A, b, c, **bad)
    with pytest.raises(lpgpu.LPError):
        lpgpu.lp_batch_create([(A, b, c)], bland_after=1)
    with pytest.raises(lpgpu.LPError):
        lpgpu.lp_server_create(1 << 30, bland_after=1)
