"""GPU parity of the non-finite stop (LP_NUMERICAL) on every solver path.

The four hand-worked overflow fixtures under tests/golden/ (Section III
Steps 1-2, with the reading for non-finite values: Step 1 stops on a NaN in row
0 or a -inf minimum; Step 2 stops on a non-finite entering-column entry or a
NaN right-hand side in any row) are run through the C ABI on each path and
compared with the oracle: status, pivot count and log are identical, and the
tableau, x, y and the objective are equal element by element, NaN included
(the payload of a NaN is not compared). The oracle's results are themselves
pinned to the fixtures' hand-worked values by the CPU tests.
"""

import sys

import numpy as np
import pytest

import oracle
from goldens import read_fixture

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")

FIXTURES = ["nonfinite_step2_nan_rhs.txt", "nonfinite_step1_neg_inf.txt", "nonfinite_step2_inf_column.txt",
            "nonfinite_step1_nan.txt"]

# the solver's paths: pivot fusion with the one-launch decision kernel
# (default, 24 pivots per group), the two-launches-per-pivot decisions, and
# one pivot per pass
PATHS = {
    "fused24": {},
    "fused_split16": dict(fuse_pivots=16, decide_kernel=1),
    "fused2": dict(fuse_pivots=2),
    "one_pivot": dict(fuse_pivots=1),
    "one_pivot_plain_launches": dict(fuse_pivots=1, plain_launches=1),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b), equal_nan=True)


def same_scalar(a, b):
    return (a != a and b != b) or a == b


def padded(fx, m, n):
    """The fixture in the top-left corner of an m x n LP whose other rows are
    0 <= 1 and whose other columns have zero cost and zero coefficients."""
    A = np.zeros((m, n))
    b = np.ones(m)
    c = np.zeros(n)
    fm, fn = fx["A"].shape
    A[:fm, :fn] = fx["A"]
    b[:fm] = fx["b"]
    c[:fn] = fx["c"]
    return A, b, c


def check(res, x, y, rows, cols, o):
    assert lpgpu.STATUS_NAMES[res["status"]] == oracle.STATUS_NAMES[o["status"]]
    assert res["pivots"] == o["pivots"]
    assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist()
    assert same(x, o["x"]) and same(y, o["y"])
    assert same_scalar(res["objective"], o["objective"])


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("name", FIXTURES)
def test_fixture_on_each_path(name, path):
    fx = read_fixture(name)
    say(f"non-finite fixture {name} on path {path}")
    o = oracle.solve(fx["A"], fx["b"], fx["c"])
    assert oracle.STATUS_NAMES[o["status"]] == fx["status"] and o["pivots"] == fx["pivots"]
    h = lpgpu.lp_create(fx["A"], fx["b"], fx["c"], **PATHS[path])
    try:
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        check(res, x, y, rows, cols, o)
        ot = oracle.OracleLP(fx["A"], fx["b"], fx["c"])
        ot.step(-1)
        assert same(lpgpu.lp_get_tableau(h), ot.tableau())
    finally:
        lpgpu.lp_destroy(h)


@pytest.mark.parametrize("path", ["fused24", "one_pivot"])
@pytest.mark.parametrize("name", FIXTURES)
def test_fixture_pivot_by_pivot(name, path):
    """The tableau after every pivot, overflowed entries included."""
    fx = read_fixture(name)
    say(f"non-finite fixture {name}, pivot by pivot, path {path}")
    h = lpgpu.lp_create(fx["A"], fx["b"], fx["c"], **PATHS[path])
    o = oracle.OracleLP(fx["A"], fx["b"], fx["c"])
    try:
        while True:
            lpgpu.lp_step(h, 1)
            st = o.step(1)
            res, _, _ = lpgpu.lp_get_solution(h)
            assert res["pivots"] == o.pivots
            assert same(lpgpu.lp_get_tableau(h), o.tableau()), f"after pivot {o.pivots}"
            if st != oracle.RUNNING:
                assert res["status"] == st
                break
    finally:
        lpgpu.lp_destroy(h)
        o.close()


@pytest.mark.parametrize("name", FIXTURES)
def test_fixture_deferred_build(name):
    """The first group reads A and c directly (build fused into its pass)."""
    import torch

    fx = read_fixture(name)
    say(f"non-finite fixture {name}, deferred build")
    o = oracle.solve(fx["A"], fx["b"], fx["c"])
    dev = torch.device("cuda", 0)
    dA, db, dc = (torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (fx["A"], fx["b"], fx["c"]))
    m, n = fx["A"].shape
    h = lpgpu.lp_create_device(m, n, dA, db, dc)
    try:
        assert lpgpu.lp_get_info(h).decide_workgroups > 0
        lpgpu.lp_reload_device(h, dA, db, dc)
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        check(res, x, y, rows, cols, o)
    finally:
        lpgpu.lp_destroy(h)


def test_fixtures_in_a_batch():
    """Batched form: the fixtures, padded to various sizes, among ordinary LPs."""
    from paper_2211_10979_amd import lpgen

    lps = []
    for k, name in enumerate(FIXTURES):
        fx = read_fixture(name)
        lps.append((fx["A"], fx["b"], fx["c"]))
        lps.append(padded(fx, 40 + 30 * k, 50 + 20 * k))
        lp = lpgen.dense_lp(7, 60 + k, 70 + k, k=k)
        lps.append((lp.A, lp.b, lp.c))
    say(f"batch of {len(lps)} LPs with the non-finite fixtures")
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        for k, (A, b, c) in enumerate(lps):
            o = oracle.solve(A, b, c)
            res, x, y = lpgpu.lp_batch_get_solution(h, k, *A.shape)
            rows, cols = lpgpu.lp_batch_get_pivots(h, k)
            check(res, x, y, rows, cols, o)
    finally:
        lpgpu.lp_batch_destroy(h)


def _served(lps):
    import time

    s = lpgpu.lp_server_create(4 << 30)
    out = []
    try:
        tickets = [lpgpu.lp_server_submit(s, A, b, c) for A, b, c in lps]
        for t, (A, _, _) in zip(tickets, lps):
            while True:
                try:
                    rows, cols = lpgpu.lp_server_get_pivots(s, t)
                    break
                except lpgpu.LPError as e:
                    if e.code != lpgpu.LP_E_PENDING:
                        raise
                    time.sleep(0.0005)
            out.append((lpgpu.lp_server_wait(s, t, *A.shape), rows, cols))
    finally:
        lpgpu.lp_server_destroy(s)
    return out


def test_fixtures_served():
    """Serving form, both lanes: the fixtures as they are (shared persistent
    kernel) and padded to 1100 x 1100 (19 MB of tableau: the large-LP lane)."""
    lps = []
    for name in FIXTURES:
        fx = read_fixture(name)
        lps.append((fx["A"], fx["b"], fx["c"]))
        lps.append(padded(fx, 1100, 1100))
    say(f"serving {len(lps)} LPs with the non-finite fixtures")
    results = _served(lps)
    for (A, b, c), ((res, x, y), rows, cols) in zip(lps, results):
        check(res, x, y, rows, cols, oracle.solve(A, b, c))
