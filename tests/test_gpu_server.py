"""GPU tests of the serving loop: results equal the oracle's, an LP gives the
same result alone and in a mix, the memory budget holds, errors are reported."""

import sys
import threading

import numpy as np
import pytest

import oracle
from paper_2211_10979_amd import lpgen

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")

GiB = 1 << 30


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mix(seed, count, lo=16, hi=400):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        m, n = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        if k % 4 == 3:  # signed entries: more pivots, some unbounded
            A = rng.integers(1, 10, size=(m, n)).astype(float) * rng.choice([-1.0, 1.0], size=(m, n), p=[0.3, 0.7])
            b = rng.integers(1, 10, size=m).astype(float)
            c = rng.integers(1, 10, size=n).astype(float)
        else:
            lp = lpgen.dense_lp(seed, m, n, k=k)
            A, b, c = lp.A, lp.b, lp.c
        out.append((A, b, c))
    return out


def serve_all(lps, budget=8 * GiB, **kw):
    """Submits every LP, then for each waits for its pivot log and result."""
    s = lpgpu.lp_server_create(budget, **kw)
    try:
        tickets = [lpgpu.lp_server_submit(s, A, b, c) for A, b, c in lps]
        results = []
        for t, (A, _, _) in zip(tickets, lps):
            rows, cols = _wait_log(s, t)
            results.append((lpgpu.lp_server_wait(s, t, *A.shape), rows, cols))
        stats = lpgpu.lp_server_get_stats(s)
    finally:
        lpgpu.lp_server_destroy(s)
    return results, stats


def _wait_log(s, t):
    import time

    while True:
        try:
            return lpgpu.lp_server_get_pivots(s, t)
        except lpgpu.LPError as e:
            if e.code != lpgpu.LP_E_PENDING:
                raise
            time.sleep(0.0005)


def check(lps, results):
    for k, ((A, b, c), ((res, x, y), rows, cols)) in enumerate(zip(lps, results)):
        o = oracle.solve(A, b, c)
        assert res["status"] == o["status"], k
        assert res["pivots"] == o["pivots"], k
        assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist(), k
        assert np.array_equal(x, o["x"]) and np.array_equal(y, o["y"]), k
        assert abs(res["objective"] - o["objective"]) <= 1e-9 * max(1.0, abs(o["objective"])), k


def test_served_results_match_the_oracle():
    lps = mix(1, 60)
    results, stats = serve_all(lps)
    check(lps, results)
    assert stats["completed"] == 60 and stats["submitted"] == 60
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_large_lane_matches_the_oracle():
    """Tableaux above 16 MiB go to the large-LP lane (resident after
    admission, solved by a lane worker with pivot fusion and the per-pivot
    decision kernels): the top of the trace, 4096 x 4096, a 3400 x 3400 LP and
    two mid-size ones, mixed with small LPs of the batched kernel."""
    big = [lpgen.dense_lp(21, 4096, 4096), lpgen.dense_lp(22, 3400, 3400), lpgen.dense_lp(23, 1300, 900),
           lpgen.dense_lp(24, 700, 2500)]
    small = mix(2, 6)
    lps = [(lp.A, lp.b, lp.c) for lp in big[:2]] + small[:3] + [(lp.A, lp.b, lp.c) for lp in big[2:]] + small[3:]
    say("serving 4096 x 4096, 3400 x 3400, 1300 x 900 and 700 x 2500 LPs with 6 small ones")
    results, stats = serve_all(lps, budget=16 * GiB)
    check(lps, results)
    assert stats["completed"] == len(lps)


def test_large_lane_budget_and_order():
    """A budget that holds about two mid-size tableaux at once: every LP still
    finishes with the oracle's result and the budget is never exceeded."""
    lps = [(lp.A, lp.b, lp.c) for lp in (lpgen.dense_lp(30 + k, 1100 + 37 * k, 1000 + 53 * k) for k in range(5))]
    lps += mix(8, 6)
    budget = 80 << 20  # each mid-size tableau is 19-27 MiB with its work block
    say("serving 5 mid-size LPs under an 80 MiB budget")
    results, stats = serve_all(lps, budget=budget)
    check(lps, results)
    assert 0 < stats["peak_bytes"] <= budget


def test_same_result_alone_and_in_the_mix():
    lps = mix(3, 40)
    target = lps[17]
    alone, _ = serve_all([target])
    mixed, _ = serve_all(lps)
    (ra, xa, ya), rows_a, cols_a = alone[0]
    (rm, xm, ym), rows_m, cols_m = mixed[17]
    assert rows_a.tolist() == rows_m.tolist() and cols_a.tolist() == cols_m.tolist()
    assert np.array_equal(xa.view(np.uint64), xm.view(np.uint64))
    assert np.array_equal(ya.view(np.uint64), ym.view(np.uint64))
    assert ra["objective"] == rm["objective"] and ra["status"] == rm["status"]


def test_large_lane_lp_same_alone_and_in_the_mix():
    """An LP of the large-LP lane gives the same bits alone and among other
    large and small LPs (two lane workers and the batched kernel running at
    once)."""
    target = lpgen.dense_lp(41, 1500, 1500)
    others = [lpgen.dense_lp(42 + k, 1200 + 100 * k, 1400 - 100 * k) for k in range(3)]
    lps = mix(9, 10)
    lps[2:2] = [(o.A, o.b, o.c) for o in others[:2]]
    lps.insert(5, (target.A, target.b, target.c))
    lps.append((others[2].A, others[2].b, others[2].c))
    alone, _ = serve_all([(target.A, target.b, target.c)])
    mixed, _ = serve_all(lps)
    (ra, xa, ya), rows_a, cols_a = alone[0]
    (rm, xm, ym), rows_m, cols_m = mixed[5]
    assert rows_a.tolist() == rows_m.tolist() and cols_a.tolist() == cols_m.tolist()
    assert np.array_equal(xa.view(np.uint64), xm.view(np.uint64))
    assert np.array_equal(ya.view(np.uint64), ym.view(np.uint64))
    assert ra["objective"] == rm["objective"] and ra["status"] == rm["status"]
    o = oracle.solve(target.A, target.b, target.c)
    assert rows_a.tolist() == o["rows"].tolist() and np.array_equal(xa, o["x"])


def test_budget_is_never_exceeded():
    lps = mix(4, 30, 300, 500)  # tableaux of about 2.5-6 MB each
    budget = 24 << 20
    results, stats = serve_all(lps, budget=budget)
    check(lps, results)
    assert stats["peak_bytes"] <= budget
    assert stats["peak_bytes"] > 0


def test_few_slots_still_finish_everything():
    lps = mix(5, 25)
    results, stats = serve_all(lps, max_slots=3)
    check(lps, results)
    assert stats["ticks"] >= 25 // 3


def test_concurrent_submitters():
    lps = mix(6, 48)
    s = lpgpu.lp_server_create(8 * GiB)
    tickets = [None] * len(lps)
    try:
        def worker(lo):
            for k in range(lo, len(lps), 4):
                A, b, c = lps[k]
                tickets[k] = lpgpu.lp_server_submit(s, A, b, c)

        threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        results = []
        for t, (A, _, _) in zip(tickets, lps):
            rows, cols = _wait_log(s, t)
            results.append((lpgpu.lp_server_wait(s, t, *A.shape), rows, cols))
    finally:
        lpgpu.lp_server_destroy(s)
    check(lps, results)


def test_errors_are_reported():
    s = lpgpu.lp_server_create(16 << 20)
    try:
        big = lpgen.dense_lp(1, 1200, 1200)  # tableau about 23 MB > 16 MiB budget
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_server_submit(s, big.A, big.b, big.c)
        assert e.value.code == lpgpu.LP_E_BUDGET
        lp = lpgen.dense_lp(1, 20, 20)
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_server_submit(s, lp.A, -lp.b, lp.c)
        assert e.value.code == lpgpu.LP_E_NEG_RHS
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_server_poll(s, 987654, 20, 20)
        assert e.value.code == lpgpu.LP_E_INVAL
        t = lpgpu.lp_server_submit(s, lp.A, lp.b, lp.c)
        res = lpgpu.lp_server_wait(s, t, 20, 20)
        assert res[0]["status"] == lpgpu.LP_OPTIMAL
        with pytest.raises(lpgpu.LPError):
            lpgpu.lp_server_wait(s, t, 20, 20)  # collected already
        assert lpgpu.lp_server_get_stats(s)["rejected"] == 1
    finally:
        lpgpu.lp_server_destroy(s)
