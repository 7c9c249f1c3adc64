"""GPU parity of pivot fusion (several pivots decided, then applied in one pass
over the tableau) against the CPU oracle, through the C ABI.

Bar: as for one pivot per pass — identical pivot log, basis and status, and
the tableau equal element by element after every group and at the end — for
every group size K in 1..16, including LPs on which a column leaves and enters
again, or enters and leaves again, inside one group.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2211_10979_amd import lpgen

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")

AUTO_FUSE = 24  # the library's group size when fuse_pivots is 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def degenerate_lp(seed, kind):
    """Small LPs with many ties and zero right-hand sides (degenerate pivots),
    kind 0: dense positive, 1: signed small integers, 2: 0..3 integers,
    3: signed reals."""
    rng = np.random.default_rng(1000 + seed)
    m, n = int(rng.integers(3, 44)), int(rng.integers(3, 44))
    if kind == 0:
        A = rng.uniform(1, 1000, (m, n))
        b = rng.uniform(1, 1000, m)
        c = rng.uniform(1, 1000, n)
    else:
        if kind == 1:
            A = rng.integers(-2, 5, (m, n)).astype(float)
        elif kind == 2:
            A = rng.integers(0, 4, (m, n)).astype(float)
        else:
            A = rng.uniform(-0.5, 1.5, (m, n))
        b = np.where(rng.random(m) < 0.4, 0.0, rng.integers(0, 10, m).astype(float))
        c = rng.integers(-2, 7, n).astype(float)
    return A, b, c


def group_events(m, n, rows, cols, K):
    """(leave-then-enter, enter-then-leave) counts inside groups of K pivots,
    from a pivot log."""
    basis = list(range(n, n + m))
    reenter = leave_entered = 0
    for g0 in range(0, len(rows), K):
        entered, left = set(), set()
        for r, q in zip(rows[g0:g0 + K], cols[g0:g0 + K]):
            leave = basis[r - 1]
            basis[r - 1] = q
            reenter += q in left
            leave_entered += leave in entered
            entered.add(q)
            left.add(leave)
    return reenter, leave_entered


def solve_and_compare(A, b, c, **opts):
    o = oracle.OracleLP(A, b, c, max_pivots=opts.get("max_pivots"))
    o.step(-1)
    h = lpgpu.lp_create(A, b, c, **opts)
    try:
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        orow, ocol = o.log()
        assert res["status"] == o.status
        assert res["pivots"] == o.pivots
        assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
        assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
        assert lpgpu.lp_get_basis(h).tolist() == o.basis().tolist()
        ox, oy, oobj = o.extract()
        assert np.array_equal(x, ox) and np.array_equal(y, oy)
        assert lpgpu.lp_get_info(h).update_fuse == opts.get("fuse_pivots", 4)
        return orow.tolist(), ocol.tolist()
    finally:
        lpgpu.lp_destroy(h)
        o.close()


@pytest.mark.parametrize("K,decide", [(2, 0), (3, 0), (4, 0), (5, 0), (8, 0), (11, 0), (16, 0), (20, 0), (32, 0), (48, 0),
                                     (4, 1), (16, 1)])
def test_degenerate_battery(K, decide):
    """120 small LPs; the battery contains in-group re-entries of both kinds.
    decide = 0: all decisions of a group in one launch; 1: two launches per
    pivot."""
    say(f"fused K={K} decide_kernel={decide}: degenerate battery")
    events = np.zeros(2, dtype=int)
    for seed in range(120):
        A, b, c = degenerate_lp(seed, seed % 4)
        rows, cols = solve_and_compare(A, b, c, fuse_pivots=K, decide_kernel=decide)
        events += group_events(A.shape[0], A.shape[1], rows, cols, K)
    # a column that has just left has a positive objective-row entry, so it
    # cannot enter at the next pivot: with K = 2 no group can re-enter one
    assert events[1] > 0 and (K == 2 or events[0] > 0), events


@pytest.mark.parametrize("K", range(1, 49))
def test_every_group_size(K):
    """Every group size from 1 to 48 with the one-launch decisions, and 1 to
    16 with two launches per pivot: 16 degenerate LPs each, log, tableau, x
    and y equal to the oracle's."""
    say(f"fused K={K}: 16 degenerate LPs")
    for seed in range(16):
        A, b, c = degenerate_lp(500 + seed, seed % 4)
        solve_and_compare(A, b, c, fuse_pivots=K)
        if K <= 16:
            solve_and_compare(A, b, c, fuse_pivots=K, decide_kernel=1)


@pytest.mark.parametrize("K,decide", [(2, 0), (4, 0), (7, 0), (8, 0), (13, 0), (16, 0), (24, 0), (31, 0), (41, 0), (7, 1),
                                     (16, 1)])
def test_group_boundaries_by_stepping(K, decide):
    """lp_step budgets that cut groups short and ones that span several
    groups: the tableau matches the oracle's after every step."""
    lp = lpgen.workload("dense_200x200")
    say(f"fused K={K} decide_kernel={decide}: dense_200x200 stepping")
    h = lpgpu.lp_create(lp.A, lp.b, lp.c, fuse_pivots=K, decide_kernel=decide)
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    try:
        budgets = [1, K, K + 1, 2 * K - 1, 3, 2 * K + 3]
        k = 0
        while True:
            every = budgets[k % len(budgets)]
            k += 1
            lpgpu.lp_step(h, every)
            st = o.step(every)
            res, _, _ = lpgpu.lp_get_solution(h)
            assert res["pivots"] == o.pivots
            assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau()), f"after pivot {o.pivots}"
            assert lpgpu.lp_get_basis(h).tolist() == o.basis().tolist()
            if st != oracle.RUNNING:
                break
        rows, cols = lpgpu.lp_get_pivots(h)
        orow, ocol = o.log()
        assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
    finally:
        lpgpu.lp_destroy(h)
        o.close()


@pytest.mark.parametrize("K,decide", [(1, 0), (3, 0), (4, 0), (8, 0), (12, 0), (16, 0), (24, 0), (32, 0), (48, 0), (12, 1)])
def test_dense_2000_full_solve(K, decide):
    lp = lpgen.workload("dense_2000x2000")
    say(f"fused K={K} decide_kernel={decide}: dense_2000x2000")
    solve_and_compare(lp.A, lp.b, lp.c, fuse_pivots=K, decide_kernel=decide)


@pytest.mark.parametrize("opts", [dict(cols_per_block=1), dict(cols_per_block=2), dict(cols_per_block=8),
                                  dict(rows_per_thread=1), dict(update_block=128, cols_per_block=4, fuse_pivots=3),
                                  dict(update_block=64, cols_per_block=8),
                                  dict(update_block=128, cols_per_block=1), dict(update_block=64, cols_per_block=2),
                                  dict(plain_launches=1), dict(chunk_pivots=9), dict(time_kernels=1),
                                  dict(cols_per_block=2, fuse_pivots=8), dict(cols_per_block=4, fuse_pivots=6),
                                  dict(cols_per_block=8, fuse_pivots=7),
                                  dict(cols_per_block=4, fuse_pivots=8, time_kernels=1),
                                  dict(cols_per_block=8, fuse_pivots=16, time_kernels=1),
                                  dict(cols_per_block=2, fuse_pivots=12), dict(cols_per_block=1, fuse_pivots=9)])
def test_update_shapes(opts):
    A, b, c = degenerate_lp(7, 1)
    lp = lpgen.dense_lp(9, 333, 444)
    say(f"fused shapes {opts}")
    cases = [(lp.A, lp.b, lp.c)]
    if "update_block" not in opts:  # a block size other than 256 needs m + 1 > 256
        cases.append((A, b, c))
    opts = dict(opts)
    K = opts.pop("fuse_pivots", 4)
    for AA, bb, cc in cases:
        solve_and_compare(AA, bb, cc, fuse_pivots=K, **opts)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 9), (9, 1), (63, 64), (127, 129), (255, 257), (2049, 300),
                                 (4095, 64), (8191, 20), (30, 3000)])
def test_shapes(m, n):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.integers(1, 10, (m, n)).astype(float) * rng.choice([-1.0, 1.0], (m, n), p=[0.3, 0.7])
    b = rng.integers(1, 10, m).astype(float)
    c = rng.integers(1, 10, n).astype(float)
    say(f"fused shape {m}x{n}")
    solve_and_compare(A, b, c, fuse_pivots=4, max_pivots=150)


def test_cap_unbounded_and_optimal_inside_a_group():
    A, b, c = degenerate_lp(3, 1)
    full = oracle.solve(A, b, c)
    say("fused: cap / unbounded / immediate optimum")
    for cap in range(1, min(full["pivots"], 10)):
        g = lpgpu.solve(A, b, c, max_pivots=cap, fuse_pivots=4)
        assert g["status"] == lpgpu.LP_ITER_LIMIT and g["pivots"] == cap
        assert g["rows"].tolist() == full["rows"][:cap].tolist()
    rng = np.random.default_rng(4)
    A = rng.integers(1, 10, (50, 30)).astype(float)
    b = rng.integers(1, 10, 50).astype(float)
    c = rng.integers(1, 10, 30).astype(float)
    A[:, 7] = -A[:, 7]
    for big in (5000.0, 0.5):  # column 7 enters first, or only after a few pivots
        cc = c.copy()
        cc[7] = big
        o = oracle.solve(A, b, cc)
        g = lpgpu.solve(A, b, cc, fuse_pivots=4)
        assert g["status"] == o["status"] == lpgpu.LP_UNBOUNDED
        assert g["rows"].tolist() == o["rows"].tolist() and g["cols"].tolist() == o["cols"].tolist()
    g = lpgpu.solve(A, b, -np.abs(c), fuse_pivots=4)
    assert g["status"] == lpgpu.LP_OPTIMAL and g["pivots"] == 0


def test_work_counter_counts_the_union_of_a_group():
    """updated_columns: per pass, the columns with a nonzero normalised
    pivot-row entry in some pivot of the group."""
    rng = np.random.default_rng(21)
    A = rng.integers(1, 10, (150, 170)).astype(float) * rng.choice([-1.0, 1.0], (150, 170), p=[0.3, 0.7])
    b = rng.integers(1, 10, 150).astype(float)
    c = rng.integers(1, 10, 170).astype(float)
    K = 4
    o = oracle.OracleLP(A, b, c)
    h = lpgpu.lp_create(A, b, c, fuse_pivots=K, time_kernels=1)
    try:
        total = 0
        for _ in range(5):
            changed = np.zeros(A.shape[1] + A.shape[0] + 1, dtype=bool)
            for _ in range(K):
                before = o.pivots
                T = o.tableau()
                o.step(1)
                if o.pivots == before:
                    break
                changed |= T[int(o.log()[0][-1])] != 0
            total += int(changed.sum())
            lpgpu.lp_step(h, K)
            t = lpgpu.lp_get_timing(h)
            assert t["pivots"] == o.pivots
            assert t["updated_columns"] == total
            assert t["update_launches"] >= 1 and t["update_ms"] > 0
            assert t["applied_launches"] == 1 and 0 < t["update_ms_applied"] <= t["update_ms"]
    finally:
        lpgpu.lp_destroy(h)
        o.close()


def test_options_are_checked():
    lp = lpgen.dense_lp(2, 600, 200)  # m + 1 > 256: every update option applies
    A, b, c = lp.A, lp.b, lp.c
    for bad in (dict(fuse_pivots=49), dict(fuse_pivots=17, decide_kernel=1), dict(fuse_pivots=-1),
                dict(fuse_pivots=4, cols_per_block=16), dict(fuse_pivots=24, cols_per_block=1),
                dict(fuse_pivots=2, rows_per_thread=4), dict(fuse_pivots=2, rows_per_thread=2),
                dict(fuse_pivots=2, select_workgroups=2),
                dict(fuse_pivots=3, update_grid_stride=2), dict(fuse_pivots=2, update_hints=1),
                dict(decide_kernel=2), dict(decide_kernel=-1), dict(decide_spin=-5), dict(decide_block=128),
                dict(fuse_pivots=24, decide_block=512)):
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_create(A, b, c, **bad)
        assert e.value.code == lpgpu.LP_E_INVAL
    # auto falls back to one pivot per pass where the fused kernels do not apply
    h = lpgpu.lp_create(A, b, c, cols_per_block=16)
    try:
        assert lpgpu.lp_get_info(h).update_fuse == 1
    finally:
        lpgpu.lp_destroy(h)
    h = lpgpu.lp_create(A, b, c)
    try:
        assert lpgpu.lp_get_info(h).update_fuse == AUTO_FUSE
    finally:
        lpgpu.lp_destroy(h)
    h = lpgpu.lp_create(A, b, c, decide_kernel=1)  # two launches per pivot: groups of at most 16
    try:
        assert lpgpu.lp_get_info(h).update_fuse == 16
    finally:
        lpgpu.lp_destroy(h)
    h = lpgpu.lp_create(A, b, c, decide_block=512)  # 512-thread decision workgroups: at most 16
    try:
        assert lpgpu.lp_get_info(h).update_fuse == 16
    finally:
        lpgpu.lp_destroy(h)


def test_decision_kernel_gives_up_instead_of_hanging():
    """With a wait limit of one poll, the workgroups of the one-launch
    decision kernel cannot all meet at a barrier: the solve stops with
    LP_STALLED and every kernel exits; a normal context then solves."""
    lp = lpgen.workload("dense_2000x2000")  # 8 decision workgroups
    say("fused: stalled decision kernel")
    g = lpgpu.solve(lp.A, lp.b, lp.c, decide_spin=1)
    assert g["status"] == lpgpu.LP_STALLED
    A, b, c = degenerate_lp(5, 1)
    solve_and_compare(A, b, c, fuse_pivots=12)


def check_against_oracle(h, o, lp):
    res, x, y = lpgpu.lp_get_solution(h)
    rows, cols = lpgpu.lp_get_pivots(h)
    orow, ocol = o.log()
    assert res["status"] == o.status and res["pivots"] == o.pivots
    assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
    assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
    assert lpgpu.lp_get_basis(h).tolist() == o.basis().tolist()
    ox, oy, _ = o.extract()
    assert np.array_equal(x, ox) and np.array_equal(y, oy)


@pytest.mark.parametrize("opts", [dict(), dict(fuse_pivots=12), dict(fuse_pivots=32), dict(plain_launches=1),
                                  dict(time_kernels=1), dict(status_readback=2)])
def test_closed_gate_resumes_without_barriers(opts):
    """decide_spin -1 closes the check-in gate of the first one-launch
    decision, as when its workgroups cannot all be resident: that launch
    writes nothing and the solve goes on with the barrier-free decision
    kernels (groups of at most 16 pivots), with the oracle's pivots, tableau,
    basis and solution."""
    lp = lpgen.workload("dense_2000x2000")
    say(f"fused: closed gate, fallback {opts}")
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    o.step(-1)
    h = lpgpu.lp_create(lp.A, lp.b, lp.c, decide_spin=-1, **opts)
    try:
        info = lpgpu.lp_get_info(h)
        K = info.update_fuse
        assert info.decide_workgroups > 0
        lpgpu.lp_solve(h)
        check_against_oracle(h, o, lp)
        info = lpgpu.lp_get_info(h)
        assert info.decide_workgroups == 0 and info.update_fuse == min(K, 16)
    finally:
        lpgpu.lp_destroy(h)
        o.close()


def test_closed_gate_on_a_deferred_build_and_stepping():
    """The gate of the first group after a deferred build closes: that
    group's pass builds the structural columns alone, the unstored slack
    columns are stored, and lp_step goes on barrier-free; the tableau matches
    the oracle's after every step."""
    import torch

    lp = lpgen.workload("dense_200x200")
    say("fused: closed gate on a deferred build, stepping")
    dev = torch.device("cuda", 0)
    dA, db, dc = (torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (lp.A, lp.b, lp.c))
    h = lpgpu.lp_create_device(lp.m, lp.n, dA, db, dc, decide_spin=-1)
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    try:
        lpgpu.lp_reload_device(h, dA, db, dc)
        while True:
            lpgpu.lp_step(h, 7)
            st = o.step(7)
            res, _, _ = lpgpu.lp_get_solution(h)
            assert res["pivots"] == o.pivots
            assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau()), f"after pivot {o.pivots}"
            if st != oracle.RUNNING:
                break
        check_against_oracle(h, o, lp)
        assert lpgpu.lp_get_info(h).decide_workgroups == 0
    finally:
        lpgpu.lp_destroy(h)
        o.close()


def test_closed_gate_in_the_solve_that_allocates_nothing():
    import torch

    lp = lpgen.workload("dense_2000x2000")
    say("fused: closed gate in lp_solve_noalloc")
    dev = torch.device("cuda", 0)
    dA, db, dc = (torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (lp.A, lp.b, lp.c))
    buf = torch.empty(lpgpu.lp_tableau_bytes(lp.m, lp.n) // 8, dtype=torch.float64, device=dev)
    o = oracle.solve(lp.A, lp.b, lp.c)
    res, x, y, rows, cols, count = lpgpu.lp_solve_noalloc(lp.m, lp.n, dA, db, dc, buf, decide_spin=-1)
    assert res["status"] == o["status"] and count == o["pivots"]
    assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist()
    assert np.array_equal(x, o["x"]) and np.array_equal(y, o["y"])


@pytest.mark.parametrize("block", [256, 512])
def test_decision_kernel_block_sizes(block):
    """The decision kernel's workgroup size changes no result."""
    say(f"fused: decision kernel with {block} threads per workgroup")
    for seed in range(0, 120, 7):
        A, b, c = degenerate_lp(seed, seed % 4)
        solve_and_compare(A, b, c, fuse_pivots=16, decide_block=block)
    lp = lpgen.workload("dense_2000x2000")
    solve_and_compare(lp.A, lp.b, lp.c, fuse_pivots=16, decide_block=block)
