"""GPU parity of the deferred build against the CPU oracle, through the C ABI.

lp_reload_device with the one-launch decision kernel does not build the
tableau at once: the first group's decisions read the structural columns from
A and c, its update pass writes them with the group's pivots applied, and a
slack column is stored only when it leaves the basis. The bar is the same as
for the built tableau: identical pivot log, basis, status, x, y and objective,
and the tableau equal element by element (lp_get_tableau stores the basic
columns first). Before every reload the tableau memory is filled with NaN, so
that any entry read before it is written shows in the results.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2211_10979_amd import lpgen

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")
torch = pytest.importorskip("torch")

from test_gpu_fused import degenerate_lp, group_events  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


class Deferred:
    """A context whose tableau lives in a caller-owned buffer, so that the
    test can poison it before each reload."""

    def __init__(self, m, n, **opts):
        self.m, self.n = m, n
        nbytes = lpgpu.lp_tableau_bytes(m, n)
        self.buf = torch.empty(nbytes // 8, dtype=torch.float64, device=torch.device("cuda", 0))
        one = dev(np.ones((m, n))), dev(np.ones(m)), dev(np.ones(n))
        self.h = lpgpu.lp_create_device(m, n, *one, device_buffer=self.buf, **opts)

    def reload(self, A, b, c):
        self.inputs = dev(A), dev(b), dev(c)  # kept alive until the next reload
        torch.cuda.synchronize()
        self.buf.fill_(float("nan"))
        torch.cuda.synchronize()
        lpgpu.lp_reload_device(self.h, *self.inputs)

    def close(self):
        lpgpu.lp_destroy(self.h)


def compare_final(h, o):
    res, x, y = lpgpu.lp_get_solution(h)
    rows, cols = lpgpu.lp_get_pivots(h)
    orow, ocol = o.log()
    assert res["status"] == o.status
    assert res["pivots"] == o.pivots
    assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
    ox, oy, oobj = o.extract()
    assert np.array_equal(x, ox) and np.array_equal(y, oy)
    assert res["objective"] == oobj or (np.isnan(res["objective"]) and np.isnan(oobj))
    assert lpgpu.lp_get_basis(h).tolist() == o.basis().tolist()
    # after the solution: lp_get_tableau stores the basic columns
    assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
    return orow.tolist(), ocol.tolist()


@pytest.mark.parametrize("K", [2, 4, 11, 16, 24, 32, 40, 48])
def test_degenerate_battery_deferred(K):
    """120 small LPs of several shapes through one context each, reloaded;
    the battery has in-group re-entries, so slack columns are stored on
    leaving and read again within the group."""
    say(f"deferred build K={K}: degenerate battery")
    events = np.zeros(2, dtype=int)
    for seed in range(120):
        A, b, c = degenerate_lp(seed, seed % 4)
        m, n = A.shape
        d = Deferred(m, n, fuse_pivots=K)
        o = oracle.OracleLP(A, b, c)
        try:
            assert lpgpu.lp_get_info(d.h).decide_workgroups > 0
            d.reload(A, b, c)
            lpgpu.lp_solve(d.h)
            o.step(-1)
            rows, cols = compare_final(d.h, o)
            events += group_events(m, n, rows, cols, K)
        finally:
            d.close()
            o.close()
    assert events[1] > 0 and (K == 2 or events[0] > 0), events


@pytest.mark.parametrize("K,readback", [(7, 1), (16, 1), (29, 1), (7, 0), (29, 2)])
def test_stepping_after_reload(K, readback):
    """A first lp_step of 0 pivots (the first pass only builds), then
    budgets that cut groups short; the tableau after every step. Read-back 2
    reads the solver state right after each group's decisions."""
    lp = lpgen.workload("dense_200x200")
    say(f"deferred build K={K} status_readback={readback}: dense_200x200 stepping")
    d = Deferred(lp.m, lp.n, fuse_pivots=K, status_readback=readback)
    assert lpgpu.lp_get_info(d.h).status_readback == (1 if readback == 1 else 2)  # 0: auto
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    try:
        d.reload(lp.A, lp.b, lp.c)
        lpgpu.lp_step(d.h, 0)
        assert np.array_equal(lpgpu.lp_get_tableau(d.h), o.tableau()), "built by a pass of no pivots"
        budgets = [1, K, K + 1, 2 * K - 1, 3]
        k = 0
        while True:
            every = budgets[k % len(budgets)]
            k += 1
            lpgpu.lp_step(d.h, every)
            st = o.step(every)
            res, _, _ = lpgpu.lp_get_solution(d.h)
            assert res["pivots"] == o.pivots
            assert np.array_equal(lpgpu.lp_get_tableau(d.h), o.tableau()), f"after pivot {o.pivots}"
            if st != oracle.RUNNING:
                break
        compare_final(d.h, o)
    finally:
        d.close()
        o.close()


def test_tableau_before_any_solve():
    """lp_get_tableau while the deferred build is pending builds it there;
    the solve then continues from the built tableau."""
    lp = lpgen.workload("dense_200x200")
    say("deferred build: tableau before the solve")
    d = Deferred(lp.m, lp.n)
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    try:
        d.reload(lp.A, lp.b, lp.c)
        assert np.array_equal(lpgpu.lp_get_tableau(d.h), o.tableau()), "initial tableau"
        lpgpu.lp_solve(d.h)
        o.step(-1)
        compare_final(d.h, o)
    finally:
        d.close()
        o.close()


@pytest.mark.parametrize("shape", [(301, 401), (300, 400), (2000, 2000)])
def test_full_solve_and_alignment(shape):
    """Odd and even n, A at an 8-byte offset (no 16-byte loads of A), and the
    dense 2000 x 2000 LP."""
    m, n = shape
    lp = lpgen.workload("dense_2000x2000") if shape == (2000, 2000) else lpgen.dense_lp(40 + n, m, n)
    say(f"deferred build: {m}x{n}")
    d = Deferred(m, n)
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    try:
        flat = torch.empty(m * n + 1, dtype=torch.float64, device=torch.device("cuda", 0))
        flat[1:] = dev(lp.A.ravel())
        dA = flat[1:].view(m, n)
        assert dA.data_ptr() % 16 == 8
        db, dc = dev(lp.b), dev(lp.c)
        torch.cuda.synchronize()
        d.buf.fill_(float("nan"))
        torch.cuda.synchronize()
        lpgpu.lp_reload_device(d.h, dA, db, dc)
        lpgpu.lp_solve(d.h)
        o.step(-1)
        compare_final(d.h, o)
        # and again from 16-byte aligned inputs, same context
        d.reload(lp.A, lp.b, lp.c)
        lpgpu.lp_solve(d.h)
        compare_final(d.h, o)
    finally:
        d.close()
        o.close()


def test_timing_counters_and_eager_option():
    """time_kernels: the first pass is timed apart and counted; eager_build = 1
    builds at once (no first pass) with the same results."""
    lp = lpgen.workload("dense_2000x2000")
    say("deferred build: counters, eager_build")
    out = {}
    for eager in (0, 1):
        d = Deferred(lp.m, lp.n, time_kernels=1, eager_build=eager)
        try:
            d.reload(lp.A, lp.b, lp.c)
            lpgpu.lp_solve(d.h)
            res, x, y = lpgpu.lp_get_solution(d.h)
            t = lpgpu.lp_get_timing(d.h)
            K = lpgpu.lp_get_info(d.h).update_fuse
            out[eager] = (res, x, y, lpgpu.lp_get_tableau(d.h))
            if eager:
                assert t["first_pass_ms"] == 0 and t["first_pass_pivots"] == 0 and t["first_pass_columns"] == 0
            else:
                assert t["first_pass_ms"] > 0
                assert t["first_pass_pivots"] == min(K, res["pivots"])
                assert 0 < t["first_pass_changed"] <= t["updated_columns"]
                assert lp.n + 1 < t["first_pass_columns"] <= lp.n + 1 + K
            # the update launches timed are those after the first group
            assert t["applied_launches"] == -(-(res["pivots"] - t["first_pass_pivots"]) // K)
        finally:
            d.close()
    (r0, x0, y0, T0), (r1, x1, y1, T1) = out[0], out[1]
    assert r0["pivots"] == r1["pivots"] and r0["objective"] == r1["objective"]
    assert np.array_equal(x0, x1) and np.array_equal(y0, y1) and np.array_equal(T0, T1)
    with pytest.raises(Exception):
        lpgpu.lp_create(lp.A[:10, :10], lp.b[:10], lp.c[:10], eager_build=2)


def test_dense_8000_bench_configuration():
    """The benchmark workload at full size in the configuration the benchmark
    times: a context from device arrays with kernel timing on, reloaded from
    device arrays (deferred build) twice; each solve's log, solution and
    final tableau equal the oracle's."""
    lp = lpgen.workload("dense_8000x8000")
    say("dense_8000x8000 deferred build: oracle")
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    o.step(-1)
    ox, oy, oobj = o.extract()
    orow, ocol = o.log()
    OT = o.tableau()
    obasis = o.basis()
    o.close()
    d = Deferred(lp.m, lp.n, time_kernels=1)
    try:
        assert lpgpu.lp_get_info(d.h).decide_workgroups > 0
        for k in range(2):
            say(f"dense_8000x8000 deferred build: gpu solve {k}")
            d.reload(lp.A, lp.b, lp.c)
            lpgpu.lp_solve(d.h)
            res, x, y = lpgpu.lp_get_solution(d.h)
            rows, cols = lpgpu.lp_get_pivots(d.h)
            assert res["status"] == lpgpu.LP_OPTIMAL and res["pivots"] == len(orow)
            assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
            assert res["objective"] == oobj
            assert np.array_equal(x, ox) and np.array_equal(y, oy)
            assert lpgpu.lp_get_basis(d.h).tolist() == obasis.tolist()
            t = lpgpu.lp_get_timing(d.h)
            assert t["first_pass_columns"] > lp.n and t["applied_launches"] >= 1
            T = lpgpu.lp_get_tableau(d.h)
            assert np.array_equal(T, OT)
            del T
    finally:
        d.close()


@pytest.mark.parametrize("K", [4, 24])
def test_degenerate_battery_early_status(K):
    """The degenerate battery with the solver state read right after each
    group's decisions (status_readback = 2)."""
    say(f"deferred build K={K}: degenerate battery, status_readback 2")
    for seed in range(120):
        A, b, c = degenerate_lp(seed, seed % 4)
        m, n = A.shape
        d = Deferred(m, n, fuse_pivots=K, status_readback=2)
        o = oracle.OracleLP(A, b, c)
        try:
            d.reload(A, b, c)
            lpgpu.lp_solve(d.h)
            o.step(-1)
            compare_final(d.h, o)
        finally:
            d.close()
            o.close()


def test_status_readback_counters_and_choice():
    """With the state read after the decisions no group is launched after the
    end (at most one pass that applies nothing: a group whose first pricing
    finds the optimum); one group behind, one is. Same results either way.
    The automatic choice and the rejected combinations."""
    lp = lpgen.workload("dense_2000x2000")
    say("status_readback: counters on dense_2000x2000")
    out = {}
    for rb in (1, 2):
        d = Deferred(lp.m, lp.n, time_kernels=1, status_readback=rb)
        try:
            assert lpgpu.lp_get_info(d.h).status_readback == rb
            d.reload(lp.A, lp.b, lp.c)
            lpgpu.lp_solve(d.h)
            res, x, y = lpgpu.lp_get_solution(d.h)
            t = lpgpu.lp_get_timing(d.h)
            idle = t["update_launches"] - t["applied_launches"]
            assert idle in ((0, 1) if rb == 2 else (1, 2)), (rb, t)
            out[rb] = (res, x, y, lpgpu.lp_get_tableau(d.h), lpgpu.lp_get_pivots(d.h), t)
            # the work counters after a pivot budget (read back with the state)
            d.reload(lp.A, lp.b, lp.c)
            lpgpu.lp_step(d.h, 5)
            lpgpu.lp_step(d.h, 30)
            out[rb] += (lpgpu.lp_get_timing(d.h),)
        finally:
            d.close()
    (r1, x1, y1, T1, l1, t1, s1), (r2, x2, y2, T2, l2, t2, s2) = out[1], out[2]
    # every work counter agrees between the two read-back modes: the
    # roofline bytes of the benchmark are computed from them
    for key in ("pivots", "updated_columns", "first_pass_pivots", "first_pass_changed", "first_pass_columns"):
        assert t1[key] == t2[key], (key, t1[key], t2[key])
        assert s1[key] == s2[key], (key, s1[key], s2[key])
    assert r1["pivots"] == r2["pivots"] and r1["objective"] == r2["objective"]
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2) and np.array_equal(T1, T2)
    assert l1[0].tolist() == l2[0].tolist() and l1[1].tolist() == l2[1].tolist()
    small = lpgen.workload("dense_200x200")
    h = lpgpu.lp_create(small.A, small.b, small.c)
    try:
        assert lpgpu.lp_get_info(h).status_readback == 2  # auto, with the one-launch decision kernel
    finally:
        lpgpu.lp_destroy(h)
    h = lpgpu.lp_create(small.A, small.b, small.c, decide_kernel=1)
    try:
        assert lpgpu.lp_get_info(h).status_readback == 1  # auto, with two launches per pivot
    finally:
        lpgpu.lp_destroy(h)
    for bad in (dict(status_readback=3), dict(status_readback=2, fuse_pivots=1),
                dict(status_readback=2, decide_kernel=1), dict(status_readback=2, chunk_pivots=100)):
        with pytest.raises(Exception):
            lpgpu.lp_create(small.A, small.b, small.c, **bad)
