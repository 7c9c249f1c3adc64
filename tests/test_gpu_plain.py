"""GPU parity of the single-LP solver against the CPU oracle, through the C ABI.

Bar: the pivot log is identical; the tableau is equal element by element
(compared with ==, so only the sign of a zero may differ, which no comparison
of the method can observe); the optimum is within 1e-9 relative (it is
expected bit-equal, since both sides perform the same roundings); every
optimal result passes the certificates.
"""

import ctypes
import os
import subprocess
import sys
import time
import tempfile

import numpy as np
import pytest

import oracle
from paper_2211_10979_amd import lpgen

pytestmark = pytest.mark.gpu

lpgpu = pytest.importorskip("paper_2211_10979_amd.lpgpu")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_lp(seed, m, n, lo=1, hi=1000, signed=False):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    if signed:
        A *= rng.choice([-1.0, 1.0], size=(m, n), p=[0.3, 0.7])
    b = rng.integers(lo, hi + 1, size=m).astype(np.float64)
    c = rng.integers(lo, hi + 1, size=n).astype(np.float64)
    return A, b, c


def assert_same_result(A, b, c, g, o):
    assert lpgpu.STATUS_NAMES[g["status"]] == oracle.STATUS_NAMES[o["status"]]
    assert g["pivots"] == o["pivots"]
    assert g["rows"].tolist() == o["rows"].tolist()
    assert g["cols"].tolist() == o["cols"].tolist()
    assert abs(g["objective"] - o["objective"]) <= 1e-9 * max(1.0, abs(o["objective"]))
    assert np.array_equal(g["x"], o["x"]) and np.array_equal(g["y"], o["y"])
    if o["status"] == oracle.OPTIMAL:
        cert = oracle.certificates(A, b, c, g["x"], g["y"], g["objective"])
        assert cert["ok"], cert


def step_compare(A, b, c, every=1, max_checks=None, **opts):
    """Advances GPU and oracle `every` pivots at a time and compares tableaux."""
    h = lpgpu.lp_create(A, b, c, **opts)
    o = oracle.OracleLP(A, b, c)
    try:
        assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau()), "initial tableau"
        checks = 0
        while True:
            lpgpu.lp_step(h, every)
            st = o.step(every)
            res, _, _ = lpgpu.lp_get_solution(h)
            assert res["pivots"] == o.pivots
            T = lpgpu.lp_get_tableau(h)
            assert np.array_equal(T, o.tableau()), f"tableau differs after pivot {o.pivots}"
            assert lpgpu.lp_get_basis(h).tolist() == o.basis().tolist()
            checks += 1
            if st != oracle.RUNNING or (max_checks and checks >= max_checks):
                break
        return h, o
    except BaseException:
        lpgpu.lp_destroy(h)
        o.close()
        raise


def test_library_version():
    assert "lpgpu" in lpgpu.lp_version()


def _fma_reference(a, b, c):
    """Correctly rounded fma on the host (glibc's fma, compiled in a helper)."""
    src = r"""
    #include <math.h>
    #include <stdint.h>
    void fma_many(int64_t n, const double* a, const double* b, const double* c, double* o) {
        for (int64_t k = 0; k < n; ++k) o[k] = fma(a[k], b[k], c[k]);
    }"""
    d = tempfile.mkdtemp()
    with open(os.path.join(d, "f.c"), "w") as f:
        f.write(src)
    so = os.path.join(d, "f.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, os.path.join(d, "f.c"), "-lm"],
                   check=True)
    lib = ctypes.CDLL(so)
    out = np.empty_like(a)
    D = ctypes.POINTER(ctypes.c_double)
    lib.fma_many(ctypes.c_int64(a.size), a.ctypes.data_as(D), b.ctypes.data_as(D), c.ctypes.data_as(D),
                 out.ctypes.data_as(D))
    return out


def test_device_division_and_fma_are_ieee():
    """Steps 2 and 3 round exactly as the host does (bitwise), subnormals included."""
    rng = np.random.default_rng(0)
    N = 10_000_000
    a = rng.standard_normal(N) * np.exp2(rng.integers(-60, 60, N))
    b = rng.standard_normal(N) * np.exp2(rng.integers(-60, 60, N))
    c = rng.standard_normal(N) * np.exp2(rng.integers(-60, 60, N))
    # subnormal and boundary cases
    k = 200_000
    a[:k] = rng.standard_normal(k) * 2.0 ** -1060
    b[k:2 * k] = rng.standard_normal(k) * 2.0 ** 1000
    c[2 * k:3 * k] = -a[2 * k:3 * k] * b[2 * k:3 * k]
    a[3 * k:4 * k] = rng.integers(1, 1000, k).astype(float)
    b[3 * k:4 * k] = rng.integers(1, 1000, k).astype(float)
    q, f = lpgpu.lp_diag_arith(a, b, c)
    with np.errstate(all="ignore"):
        qh = a / b
    assert np.array_equal(q.view(np.uint64), qh.view(np.uint64))
    fh = _fma_reference(a, b, c)
    assert np.array_equal(f.view(np.uint64), fh.view(np.uint64))


def test_dense_200_every_pivot():
    lp = lpgen.workload("dense_200x200")
    say("dense_200x200: stepping one pivot at a time")
    h, o = step_compare(lp.A, lp.b, lp.c, every=1)
    try:
        assert o.status == oracle.OPTIMAL
    finally:
        lpgpu.lp_destroy(h)
        o.close()
    g = lpgpu.solve(lp.A, lp.b, lp.c)
    assert_same_result(lp.A, lp.b, lp.c, g, oracle.solve(lp.A, lp.b, lp.c))


def test_dense_2000_every_pivot():
    lp = lpgen.workload("dense_2000x2000")
    say("dense_2000x2000: stepping one pivot at a time")
    h, o = step_compare(lp.A, lp.b, lp.c, every=1)
    lpgpu.lp_destroy(h)
    o.close()
    g = lpgpu.solve(lp.A, lp.b, lp.c)
    assert_same_result(lp.A, lp.b, lp.c, g, oracle.solve(lp.A, lp.b, lp.c))


def test_dense_8000_full_solve():
    """The benchmark workload at full size: log, solution and the final tableau."""
    lp = lpgen.workload("dense_8000x8000")
    say("dense_8000x8000: oracle")
    o = oracle.OracleLP(lp.A, lp.b, lp.c)
    o.step(-1)
    ox, oy, oobj = o.extract()
    orow, ocol = o.log()
    say("dense_8000x8000: gpu", o.pivots, "pivots")
    h = lpgpu.lp_create(lp.A, lp.b, lp.c)
    try:
        assert lpgpu.lp_get_info(h).status_readback == 2  # the solution handed over in mapped memory
        t0 = time.perf_counter()
        lpgpu.lp_solve(h)
        wall_ms = 1e3 * (time.perf_counter() - t0)
        res, x, y = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        assert res["status"] == lpgpu.LP_OPTIMAL
        # the device time from the device clock: positive, within the call
        assert 0.0 < res["solve_ms"] < wall_ms, (res["solve_ms"], wall_ms)
        assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
        assert abs(res["objective"] - oobj) <= 1e-9 * max(1.0, abs(oobj))
        assert np.array_equal(x, ox) and np.array_equal(y, oy)
        T = lpgpu.lp_get_tableau(h)
        assert np.array_equal(T, o.tableau())
        del T
        cert = oracle.certificates(lp.A, lp.b, lp.c, x, y, res["objective"])
        assert cert["ok"], cert
        say("dense_8000x8000 solve ms", res["solve_ms"])
    finally:
        lpgpu.lp_destroy(h)
        o.close()


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (15, 15), (16, 16), (31, 33), (63, 64), (64, 63), (65, 65), (127, 129),
          (128, 128), (255, 257), (256, 256), (300, 200), (511, 513), (1023, 100), (100, 1023), (2049, 300),
          (4095, 64), (8191, 20)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_random_shapes_every_pivot(m, n):
    say(f"shape {m}x{n}")
    A, b, c = rand_lp(m * 1000 + n, m, n, 1, 9, signed=True)
    h, o = step_compare(A, b, c, every=1, max_checks=60)
    try:
        if o.status == oracle.RUNNING:
            lpgpu.lp_solve(h)
            o.step(-1)
            assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
        g_res, gx, gy = lpgpu.lp_get_solution(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        ox, oy, oobj = o.extract()
        orow, ocol = o.log()
        assert g_res["status"] == o.status
        assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
        assert np.array_equal(gx, ox) and np.array_equal(gy, oy)
    finally:
        lpgpu.lp_destroy(h)
        o.close()


@pytest.mark.parametrize("seed", range(6))
def test_degenerate_ties(seed):
    """Small integers: exact ties in pricing and in the ratio test."""
    A, b, c = rand_lp(seed, 40 + 7 * seed, 50 + 5 * seed, 1, 3)
    g = lpgpu.solve(A, b, c)
    assert_same_result(A, b, c, g, oracle.solve(A, b, c))


def test_general_row_layout_large_m():
    """m + 1 rows beyond the register-resident form: the general update kernel."""
    A, b, c = rand_lp(77, 9000, 40, 1, 9, signed=True)
    h, o = step_compare(A, b, c, every=3, max_checks=20)
    lpgpu.lp_destroy(h)
    o.close()
    g = lpgpu.solve(A, b, c)
    assert_same_result(A, b, c, g, oracle.solve(A, b, c))


@pytest.mark.parametrize("opts", [dict(cols_per_block=1), dict(cols_per_block=2), dict(cols_per_block=4),
                                  dict(cols_per_block=8), dict(cols_per_block=16),
                                  dict(cols_per_block=1, rows_per_thread=8), dict(cols_per_block=2, rows_per_thread=4),
                                  dict(cols_per_block=16, rows_per_thread=2), dict(rows_per_thread=8),
                                  dict(update_grid_stride=4, update_unroll=2), dict(update_grid_stride=1),
                                  dict(update_grid_stride=8, update_unroll=8, update_block=512),
                                  dict(update_block=128, cols_per_block=2), dict(update_block=1024, cols_per_block=1),
                                  dict(select_workgroups=2), dict(select_workgroups=7), dict(select_workgroups=64),
                                  dict(plain_launches=1), dict(chunk_pivots=1), dict(chunk_pivots=33)])
def test_launch_options_do_not_change_results(opts):
    A, b, c = rand_lp(5, 333, 444, 1, 9, signed=True)
    g = lpgpu.solve(A, b, c, **opts)
    assert_same_result(A, b, c, g, oracle.solve(A, b, c))


def test_unbounded_and_zero_pivot_cases():
    A, b, c = rand_lp(4, 50, 30, 1, 9)
    A[:, 7] = -A[:, 7]
    c[7] = 5000.0
    g = lpgpu.solve(A, b, c)
    assert g["status"] == lpgpu.LP_UNBOUNDED and g["pivots"] == 0
    assert_same_result(A, b, c, g, oracle.solve(A, b, c))
    g = lpgpu.solve(A, b, -np.abs(c))
    assert g["status"] == lpgpu.LP_OPTIMAL and g["pivots"] == 0 and g["objective"] == 0.0


def test_iteration_cap_and_resume():
    A, b, c = rand_lp(8, 120, 150, 1, 9, signed=True)
    full = oracle.solve(A, b, c)
    assert full["pivots"] >= 4
    g = lpgpu.solve(A, b, c, max_pivots=3)
    assert g["status"] == lpgpu.LP_ITER_LIMIT and g["pivots"] == 3
    assert g["rows"].tolist() == full["rows"][:3].tolist()
    h = lpgpu.lp_create(A, b, c)
    try:
        lpgpu.lp_step(h, 2)
        res, _, _ = lpgpu.lp_get_solution(h)
        assert res["status"] == lpgpu.LP_RUNNING and res["pivots"] == 2
        lpgpu.lp_solve(h)
        rows, cols = lpgpu.lp_get_pivots(h)
        assert rows.tolist() == full["rows"].tolist() and cols.tolist() == full["cols"].tolist()
    finally:
        lpgpu.lp_destroy(h)


def test_repeat_solves_are_identical():
    lp = lpgen.dense_lp(31, 700, 900)
    tabs = []
    for _ in range(3):
        h = lpgpu.lp_create(lp.A, lp.b, lp.c)
        lpgpu.lp_solve(h)
        tabs.append(lpgpu.lp_get_tableau(h).copy())
        lpgpu.lp_destroy(h)
    for T in tabs[1:]:
        assert np.array_equal(T.view(np.uint64), tabs[0].view(np.uint64))


def test_torch_buffers_and_device_inputs():
    torch = pytest.importorskip("torch")
    lp = lpgen.dense_lp(12, 500, 600)
    dev = torch.device("cuda", 0)
    dA = torch.from_numpy(lp.A).to(dev)
    db = torch.from_numpy(lp.b).to(dev)
    dc = torch.from_numpy(lp.c).to(dev)
    nbytes = lpgpu.lp_tableau_bytes(500, 600)
    buf = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    h = lpgpu.lp_create_device(500, 600, dA, db, dc, device_buffer=buf, stream=stream)
    try:
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        o = oracle.solve(lp.A, lp.b, lp.c)
        rows, cols = lpgpu.lp_get_pivots(h)
        assert rows.tolist() == o["rows"].tolist()
        assert np.array_equal(x, o["x"])
        info = lpgpu.lp_get_info(h)
        assert info.tableau == buf.data_ptr()
        # rebuild from the same device inputs and solve again
        lpgpu.lp_reload_device(h, dA, db, dc)
        lpgpu.lp_solve(h)
        res2, x2, _ = lpgpu.lp_get_solution(h)
        assert res2["pivots"] == res["pivots"] and np.array_equal(x2, x)
    finally:
        lpgpu.lp_destroy(h)
        torch.cuda.synchronize()


def test_bad_inputs_are_rejected():
    A, b, c = rand_lp(1, 5, 5)
    with pytest.raises(lpgpu.LPError) as e:
        lpgpu.lp_create(A, -b, c)
    assert e.value.code == lpgpu.LP_E_NEG_RHS
    A2 = A.copy()
    A2[1, 1] = np.inf
    with pytest.raises(lpgpu.LPError) as e:
        lpgpu.lp_create(A2, b, c)
    assert e.value.code == lpgpu.LP_E_INVAL
    for bad in (3, 32, 64, -1):
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_create(A, b, c, cols_per_block=bad)
        assert e.value.code == lpgpu.LP_E_INVAL
    for bad in (3, 16, -2):
        with pytest.raises(lpgpu.LPError) as e:
            lpgpu.lp_create(A, b, c, rows_per_thread=bad)
        assert e.value.code == lpgpu.LP_E_INVAL


def test_work_counter_and_kernel_timing():
    """updated_columns counts the columns with a nonzero normalised pivot-row
    entry, pivot by pivot, and timing mode times one update per pivot."""
    A, b, c = rand_lp(21, 150, 170, 1, 9, signed=True)
    h = lpgpu.lp_create(A, b, c, time_kernels=1, chunk_pivots=4)
    o = oracle.OracleLP(A, b, c)
    try:
        total = 0
        for _ in range(12):
            T = o.tableau()
            before = o.pivots
            o.step(1)
            if o.pivots == before:
                break
            r = int(o.log()[0][-1])
            total += int(np.count_nonzero(T[r]))
            lpgpu.lp_step(h, 1)
            t = lpgpu.lp_get_timing(h)
            assert t["pivots"] == o.pivots
            assert t["updated_columns"] == total
            assert t["update_launches"] >= 1 and t["update_ms"] > 0
        lpgpu.lp_solve(h)
        t = lpgpu.lp_get_timing(h)
        o.step(-1)
        assert t["pivots"] == o.pivots
    finally:
        lpgpu.lp_destroy(h)
        o.close()


@pytest.mark.parametrize("opts", [dict(time_kernels=1), dict(time_kernels=1, plain_launches=1)])
def test_timing_mode_keeps_results(opts):
    lp = lpgen.dense_lp(5, 900, 1100)
    g = lpgpu.solve(lp.A, lp.b, lp.c, **opts)
    assert_same_result(lp.A, lp.b, lp.c, g, oracle.solve(lp.A, lp.b, lp.c))


def test_device_inputs_at_any_alignment():
    """A caller's device A may be a view 8 bytes off a 16-byte boundary, with
    an odd or even n: the build reads it either way."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda", 0)
    for m, n in ((300, 400), (301, 401)):
        lp = lpgen.dense_lp(40 + n, m, n)
        flat = torch.empty(m * n + 1, dtype=torch.float64, device=dev)
        flat[1:] = torch.from_numpy(lp.A.ravel()).to(dev)
        dA = flat[1:].view(m, n)
        assert dA.data_ptr() % 16 == 8
        db = torch.from_numpy(lp.b).to(dev)
        dc = torch.from_numpy(lp.c).to(dev)
        h = lpgpu.lp_create_device(m, n, dA, db, dc)
        o = oracle.OracleLP(lp.A, lp.b, lp.c)
        try:
            assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau()), "initial tableau"
            lpgpu.lp_solve(h)
            o.step(-1)
            rows, cols = lpgpu.lp_get_pivots(h)
            orow, ocol = o.log()
            assert rows.tolist() == orow.tolist() and cols.tolist() == ocol.tolist()
            assert np.array_equal(lpgpu.lp_get_tableau(h), o.tableau())
        finally:
            lpgpu.lp_destroy(h)
            o.close()
