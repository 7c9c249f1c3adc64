"""GPU parity of the batched solver: every LP of a batch follows exactly the
pivot sequence of the CPU oracle (and of the single-LP solver), whatever the
kernel shape and the mix of sizes and outcomes."""

import os
import sys
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


def mixed_lps(seed, count, lo=1, hi=130):
    """Uneven sizes and every outcome: optimal, unbounded, no pivot."""
    rng = np.random.default_rng(seed)
    lps = []
    for k in range(count):
        m, n = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        kind = k % 5
        if kind == 0:
            lp = lpgen.dense_lp(seed, m, n, k=k)
            A, b, c = lp.A, lp.b, lp.c
        else:
            A = rng.integers(1, 10, size=(m, n)).astype(float)
            if kind in (1, 2):
                A *= rng.choice([-1.0, 1.0], size=(m, n), p=[0.3, 0.7])
            b = rng.integers(1, 10, size=m).astype(float)
            c = rng.integers(1, 10, size=n).astype(float)
            if kind == 3:
                c = -c  # optimal at the origin: no pivot
        lps.append((A, b, c))
    return lps


def check_batch(h, lps):
    for k, (A, b, c) in enumerate(lps):
        m, n = A.shape
        res, x, y = lpgpu.lp_batch_get_solution(h, k, m, n)
        rows, cols = lpgpu.lp_batch_get_pivots(h, k)
        o = oracle.solve(A, b, c)
        assert res["status"] == o["status"], k
        assert res["pivots"] == o["pivots"], k
        assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist(), k
        assert np.array_equal(x, o["x"]) and np.array_equal(y, o["y"]), k
        assert abs(res["objective"] - o["objective"]) <= 1e-9 * max(1.0, abs(o["objective"])), k
        if o["status"] == oracle.OPTIMAL:
            assert oracle.certificates(A, b, c, x, y, res["objective"])["ok"], k


def test_batch_mixed_sizes_and_outcomes():
    lps = mixed_lps(3, 80)
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        check_batch(h, lps)
    finally:
        lpgpu.lp_batch_destroy(h)


def test_batch_workload_512():
    """The 512-LP workload: m, n uniform on [32, 512], generator LPs."""
    sizes = lpgen.batch_sizes(lpgen.BATCH_SEED, 512)
    lps = [(lp.A, lp.b, lp.c) for lp in (lpgen.dense_lp(lpgen.BATCH_SEED, m, n, k=k)
                                         for k, (m, n) in enumerate(sizes))]
    say("batch of 512: create")
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        say("batch of 512 solved in", lpgpu.lp_batch_solve_ms(h), "ms")
        check_batch(h, lps)
    finally:
        lpgpu.lp_batch_destroy(h)


@pytest.mark.parametrize("block,unroll", [(256, 1), (256, 2), (256, 4), (256, 8), (512, 1), (512, 2), (512, 4),
                                          (1024, 1), (1024, 2), (1024, 4)])
def test_every_kernel_shape_gives_the_same_pivots(block, unroll):
    lps = mixed_lps(11, 30, 1, 300)
    h = lpgpu.lp_batch_create(lps, batch_block=block, batch_unroll=unroll)
    try:
        assert lpgpu.lp_batch_get_shape(h)["block"] == block
        lpgpu.lp_batch_solve(h)
        check_batch(h, lps)
    finally:
        lpgpu.lp_batch_destroy(h)


def test_batch_equals_solo_solver_bitwise():
    lps = mixed_lps(5, 12, 100, 400)
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        for k, (A, b, c) in enumerate(lps):
            g = lpgpu.solve(A, b, c)
            res, x, y = lpgpu.lp_batch_get_solution(h, k, *A.shape)
            assert np.array_equal(x.view(np.uint64), g["x"].view(np.uint64))
            assert np.array_equal(y, g["y"])
            assert res["objective"] == g["objective"]
    finally:
        lpgpu.lp_batch_destroy(h)


def test_reset_and_resolve_are_identical():
    lps = mixed_lps(7, 20)
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        first = [lpgpu.lp_batch_get_solution(h, k, *A.shape) for k, (A, _, _) in enumerate(lps)]
        lpgpu.lp_batch_reset(h)
        lpgpu.lp_batch_solve(h)
        for k, (A, _, _) in enumerate(lps):
            r2, x2, y2 = lpgpu.lp_batch_get_solution(h, k, *A.shape)
            assert r2["pivots"] == first[k][0]["pivots"] and np.array_equal(x2, first[k][1])
    finally:
        lpgpu.lp_batch_destroy(h)


def test_iteration_cap_in_batch():
    lps = mixed_lps(9, 10, 40, 80)
    h = lpgpu.lp_batch_create(lps, max_pivots=2)
    try:
        lpgpu.lp_batch_solve(h)
        for k, (A, b, c) in enumerate(lps):
            res, _, _ = lpgpu.lp_batch_get_solution(h, k, *A.shape)
            o = oracle.solve(A, b, c, max_pivots=2)
            assert res["status"] == o["status"] and res["pivots"] == o["pivots"]
    finally:
        lpgpu.lp_batch_destroy(h)


def test_autotuner_writes_and_reuses_its_cache(monkeypatch):
    lps = mixed_lps(13, 40, 20, 200)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        h = lpgpu.lp_batch_create(lps)
        try:
            best = lpgpu.lp_batch_autotune(h, path, trials=1)
            shape = lpgpu.lp_batch_get_shape(h)
            assert best > 0
            lpgpu.lp_batch_solve(h)
            check_batch(h, lps)
        finally:
            lpgpu.lp_batch_destroy(h)
        line = open(path).read().strip().splitlines()[-1]
        assert f'"block": {shape["block"]}' in line and '"key": "batch/count64/m256/n256"' in line
        monkeypatch.setenv("LP_AUTOTUNE_CACHE", path)
        h2 = lpgpu.lp_batch_create(lps)
        try:
            assert lpgpu.lp_batch_get_shape(h2) == shape
        finally:
            lpgpu.lp_batch_destroy(h2)


def test_lp_beyond_the_lds_limit_uses_a_global_work_area():
    """F, R and the list of a 3300 x 3300 LP exceed 64 KiB: that LP keeps them
    in global memory, next to LPs that use LDS, with the same pivots."""
    big = lpgen.dense_lp(17, 3300, 3300)
    lps = [(big.A, big.b, big.c)] + mixed_lps(19, 5, 20, 200)
    say("batch with a 3300 x 3300 LP")
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_solve(h)
        check_batch(h, lps)
    finally:
        lpgpu.lp_batch_destroy(h)


# Shapes that split large LPs over several workgroups (block, unroll,
# workgroups per CU, most parts per LP).
SPLIT_SHAPES = [(256, 2, 2, 8), (512, 2, 2, 4), (512, 2, 2, 8), (1024, 2, 1, 4), (1024, 2, 1, 8), (1024, 4, 1, 4),
                (1024, 4, 1, 8)]


def heavy_mix(seed):
    """A few large LPs among many small ones: the large ones get split."""
    big = [lpgen.dense_lp(seed, m, n, k=k) for k, (m, n) in enumerate([(480, 500), (450, 470), (400, 512), (300, 350)])]
    return [(lp.A, lp.b, lp.c) for lp in big] + mixed_lps(seed + 1, 60, 10, 120)


@pytest.mark.parametrize("shape", SPLIT_SHAPES)
def test_split_lps_follow_the_oracle(shape):
    """Each part of a split LP rewrites a share of its columns and the parts
    meet twice per pivot: pivots, x, y as the oracle's, again after a reset."""
    lps = heavy_mix(29)
    say(f"split shape {shape}")
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_set_shape(h, *shape)
        sp = lpgpu.lp_batch_get_split(h)
        assert sp["max_parts"] == shape[3] and sp["split_lps"] >= 4, sp
        assert sp["queue_entries"] >= len(lps) + 4, sp
        lpgpu.lp_batch_solve(h)
        check_batch(h, lps)
        lpgpu.lp_batch_reset(h)
        lpgpu.lp_batch_solve(h)
        check_batch(h, lps)
    finally:
        lpgpu.lp_batch_destroy(h)


def test_split_batch_equals_whole_batch_bitwise():
    """The 512-LP workload with its largest LPs split gives the bits of the
    batch without splitting, LP by LP."""
    sizes = lpgen.batch_sizes(lpgen.BATCH_SEED, 512)
    lps = [(lp.A, lp.b, lp.c) for lp in (lpgen.dense_lp(lpgen.BATCH_SEED, m, n, k=k)
                                         for k, (m, n) in enumerate(sizes))]
    h = lpgpu.lp_batch_create(lps)
    try:
        lpgpu.lp_batch_set_shape(h, 1024, 2, 1, 1)
        lpgpu.lp_batch_solve(h)
        whole = [lpgpu.lp_batch_get_solution(h, k, *A.shape) for k, (A, _, _) in enumerate(lps)]
        logs = [lpgpu.lp_batch_get_pivots(h, k) for k in range(len(lps))]
        for shape in ((1024, 2, 1, 8), (512, 2, 2, 4)):
            say(f"batch of 512, split shape {shape}")
            lpgpu.lp_batch_set_shape(h, *shape)
            assert lpgpu.lp_batch_get_split(h)["split_lps"] > 0
            lpgpu.lp_batch_reset(h)
            lpgpu.lp_batch_solve(h)
            for k, (A, _, _) in enumerate(lps):
                res, x, y = lpgpu.lp_batch_get_solution(h, k, *A.shape)
                rows, cols = lpgpu.lp_batch_get_pivots(h, k)
                assert res["status"] == whole[k][0]["status"] and res["pivots"] == whole[k][0]["pivots"], k
                assert rows.tolist() == logs[k][0].tolist() and cols.tolist() == logs[k][1].tolist(), k
                assert np.array_equal(x.view(np.uint64), whole[k][1].view(np.uint64)), k
                assert np.array_equal(y.view(np.uint64), whole[k][2].view(np.uint64)), k
    finally:
        lpgpu.lp_batch_destroy(h)


def test_split_gate_closed_runs_the_lp_whole():
    """decide_spin = -1 closes every split LP's check-in gate at once: the
    workgroup that closed it runs the LP alone, the other parts leave."""
    lps = heavy_mix(31)
    h = lpgpu.lp_batch_create(lps, decide_spin=-1)
    try:
        lpgpu.lp_batch_set_shape(h, 1024, 2, 1, 8)
        assert lpgpu.lp_batch_get_split(h)["split_lps"] >= 4
        for _ in range(2):  # the gates reopen for the next solve
            lpgpu.lp_batch_solve(h)
            check_batch(h, lps)
            lpgpu.lp_batch_reset(h)
    finally:
        lpgpu.lp_batch_destroy(h)


def test_set_shape_rejects_unknown_shapes():
    lps = mixed_lps(33, 4)
    h = lpgpu.lp_batch_create(lps)
    try:
        with pytest.raises(lpgpu.LPError):
            lpgpu.lp_batch_set_shape(h, 1024, 2, 1, 3)
        with pytest.raises(lpgpu.LPError):
            lpgpu.lp_batch_set_shape(h, 768, 2, 1, 1)
        lpgpu.lp_batch_set_shape(h, 256, 1, 2, 1)
        assert lpgpu.lp_batch_get_split(h) == dict(max_parts=1, split_lps=0, queue_entries=len(lps))
    finally:
        lpgpu.lp_batch_destroy(h)


def test_split_lps_stop_like_the_oracle():
    """Split LPs that end unbounded, at the iteration cap, or at once (no
    pivot), beside whole ones: status, pivots and log as the oracle's."""
    rng = np.random.default_rng(37)
    lps = []
    for k, (m, n) in enumerate([(460, 500), (430, 480), (500, 420), (380, 450)]):
        A = rng.integers(1, 10, size=(m, n)).astype(float)
        if k % 2 == 0:
            A *= rng.choice([-1.0, 1.0], size=(m, n), p=[0.4, 0.6])  # often unbounded
        b = rng.integers(1, 10, size=m).astype(float)
        c = rng.integers(1, 10, size=n).astype(float)
        if k == 3:
            c = -c  # optimal at the origin: no pivot
        lps.append((A, b, c))
    lps += mixed_lps(39, 40, 10, 100)
    for cap in (None, 3):
        kw = {} if cap is None else dict(max_pivots=cap)
        say(f"split LPs, stops, cap {cap}")
        h = lpgpu.lp_batch_create(lps, **kw)
        try:
            lpgpu.lp_batch_set_shape(h, 1024, 2, 1, 8)
            assert lpgpu.lp_batch_get_split(h)["split_lps"] >= 3
            lpgpu.lp_batch_solve(h)
            for k, (A, b, c) in enumerate(lps):
                res, x, y = lpgpu.lp_batch_get_solution(h, k, *A.shape)
                rows, cols = lpgpu.lp_batch_get_pivots(h, k)
                o = oracle.solve(A, b, c, **kw)
                assert res["status"] == o["status"] and res["pivots"] == o["pivots"], (k, res, o["status"])
                assert rows.tolist() == o["rows"].tolist() and cols.tolist() == o["cols"].tolist(), k
        finally:
            lpgpu.lp_batch_destroy(h)
