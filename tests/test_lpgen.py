"""The seeded input generator: published SplitMix64 outputs, ranges, determinism."""

import hashlib

import numpy as np

from paper_2211_10979_amd import lpgen


def test_splitmix64_published_vector():
    # SplitMix64 started from state 0: the first outputs published with the
    # algorithm (used to seed the xoshiro family).
    got = [int(v) for v in lpgen.Stream(0).raw(4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_block_draws_equal_sequential_draws():
    s1 = lpgen.Stream(12345)
    whole = s1.raw(1000)
    s2 = lpgen.Stream(12345)
    parts = np.concatenate([s2.raw(1), s2.raw(499), s2.raw(500)])
    assert np.array_equal(whole, parts)
    assert int(whole[0]) == lpgen.mix64(12345 + lpgen.GOLDEN)


def test_dense_lp_ranges_and_determinism():
    lp = lpgen.dense_lp(1, 37, 53)
    for arr in (lp.A, lp.b, lp.c):
        assert arr.dtype == np.float64
        assert arr.min() >= 1 and arr.max() <= 1000
        assert np.array_equal(arr, np.round(arr))
    lp2 = lpgen.dense_lp(1, 37, 53)
    assert np.array_equal(lp.A, lp2.A) and np.array_equal(lp.b, lp2.b) and np.array_equal(lp.c, lp2.c)
    assert not np.array_equal(lpgen.dense_lp(2, 37, 53).A, lp.A)
    assert not np.array_equal(lpgen.dense_lp(1, 37, 53, k=1).A, lp.A)


def test_draw_order_a_then_b_then_c():
    m, n = 5, 4
    lp = lpgen.dense_lp(7, m, n)
    s = lpgen.lp_stream(7, 0)
    v = s.integers(m * n + m + n, 1, 1000).astype(np.float64)
    assert np.array_equal(lp.A.ravel(), v[: m * n])
    assert np.array_equal(lp.b, v[m * n: m * n + m])
    assert np.array_equal(lp.c, v[m * n + m:])


def test_uniform_histogram():
    v = lpgen.Stream(99).integers(200_000, 1, 1000)
    counts = np.bincount(v, minlength=1001)[1:]
    assert counts.min() > 120 and counts.max() < 290  # mean 200


def test_batch_and_trace_sizes():
    sizes = lpgen.batch_sizes(lpgen.BATCH_SEED, 512)
    arr = np.array(sizes)
    assert arr.min() >= 32 and arr.max() <= 512
    assert len(set(sizes)) > 400
    tsizes, gaps = lpgen.trace_sizes(lpgen.TRACE_SEED, 2000)
    t = np.array(tsizes)
    assert t.min() >= 64 and t.max() <= 4096
    lg = np.log2(t / 64.0) / 6.0
    assert abs(lg.mean() - 0.5) < 0.03  # log-uniform
    assert abs(gaps.mean() - 1.0) < 0.08 and gaps.min() >= 0


def test_workload_fingerprint_stable():
    lp = lpgen.workload("dense_200x200")
    h = hashlib.sha256(lp.A.tobytes() + lp.b.tobytes() + lp.c.tobytes()).hexdigest()
    lp2 = lpgen.workload("dense_200x200")
    assert h == hashlib.sha256(lp2.A.tobytes() + lp2.b.tobytes() + lp2.c.tobytes()).hexdigest()
    assert lp.A[0, :3].tolist() == lpgen.dense_lp(1, 200, 200).A[0, :3].tolist()


def test_parallel_values_equal_sequential_rejection_path():
    for count in (1, 1000, (1 << 20) * 3 + 17):
        a = lpgen.Stream(2024).values(count, 1, 1000)
        b = lpgen.Stream(2024).integers(count, 1, 1000).astype(np.float64)
        assert np.array_equal(a, b)


def test_rejection_path_is_taken_when_a_draw_is_rejected():
    # span 3 * 2^62: a draw is rejected with probability 1/4, so the exact
    # sequential path must be used and must agree with integers()
    span = 3 << 62
    a = lpgen.Stream(7).values(5000, 0, span - 1)
    b = lpgen.Stream(7).integers(5000, 0, span - 1).astype(np.float64)
    assert np.array_equal(a, b)


def _numpy_draws(fn):
    """Runs fn with the numpy draws (the C build switched off)."""
    saved = lpgen._NATIVE
    lpgen._NATIVE = False
    try:
        return fn()
    finally:
        lpgen._NATIVE = saved


def test_native_draws_equal_numpy_draws():
    if lpgen._native() is None:
        import pytest

        pytest.skip("liblpgen.so not built")
    for seed, m, n, k in ((1, 37, 53, 0), (5, 300, 7, 12), (3, 1, 1, 9), (4, 513, 64, 511)):
        a = lpgen.dense_lp(seed, m, n, k=k)
        b = _numpy_draws(lambda: lpgen.dense_lp(seed, m, n, k=k))
        assert np.array_equal(a.A, b.A) and np.array_equal(a.b, b.b) and np.array_equal(a.c, b.c)
    # a span that rejects about one draw in 16: same values and the same
    # stream position afterwards (the next draws agree too)
    lo, hi = 0, 3 << 60
    s1 = lpgen.Stream(77)
    v1 = np.concatenate([s1.values(4000, lo, hi), s1.values(10, 1, 1000)])
    v2 = _numpy_draws(lambda: (lambda s: np.concatenate([s.values(4000, lo, hi), s.values(10, 1, 1000)]))(
        lpgen.Stream(77)))
    assert np.array_equal(v1, v2)
    assert s1.drawn > 4010  # some draws were rejected
