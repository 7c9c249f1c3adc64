"""Host-side arithmetic the kernels rely on, checked on the CPU."""

import numpy as np


def magic(nvec):
    return ((1 << 36) + nvec - 1) // nvec


def test_item_split_by_reciprocal_is_exact():
    """(item * ceil(2^36/nvec)) >> 36 == item // nvec for item < 2^24, nvec < 2^12."""
    rng = np.random.default_rng(0)
    for nvec in list(range(1, 300)) + [int(v) for v in rng.integers(300, 4096, 200)] + [4095]:
        mg = magic(nvec)
        items = np.concatenate([np.arange(0, 5000), rng.integers(0, 1 << 24, 5000),
                                np.array([(1 << 24) - 1, nvec * 4096 - 1])]).astype(np.uint64)
        items = items[items < (1 << 24)]
        got = (items.astype(object) * mg) >> 36
        assert all(int(g) == int(i) // nvec for g, i in zip(got, items))


def test_multiples_and_neighbours():
    for nvec in (1, 2, 3, 7, 33, 257, 1025, 2049, 4095):
        mg = magic(nvec)
        for q in (0, 1, 2, 100, ((1 << 24) - 1) // nvec):
            for it in (q * nvec - 1, q * nvec, q * nvec + nvec - 1):
                if 0 <= it < (1 << 24):
                    assert (it * mg) >> 36 == it // nvec
