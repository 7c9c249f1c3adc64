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


def test_profile_summary_tables(tmp_path):
    """The rocprofv3 CSV summaries: per-kernel stats, per-grid averages from
    the kernel trace, and counter averages over dispatches above a floor."""
    from paper_2211_10979_amd import profile_summary as ps

    (tmp_path / "run_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"lpgpu::k_a<256>(double*)",3,300000,100000,90.0,50000,150000,1.0\n')
    (tmp_path / "run_kernel_trace.csv").write_text(
        '"Kernel_Name","Start_Timestamp","End_Timestamp","Grid_Size_X","Grid_Size_Y","Grid_Size_Z"\n'
        '"lpgpu::k_a<256>(double*)",0,150000,1024,1,1\n'
        '"lpgpu::k_a<256>(double*)",0,50000,64,1,1\n'
        '"lpgpu::k_a<256>(double*)",0,100000,1024,1,1\n')
    (tmp_path / "run_counter_collection.csv").write_text(
        '"Kernel_Name","Counter_Name","Counter_Value"\n'
        '"lpgpu::k_a<256>(double*)","FETCH_SIZE",10.0\n'
        '"lpgpu::k_a<256>(double*)","FETCH_SIZE",1000.0\n'
        '"lpgpu::k_a<256>(double*)","FETCH_SIZE",3000.0\n')
    text = ps.summarize(str(tmp_path), kernel="k_a", min_value=100.0, by_grid=True)
    assert "| lpgpu::k_a<256> | 3 | 300.0 | 100.00 | 50.00 | 150.00 |" in text
    assert "| lpgpu::k_a<256> | 1024 | 2 | 125.00 | 100.00 | 150.00 |" in text
    assert "| lpgpu::k_a<256> | 64 | 1 | 50.00 | 50.00 | 50.00 |" in text
    assert "| lpgpu::k_a<256> | FETCH_SIZE | 2 | 2000.0 |" in text
