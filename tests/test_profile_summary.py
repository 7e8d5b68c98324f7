"""The rocprofv3 summary tool on synthetic CSV output: per-kernel statistics,
the GPU busy fraction (union of kernel intervals), and PMC traffic scaled by
the device copy of known size."""
import os

from paper_2005_14454_amd import profile_summary as ps


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join(str(v) for v in r) + "\n")


def test_trace_statistics_and_busy_fraction(tmp_path):
    d = tmp_path / "trace"
    rows = [
        ('"void ah::(anonymous namespace)::k_step2_tile<float, 64, 8>(x)"', 704, 720896, 0, 4_000_000),
        ('"void ah::(anonymous namespace)::k_step2_tile<float, 64, 8>(x)"', 704, 720896, 4_000_000, 8_000_000),
        ('"void ah::(anonymous namespace)::k_step2_tile<float, 64, 8>(x)"', 704, 1408, 8_000_000, 8_500_000),
        ('"k_fold_batch(y)"', 256, 16384, 9_000_000, 10_000_000),
    ]
    _write(str(d / "host" / "123" / "run_kernel_trace.csv"),
           ["Kernel_Name", "Workgroup_Size", "Grid_Size", "Start_Timestamp", "End_Timestamp"], rows)
    text = ps.trace(str(d), "note", window="k_step2_tile")
    assert "k_step2_tile<float, 64, 8>" in text and "k_fold_batch" in text
    # one row per launch geometry: the two large launches, then the small one
    lines = [l.split() for l in text.splitlines() if l.startswith("k_step2_tile")]
    assert lines[0][-5:] == ["720896", "2", "4.0000", "4.0000", "4.0000"]
    assert lines[1][-5:] == ["1408", "1", "0.5000", "0.5000", "0.5000"]
    assert "GPU busy (union of kernel intervals) 0.950 of 0.01 s" in text
    assert "GPU busy between the first and last k_step2_tile: 1.000" in text
    assert ps.busy_fraction([(0, 10), (5, 20), (30, 40)])[0] == 0.75
    # stretches with no kernel: only those of at least the given length
    assert ps.idle_gaps([(0, 10), (5, 20), (30, 40), (2_000_000_040, 2_000_000_050)], 1.0) == [(40e-9, 2.0)]


def test_traffic_is_scaled_by_the_copy(tmp_path):
    gib = 1 << 30
    fetch, write = tmp_path / "f", tmp_path / "w"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy moves 1 GiB each way; FETCH_SIZE reads half, WRITE_SIZE all of it
    _write(str(fetch / "a" / "run_counter_collection.csv"), hdr,
           [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", gib / 1024 / 2),
            (2, '"k_step2_tile<float, 64, 8>(int)"', "FETCH_SIZE", 1000.0)])
    _write(str(write / "a" / "run_counter_collection.csv"), hdr,
           [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", gib / 1024),
            (2, '"k_step2_tile<float, 64, 8>(int)"', "WRITE_SIZE", 3000.0)])
    text = ps.traffic(str(fetch), str(write), N=8, copy_bytes=gib)
    assert "fetch factor 2.0000, write factor 1.0000" in text
    row = [l for l in text.splitlines() if l.startswith("k_step2_tile")][0].split()
    # read 2 x 1000 KiB, write 3000 KiB; algorithmic 40 B per site for 8^3 sites
    assert row[-5:] == [f"{2000 * 1024 / 1e9:.3f}", f"{3000 * 1024 / 1e9:.3f}", f"{5000 * 1024 / 1e9:.3f}",
                        f"{40 * 4 * 512 / 1e9:.3f}", "1"]


def test_counters_mean_and_valu_per_site_update(tmp_path):
    d = tmp_path / "c"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # two dispatches of a two-step launch on a 4^3 lattice: 128 site-updates each
    _write(str(d / "a" / "run_counter_collection.csv"), hdr,
           [(1, '"k_step2_tile<float, 64, 8>(x)"', "SQ_INSTS_VALU", 100.0),
            (1, '"k_step2_tile<float, 64, 8>(x)"', "SQ_WAVES", 4.0),
            (2, '"k_step2_tile<float, 64, 8>(x)"', "SQ_INSTS_VALU", 300.0),
            (2, '"k_step2_tile<float, 64, 8>(x)"', "SQ_WAVES", 4.0)])
    text = ps.counters(str(d), N=4)
    row = [l for l in text.splitlines() if l.startswith("k_step2_tile")][0].split()
    # mean 200 wave instructions x 64 lanes / 128 site-updates
    assert row[-4:] == ["2", "200", "4", f"{200 * 64 / 128:.1f}"]
