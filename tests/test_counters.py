"""Counter calibration of paper_1811_07717_amd.counters on a synthetic
rocprofv3 counter file: bytes = FETCH_SIZE x (true read / counted read of the
copy) + WRITE_SIZE x (true write / counted write of the copy)."""
import csv

from paper_1811_07717_amd import counters

HEAD = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, val) in enumerate(rows):
            w.writerow([i, name, "X", val])


def test_calibration_and_traffic_file(tmp_path):
    spmm = "void (anonymous namespace)::k_spmm<32, 2, double, double, true>(Geom, ...)"
    upd = "void (anonymous namespace)::k_update<32, 2, double>(Geom, ...)"
    copy = "zi::(anonymous namespace)::k_copy2(double2 const*, double2*, unsigned long)"
    # the copy moves 1 MiB each way; FETCH counts half of it, WRITE all of it
    _write(tmp_path / "f.csv", [(copy, 512.0), (spmm, 100.0), (spmm, 300.0), (upd, 50.0),
                                (upd, 50.0)])
    _write(tmp_path / "w.csv", [(copy, 1024.0), (spmm, 10.0), (spmm, 30.0), (upd, 5.0),
                                (upd, 5.0)])
    res, ff, wf = counters.summarize(tmp_path / "f.csv", tmp_path / "w.csv", copy_mib=1.0)
    assert ff == 2.0 and wf == 1.0
    assert res["spmm_pq"]["launches"] == 2 and res["spmm_pq"]["slabs"] == 1
    assert res["spmm_pq"]["bytes_per_launch"] == int((200.0 * 2 + 20.0) * 1024)
    assert res["update"]["bytes_per_launch"] == int((50.0 * 2 + 5.0) * 1024)
    # an SpMM run as two slab launches per product (one update per product)
    _write(tmp_path / "f2.csv", [(copy, 512.0), (spmm, 100.0), (spmm, 300.0), (upd, 50.0)])
    _write(tmp_path / "w2.csv", [(copy, 1024.0), (spmm, 10.0), (spmm, 30.0), (upd, 5.0)])
    res, _, _ = counters.summarize(tmp_path / "f2.csv", tmp_path / "w2.csv", copy_mib=1.0)
    assert res["spmm_pq"]["slabs"] == 2
    assert res["spmm_pq"]["bytes_per_launch"] == 2 * int((200.0 * 2 + 20.0) * 1024)
    assert "copy" not in res


def test_source_hash_is_stable():
    assert counters.source_hash() == counters.source_hash()
    assert len(counters.source_hash()) == 16


def test_phase_gaps(tmp_path):
    # two phases cut at a marker; overlapping kernels count once as busy
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerow(["k_a", 0, 10_000])
        w.writerow(["k_b", 5_000, 20_000])        # overlaps k_a
        w.writerow(["k_c", 80_000, 90_000])       # after a 60 us gap
        w.writerow(["zi::k_copy2(x)", 100_000, 101_000])
        w.writerow(["k_d", 200_000, 210_000])
    ph = counters.phase_gaps(str(path))
    assert len(ph) == 2
    assert ph[0]["span_us"] == 90.0 and ph[0]["busy_us"] == 30.0 and ph[0]["idle_us"] == 60.0
    assert ph[0]["dispatches"] == 3 and ph[0]["gaps_over_50us"] == 1
    assert ph[0]["longest_gaps_us"] == [60.0]
    assert ph[1]["busy_us"] == 10.0 and ph[1]["idle_us"] == 0.0


def test_ring_kernels_are_classified(tmp_path):
    ring = "void (anonymous namespace)::k_spmm_ring<double, true>(Geom, int const*)"
    ringf = "void (anonymous namespace)::k_spmm_ring<float, false>(Geom, int const*)"
    front = "void (anonymous namespace)::k_spmm_sr<8, 1>(Geom, int const*)"
    upd = "void (anonymous namespace)::k_update<32, 2, double>(Geom, ...)"
    copy = "zi::(anonymous namespace)::k_copy2(double2 const*, double2*, unsigned long)"
    rows = [(copy, 512.0), (ring, 100.0), (ringf, 40.0), (front, 7.0), (upd, 50.0)]
    _write(tmp_path / "f.csv", rows)
    _write(tmp_path / "w.csv", rows)
    res = counters.per_kernel(tmp_path / "f.csv", "ring")
    assert res["spmm_sr"] == (100.0, 1) and res["spmm_pq"] == (40.0, 1)
    res = counters.per_kernel(tmp_path / "f.csv", "8, 1")
    assert res["spmm_sr"] == (7.0, 1) and "spmm_pq" not in res
