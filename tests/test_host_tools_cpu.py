"""Host-side measurement logic on the CPU: the calibration of rocprofv3
FETCH_SIZE / WRITE_SIZE counters against a copy of known size, kernel-trace
statistics, and bench.py's algorithmic byte model of the five passes."""

import csv
import os

import pytest

from paper_2505_22313_amd import profiling as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_calibration(tmp_path):
    """A copy of 4 GiB that FETCH_SIZE reports at half and WRITE_SIZE in full
    gives factors 2 and 1; a pass kernel's per-dispatch average is scaled by
    them.  Only the largest copy dispatch calibrates."""
    kib = 4 * 1024 ** 3 / 1024
    copy = "__amd_rocclr_copyBuffer"
    pass_c = "void dop::k_pass_c<16>(dop::KParams)"
    write_counters(tmp_path / "f", [(copy, "FETCH_SIZE", 16.0), (copy, "FETCH_SIZE", kib / 2),
                                    (pass_c, "FETCH_SIZE", 1000.0), (pass_c, "FETCH_SIZE", 3000.0)])
    write_counters(tmp_path / "w", [(copy, "WRITE_SIZE", 4.0), (copy, "WRITE_SIZE", kib),
                                    (pass_c, "WRITE_SIZE", 500.0), (pass_c, "WRITE_SIZE", 500.0)])
    t = pr.traffic(str(tmp_path / "f"), str(tmp_path / "w"))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    k = t["kernels"]["pass_c"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert k["write_bytes"] == pytest.approx(500.0 * 1024)
    assert k["traffic_bytes"] == pytest.approx(k["fetch_bytes"] + k["write_bytes"])
    assert t["source_sha"] == pr.kernel_source_hash()


def test_traffic_needs_calibration_copy(tmp_path):
    write_counters(tmp_path / "f", [("void dop::k_pass_c<16>(dop::KParams)", "FETCH_SIZE", 1.0)])
    write_counters(tmp_path / "w", [("void dop::k_pass_c<16>(dop::KParams)", "WRITE_SIZE", 1.0)])
    with pytest.raises(RuntimeError):
        pr.traffic(str(tmp_path / "f"), str(tmp_path / "w"))


def test_pass_names_and_stats(tmp_path):
    assert pr.pass_name("void dop::k_pass_a_fwd<16, 0>(dop::KParams)") == "pass_a_fwd"
    assert pr.pass_name("void dop::k_pass_b_inv<105>(dop::KParams)") == "pass_b_inv"
    assert pr.pass_name("__amd_rocclr_copyBuffer") is None
    os.makedirs(tmp_path / "t")
    with open(tmp_path / "t" / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "k", "Calls": 93, "AverageNs": 15_793_000, "MinNs": 15_629_000,
                    "MaxNs": 15_987_000, "Percentage": 32.1})
    (row,) = pr.stats(str(tmp_path / "t"))
    assert row["calls"] == 93 and row["avg_ms"] == pytest.approx(15.793)


def test_bench_byte_model():
    """51 B per padded pixel and wavelength at N = M/2 in steady state (the
    first wavelength writes the PSF without reading it).  With N = M nothing
    is pruned: the field moves 64 B (A writes, A' reads, B, C, B' read and
    write), h adds 4 B and the PSF read-modify-write 8 B."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    m = 65536
    steady = bench.pass_bytes(m // 2, m, k_first=False)
    first = bench.pass_bytes(m // 2, m, k_first=True)
    assert sum(steady.values()) / m ** 2 == pytest.approx(51.0)
    assert sum(steady.values()) - sum(first.values()) == pytest.approx(4.0 * (m // 2) ** 2)
    full = bench.pass_bytes(m, m, k_first=False)
    assert sum(full.values()) / m ** 2 == pytest.approx(64.0 + 4.0 + 8.0)


def test_bench_group_byte_model():
    """Wavelength groups: pass A reads h once per group and pass A' touches
    the PSF once per group; one group per wavelength is the per-wavelength
    accounting (the first wavelength writes the PSF without reading it)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    n, m, k = 32768, 65536, 31
    per = bench.step_pass_bytes(n, m, k, k)
    steady = bench.pass_bytes(n, m, k_first=False)
    first = bench.pass_bytes(n, m, k_first=True)
    for name in per:
        assert per[name] == pytest.approx(first[name] + (k - 1) * steady[name])
    grouped = bench.step_pass_bytes(n, m, k, 8)  # 7 groups of 4 and one of 3
    saved = sum(per.values()) - sum(grouped.values())
    assert saved == pytest.approx((k - 8) * (4.0 * n * n + 8.0 * n * n))
    assert sum(grouped.values()) / (k * float(m) * m) == pytest.approx(48.74, abs=0.01)
    # rectangular: rows x columns
    r = bench.step_pass_bytes((300, 200), (720, 240), 2, 1)
    assert r["pass_a_fwd"] == pytest.approx(2 * 8.0 * 300 * 240 + 4.0 * 300 * 200)
    assert r["pass_c"] == pytest.approx(2 * 2 * 8.0 * 720 * 240)
