"""Host logic of bench.py: kernel naming, the counter summaries built from
rocprofv3 --pmc CSV files (calibrated HBM bytes, SQ/TCC/TCP ratios), the
source-hash gate on stored traffic figures and the one-GPU guard. No GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

K2_INV = "void fftb::k2r_kernel<1, double, 18, 8, false, false, 16, true, 8, 2>(fftb::KArgs)"
K2_FWD = "void fftb::k2r_kernel<-1, double, 18, 8, false, true, 8, true, 8, 1>(fftb::KArgs)"
K1_INV = "void fftb::k1b_kernel<1, double, 45, 4>(fftb::KArgs)"
K1_FWD = "void fftb::k1b_kernel<-1, float, 45, 4>(fftb::KArgs)"
K3 = "void fftb::k3r_kernel<double>(fftb::KArgs)"
COPY = "__amd_rocclr_copyBuffer"


def test_kernel_ids():
    assert bench.kernel_id(K2_INV) == "plane_inverse"
    assert bench.kernel_id(K2_FWD) == "plane_forward"
    assert bench.kernel_id(K1_INV) == "column_inverse"
    assert bench.kernel_id(K1_FWD) == "column_forward"
    assert bench.kernel_id(K3) == "combine_forward"
    assert bench.kernel_id("void fftb::k1r_kernel<-1, double, 16, 8>(fftb::KArgs)") == "column_forward"
    assert bench.kernel_id(COPY) is None


def write_pmc(d, rows):
    """rows: (dispatch, kernel, counter, value, start_ns, end_ns)."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)


def test_summarize_counters_calibration(tmp_path, monkeypatch):
    # the copy reads FETCH 0.5 GiB and WRITE 1 GiB for a 1 GiB copy: factors 2 and 1
    gib_kib = 1 << 20
    write_pmc(tmp_path / "cf", [(1, COPY, "FETCH_SIZE", gib_kib / 2, 0, 1)])
    write_pmc(tmp_path / "cw", [(1, COPY, "WRITE_SIZE", gib_kib, 0, 1)])
    # two launches of the inverse plane kernel, one of the combine
    write_pmc(tmp_path / "f", [(1, K2_INV, "FETCH_SIZE", 1000, 0, 1), (2, K2_INV, "FETCH_SIZE", 3000, 0, 1),
                               (3, K3, "FETCH_SIZE", 500, 0, 1), (4, COPY, "FETCH_SIZE", 7, 0, 1)])
    write_pmc(tmp_path / "w", [(1, K2_INV, "WRITE_SIZE", 4000, 0, 1), (2, K2_INV, "WRITE_SIZE", 6000, 0, 1),
                               (3, K3, "WRITE_SIZE", 100, 0, 1)])
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")

    class A:
        workload = "wl"
        summarize_counters = [str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw")]

    bench.summarize_counters(A)
    d = json.load(open(tmp_path / "profiles" / "traffic.json"))["wl"]
    assert d["fetch_factor"] == pytest.approx(2.0) and d["write_factor"] == pytest.approx(1.0)
    # mean per dispatch: fetch 2000 KiB x 2 + write 5000 KiB x 1
    assert d["bytes_per_launch"]["plane_inverse"] == pytest.approx((2000 * 2 + 5000) * 1024.0)
    assert d["bytes_per_launch"]["combine_forward"] == pytest.approx((500 * 2 + 100) * 1024.0)
    assert set(d["bytes_per_launch"]) == {"plane_inverse", "combine_forward"}
    # the stored figure is used only on the kernel source it was taken on
    assert bench.traffic_from_profiles("wl", "abc", "plane_inverse") == pytest.approx(9000 * 1024.0)
    assert bench.traffic_from_profiles("wl", "other", "plane_inverse") is None
    assert bench.traffic_from_profiles("nope", "abc", "plane_inverse") is None


def test_summarize_pmc_ratios(tmp_path, capsys):
    # one dispatch of 2 ms: 8 XCDs at 2 GHz busy = 8 * 4e6 cycles; 256 CUs
    # with 8 waves each resident throughout = 8 * 256 * 4e6 / 4 quad-cycles
    busy = 8 * 4e6
    wave_cycles = 8 * 256 * 4e6 / 4
    write_pmc(tmp_path / "A", [
        (1, K2_INV, "SQ_WAVES", 2048, 0, 2_000_000),
        (1, K2_INV, "SQ_INSTS_VALU", 2048 * 100, 0, 2_000_000),
        (1, K2_INV, "SQ_WAVE_CYCLES", wave_cycles, 0, 2_000_000),
        (1, K2_INV, "SQ_WAIT_INST_ANY", wave_cycles / 4, 0, 2_000_000),
        (1, K2_INV, "GRBM_GUI_ACTIVE", busy, 0, 2_000_000),
        (2, COPY, "SQ_WAVES", 5, 0, 10),
    ])
    write_pmc(tmp_path / "B", [
        (1, K2_INV, "TCC_HIT_sum", 300, 0, 2_000_000),
        (1, K2_INV, "TCC_MISS_sum", 100, 0, 2_000_000),
        (1, K2_INV, "TCP_TCC_READ_REQ_sum", 10, 0, 2_000_000),
        (1, K2_INV, "TCP_TCC_READ_REQ_LATENCY_sum", 5000, 0, 2_000_000),
    ])
    bench.summarize_pmc([str(tmp_path / "A"), str(tmp_path / "B")])
    out = capsys.readouterr().out.strip().splitlines()
    hdr = [c.strip() for c in out[-3].strip("|").split("|")]
    row = [c.strip() for c in out[-1].strip("|").split("|")]
    got = dict(zip(hdr, row))
    assert got["kernel"] == "plane_inverse"
    assert float(got["mean dispatch ms"]) == pytest.approx(2.0)
    assert float(got["VALU insts / wave"]) == pytest.approx(100)
    assert float(got["waiting / resident"]) == pytest.approx(0.25)
    assert float(got["L2 hit rate"]) == pytest.approx(0.75)
    assert float(got["L2 read latency (cycles)"]) == pytest.approx(500)
    assert float(got["clock (GHz)"]) == pytest.approx(2.0)
    assert float(got["resident waves / CU"]) == pytest.approx(8.0)
    assert got["LDS insts / wave"] == ""  # counter not collected
    assert not any("copyBuffer" in line for line in out)


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
