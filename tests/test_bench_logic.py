"""Host-only checks of bench.py's measurement bookkeeping: the rocprofv3 summary (counter
calibration, the dispatches that formed a product, the bytes line the roofline reads back) on
synthetic counter files of known content, the scaling of the profiled bytes to the timed
launches, and the kernel-name matching.  No GPU is needed."""
import csv
import io
import json
import os
from contextlib import redirect_stdout
from types import SimpleNamespace

import pytest

import bench

KI = 1024.0


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(path, kernel, counter, values):
    _write_csv(path, ["Kernel_Name", "Counter_Name", "Counter_Value"],
               [[kernel, counter, v] for v in values])


LDS0 = "void pdlp::k_lds_rows<0>(pdlp::CsrDev, pdlp::DevState*, double const*, double const*, int, double*, int)"
PANEL1 = "void pdlp::k_panel_rows<1, 8>(pdlp::CsrDev, pdlp::DevState*, double const*, double const*, int, double*, int, int)"


@pytest.fixture
def profile_dir(tmp_path):
    d = tmp_path / "prof"
    # calibration: a 1 GiB copy reads FETCH_SIZE = 0.5 GiB and writes WRITE_SIZE = 1 GiB (in KiB)
    _counters(str(d / "copy_fetch" / "run_counter_collection.csv"), "copy_kernel", "FETCH_SIZE", [524288.0])
    _counters(str(d / "copy_write" / "run_counter_collection.csv"), "copy_kernel", "WRITE_SIZE", [1048576.0])
    # the K~ first pass: one dispatch that returned at once (below 20% of the largest fetch),
    # three that formed the product; a copy-rate probe's kernel in the same run
    _counters(str(d / "fetch" / "run_counter_collection.csv"), LDS0, "FETCH_SIZE", [10.0, 1000.0, 1000.0, 1100.0])
    with open(d / "fetch" / "run_counter_collection.csv", "a") as fh:
        fh.write('"__amd_rocclr_copyBuffer","FETCH_SIZE",999999\n')
    _counters(str(d / "write" / "run_counter_collection.csv"), LDS0, "WRITE_SIZE", [5.0, 500.0, 520.0, 500.0])
    _counters(str(d / "fetch2.csv"), PANEL1, "FETCH_SIZE", [1.0])      # not under fetch/: ignored
    _write_csv(str(d / "trace" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [[LDS0, 0, 400_000], [LDS0, 500_000, 900_000], [LDS0, 1_000_000, 1_002_000]])
    line = {"workload": "test LP m=1000 n=2000 nnz=30000", "value": 1.0, "layouts": {"K": 3, "KT": 2},
            "passes": {"dual_pass1": {"avg_us": 400.0}}}
    (d / "bench_trace.json").write_text(json.dumps(line) + "\n")
    return str(d)


def _traffic_line(text):
    last = [ln for ln in text.splitlines() if ln.startswith("bench-traffic: ")]
    assert len(last) == 1
    return json.loads(last[0][len("bench-traffic: "):])


def test_summary_scales_counters_by_the_copy_calibration(profile_dir):
    out = io.StringIO()
    with redirect_stdout(out):
        bench.summarize_profile(profile_dir)
    text = out.getvalue()
    t = _traffic_line(text)
    assert t["sources_sha256"] == bench.kernel_sources_digest()
    # median of the three product dispatches: fetch 1000 KiB x 2 (calibration), write 500 KiB x 1
    assert t["bytes_per_dispatch"] == {"k_lds_rows<0>": round(1000.0 * KI * 2.0 + 500.0 * KI)}
    assert "FETCH_SIZE x 2.000 KiB + WRITE_SIZE x 1.000 KiB" in text
    # the per-pass table: measured bytes against the algorithmic bytes of the K~ product
    alg = bench.pass_bytes(SimpleNamespace(m=1000, n=2000, nnz=30000))["dual_pass1"]
    row = [ln for ln in text.splitlines() if ln.startswith("dual_pass1")]
    assert len(row) == 1
    fields = row[0].split()
    assert fields[1] == "k_lds_rows<0>"
    assert float(fields[2]) == pytest.approx((1000.0 * KI * 2.0 + 500.0 * KI) / 1e6, abs=0.05)
    assert float(fields[3]) == pytest.approx(alg / 1e6, abs=0.05)


def test_profiled_bytes_need_the_current_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    stale = tmp_path / "stale.txt"
    good.write_text("x\nbench-traffic: " + json.dumps({"sources_sha256": bench.kernel_sources_digest(),
                                                       "bytes_per_dispatch": {"k_lds_rows<0>": 7}}) + "\n")
    stale.write_text("bench-traffic: " + json.dumps({"sources_sha256": "0" * 64,
                                                     "bytes_per_dispatch": {"k_lds_rows<0>": 7}}) + "\n")
    monkeypatch.setitem(bench.PROFILES, "large", str(good))
    monkeypatch.setitem(bench.PROFILES, "truncated", str(stale))
    assert bench.profiled_bytes("large") == {"k_lds_rows<0>": 7}
    assert bench.profiled_bytes("truncated") is None


def test_traffic_is_scaled_to_the_launches_that_formed_a_product(monkeypatch):
    lp = SimpleNamespace(m=1000, n=2000, nnz=30000)
    full = bench.pass_bytes(lp)["dual_pass1"]
    monkeypatch.setattr(bench, "profiled_bytes", lambda which="large": {"k_lds_rows<0>": 4.0e6})
    # a quarter of the timed first-pass launches returned at once (a rejected attempt): the
    # algorithmic bytes per launch are 3/4 of a product's, and so is the traffic
    r = {"roofline": {"kernel": "k_lds_rows<0>: K~ x' product", "pass": "dual_pass1"},
         "passes": {"dual_pass1": {"algorithmic_bytes_per_launch": 0.75 * full}}}
    bench.attach_traffic(r, lp)
    assert r["roofline"]["traffic"] == pytest.approx(3.0e6)
    assert r["roofline"]["traffic_over_algorithmic"] == pytest.approx(3.0e6 / (0.75 * full))
    # a combine's bytes do not depend on whether the first pass formed its product
    monkeypatch.setattr(bench, "profiled_bytes", lambda which="large": {"k_dual_combine": 5.0e5})
    r = {"roofline": {"kernel": "k_dual_combine: combine", "pass": "dual_combine"},
         "passes": {"dual_combine": {"algorithmic_bytes_per_launch": 56.0 * lp.m}}}
    bench.attach_traffic(r, lp)
    assert r["roofline"]["traffic"] == pytest.approx(5.0e5)
    # a kernel the profile does not cover leaves the field as it was
    r = {"roofline": {"kernel": "k_panel_rows<0>: K~ x' product", "pass": "dual_pass1", "traffic": None},
         "passes": {"dual_pass1": {"algorithmic_bytes_per_launch": full}}}
    bench.attach_traffic(r, lp)
    assert r["roofline"]["traffic"] is None


def test_kernel_names():
    assert bench._short_kernel(LDS0) == "k_lds_rows<0>"
    assert bench._short_kernel(PANEL1) == "k_panel_rows<1, 8>"
    names = {"k_panel_rows<1, 8>": 1, "k_lds_rows<0>": 2, "k_panel_rows<0, 8>": 3, "k_panel_rows<0, 16>": 4}
    assert bench._match_kernel("k_lds_rows<0>", names) == "k_lds_rows<0>"
    assert bench._match_kernel("k_panel_rows<1>", names) == "k_panel_rows<1, 8>"
    assert bench._match_kernel("k_panel_rows<0>", names) is None     # two candidates
    assert bench._match_kernel("k_lds_rows<1>", names) is None
