"""CPU: the profile summaries that the benchmark's `traffic` figures come
from.  Counter values are scaled by what the same counter reads for the
512 MiB device-to-device copy of the run; the summary is keyed by the hash
of the sweep source that bench.py checks before it reports the figure."""
import csv
import json
import os
import sys

import pytest

from paper_1803_09876_amd import rocprof_summary as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SWEEP = "void jsw::k_sweep<double, 3, 0, false, 1, true, true>(jsw::SweepArgs<double>)"
COPY = "__amd_rocclr_copyBuffer"


def _counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(rows):
            w.writerow([i, name, counter, value])


def test_traffic_scaled_by_the_copy(tmp_path):
    # the copy reads 512 MiB and FETCH_SIZE says half of it: scale 2; WRITE_SIZE says all of it: scale 1
    _counters(tmp_path / "f", "FETCH_SIZE", [(COPY, 262144.0), (SWEEP, 100.0), (SWEEP, 300.0), ("other", 5.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(COPY, 524288.0), (SWEEP, 50.0), (SWEEP, 50.0)])
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    R.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_sweep<double", "key", str(out_json), str(out_md), "cmd")
    rec = json.load(open(out_json))["key"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["dispatches"] == [2, 2]
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(200.0 * 2.0 * 1024.0)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(50.0 * 1024.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(200.0 * 2048.0 + 50.0 * 1024.0)
    assert "cmd" in open(out_md).read()


def test_traffic_needs_the_copy(tmp_path):
    _counters(tmp_path / "f", "FETCH_SIZE", [(SWEEP, 100.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(COPY, 524288.0), (SWEEP, 50.0)])
    with pytest.raises(SystemExit):
        R.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_sweep<double", "key", str(tmp_path / "t.json"),
                  str(tmp_path / "t.md"), "cmd")


def test_summary_hash_is_the_one_bench_checks(tmp_path):
    _counters(tmp_path / "f", "FETCH_SIZE", [(COPY, 262144.0), (SWEEP, 1.0)])
    _counters(tmp_path / "w", "WRITE_SIZE", [(COPY, 524288.0), (SWEEP, 1.0)])
    out_json = tmp_path / "t.json"
    R.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_sweep<double", "key", str(out_json),
              str(tmp_path / "t.md"), "cmd")
    sys.path.insert(0, ROOT)
    import bench
    assert json.load(open(out_json))["key"]["source_hash"] == bench._source_hash()


def test_committed_traffic_matches_the_current_sweep_source():
    """profiles/traffic.json was taken on the sweep source as committed (else
    bench.py would report the traffic as null)."""
    sys.path.insert(0, ROOT)
    import bench
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert "k_sweep<double> tetcheck96_s8" in data
    for key, rec in data.items():
        assert rec["source_hash"] == bench._source_hash(), key


def test_counters_derived_rates(tmp_path):
    path = tmp_path / "c"
    os.makedirs(path)
    with open(path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for name, value in (("TCC_HIT_sum", 3.0), ("TCC_MISS_sum", 1.0), ("SQ_WAVE_CYCLES", 10.0),
                            ("SQ_BUSY_CYCLES", 5.0), ("SQ_WAVES", 2048.0)):
            w.writerow([0, SWEEP, name, value])
    out = tmp_path / "c.md"
    R.counters(str(path), "k_sweep<double", str(out), "title", "cmd")
    text = open(out).read()
    assert "L2 hit rate: 0.750" in text and ": 2.0." in text and "2048" in text
