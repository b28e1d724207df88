"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that a
committed counter record is used only for the configuration and kernel source
it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_record_is_keyed(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel v1\n")
    cfg = {"n": 10, "trees": 3}
    rec = {"config": cfg, "source_sha256_16": bench.kernel_source_hash(str(src)),
           "hbm_bytes_per_launch": 123.0, "units_per_launch": 7}
    (tmp_path / "rec.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("rec.json", str(src), cfg) == (123.0, 7)
    assert bench.measured_traffic("rec.json", str(src), {"n": 10, "trees": 4}) is None
    assert bench.measured_traffic("missing.json", str(src), cfg) is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("rec.json", str(src), cfg) is None


def test_committed_records_are_well_formed():
    """The committed records name their kernel source, its hash and the
    configuration they were taken on (bench.py reports traffic as null once
    the source or the configuration differs)."""
    for name, src in [("filter_search-23Mx384_counters.json", "paper_2508_21682_amd/csrc/hf_bfilter.hip"),
                      ("k_band_graph-3Mx384_counters.json", "paper_2508_21682_amd/csrc/hf_graph.hip")]:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert rec["source"] == src and len(rec["source_sha256_16"]) == 16
        assert rec["config"] and rec["commands"]
        assert rec["hbm_bytes_per_launch"] > 0 and rec["units_per_launch"] > 0
