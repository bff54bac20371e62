"""Host logic of bench.py (no GPU): the one-GPU contract, the counter-traffic lookup that is
valid only for the kernel source it was measured on, and the iteration byte model."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_pmc_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"// kernel source A\n")
    pmc = tmp_path / "pmc.json"
    pmc.write_text(json.dumps({"bytes_per_row": 1000.0,
                               "kernel_source_sha256": hashlib.sha256(src.read_bytes()).hexdigest()}))
    monkeypatch.setattr(bench, "PMC_FILE", str(pmc))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.pmc_traffic(3.5) == pytest.approx(3500.0)
    src.write_bytes(b"// kernel source B\n")       # the kernel changed since the counters were taken
    assert bench.pmc_traffic(3.5) is None
    monkeypatch.setattr(bench, "PMC_FILE", str(tmp_path / "missing.json"))
    assert bench.pmc_traffic(3.5) is None


def test_committed_pmc_summary_is_well_formed():
    with open(bench.PMC_FILE) as f:
        pm = json.load(f)
    assert pm["bytes_per_row"] > pm["algorithmic_write_bytes_per_row"] > 0
    assert len(pm["kernel_source_sha256"]) == 64
    assert pm["copy_probe"]["write_factor"] == pytest.approx(1.0, abs=0.05)


def test_iteration_model_bytes_grows_with_the_blocks():
    cfg = synth.get_config("c3")
    one, two = bench.iteration_model_bytes(cfg, 1000), bench.iteration_model_bytes(cfg, 2000)
    assert 0 < one < two < 2 * one   # per-block work plus a once-per-iteration tail
