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
    pmc.write_text(json.dumps({
        "kernel_source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(), "work_level": 9,
        "by_batch": {"16": {"kernels": {
            "k_conv_cols": {"bytes_per_output_row": 1000.0},
            "k_ntt_rows_ks8": {"fetch_bytes_per_dispatch": 300.0, "write_bytes_per_dispatch": 200.0}}},
            "32": {"kernels": {"k_ntt_rows_ks8": {"fetch_bytes_per_dispatch": 600.0, "write_bytes_per_dispatch": 400.0}},
                   "sq": {"k_ntt_rows_ks8": {"valu_insts_per_dispatch": 1e6}}}}}))
    monkeypatch.setattr(bench, "PMC_FILE", str(pmc))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.pmc_traffic("k_conv_cols", 16, 9, rows=3.5) == pytest.approx(3500.0)
    assert bench.pmc_traffic("k_ntt_rows_ks8", 16, 9) == pytest.approx(500.0)
    assert bench.pmc_traffic("k_ntt_rows_ks8", 32, 9) == pytest.approx(1000.0)
    assert bench.pmc_traffic("k_ntt_rows_ks8", 24, 9) is None    # a chunk size not measured
    v = bench.pmc_valu("k_ntt_rows_ks8", 32, 9, 100.0)            # 1e6 wave instructions in 100 us
    assert v["lane_ops_per_s"] == pytest.approx(6.4e11) and v["frac"] == pytest.approx(6.4e11 / bench.VALU_PEAK_LANE_OPS, abs=1e-4)
    assert bench.pmc_valu("k_ntt_rows_ks8", 16, 9, 100.0) is None  # no SQ pass at this size
    assert bench.pmc_traffic("k_ntt_rows_ks8", 16, 23) is None   # another working level
    assert bench.pmc_traffic("k_tensor", 16, 9) is None          # not measured
    src.write_bytes(b"// kernel source B\n")       # the kernel changed since the counters were taken
    assert bench.pmc_traffic("k_ntt_rows_ks8", 16, 9) is None
    monkeypatch.setattr(bench, "PMC_FILE", str(tmp_path / "missing.json"))
    assert bench.pmc_traffic("k_ntt_rows_ks8", 16, 9) is None


def test_committed_pmc_summary_is_well_formed():
    with open(bench.PMC_FILE) as f:
        pm = json.load(f)
    assert len(pm["kernel_source_sha256"]) == 64
    assert pm["by_batch"]
    for ent in pm["by_batch"].values():
        assert ent["copy_probe"]["write_factor"] == pytest.approx(1.0, abs=0.05)
        conv = ent["kernels"]["k_conv_cols"]
        assert conv["bytes_per_output_row"] >= conv["algorithmic_write_bytes_per_row"] > 0
        ks = ent["kernels"]["k_ntt_rows_ks8"]
        assert ks["fetch_bytes_per_dispatch"] > 0 and ks["write_bytes_per_dispatch"] > 0


def test_iteration_model_bytes_grows_with_the_blocks():
    cfg = synth.get_config("c3")
    one, two = bench.iteration_model_bytes(cfg, 1000), bench.iteration_model_bytes(cfg, 2000)
    assert 0 < one < two < 2 * one   # per-block work plus a once-per-iteration tail


def test_iteration_model_bytes_shrink_with_the_working_level():
    cfg = synth.get_config("c3")
    top = bench.iteration_model_bytes(cfg, 1000)
    assert bench.iteration_model_bytes(cfg, 1000, level=len(cfg["q_bits"]) - 1) == top
    assert bench.iteration_model_bytes(cfg, 1000, level=9) < 0.6 * top
