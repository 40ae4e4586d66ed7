"""Host-side logic of bench.py (no GPU): the one-GPU guard, kernel naming of the
product classes and the rule that HBM traffic figures are used only for the
kernel sources they were measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_kernel_names():
    assert bench.kernel_name({"b": 9, "rows": 8, "variant": 4}) == "k_product_ring<9, 8, 2>"
    assert bench.kernel_name({"b": 9, "rows": 8, "variant": 4, "precision": 2}) == "k_product_mfma_bf16<8>"
    assert bench.kernel_name({"b": 4, "rows": 4, "variant": 3}) == "k_product_ring<4, 4, 3>"
    assert bench.kernel_name({"b": 9, "rows": 8, "variant": 4, "precision": 1}).endswith("(FP32)")
    assert "2 waves" in bench.kernel_name({"b": 9, "rows": 8, "variant": 5})


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    assert bench.measured_traffic("no_such_profile.json") is None
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = bench.kernel_sources_sha()
    rec = {"sources_sha256_16": sha, "hbm_bytes_per_launch": 1.5e11}
    (prof / "t.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: sha)
    assert bench.measured_traffic("t.json") == 1.5e11
    rec["sources_sha256_16"] = "0000000000000000"
    (prof / "t.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("t.json") is None
