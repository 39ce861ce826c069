"""Host-side logic of bench.py (no GPU): the roofline work figures, the
gate on the committed stage (a) traffic summary, and the one-GPU limit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_stage_a_work_per_pair():
    # 2 (52 n + 72) algorithmic flops; the kernel issues 2 per real unit
    # (28 n + 56 units) and 6 per power of the chain
    assert bench.stage_a_flops_per_pair(10) == 1184.0
    assert bench.stage_a_flops_executed_per_pair(10) == 2 * (28 * 10 + 56) + 6 * 25
    assert bench.stage_a_flops_executed_per_pair(0) == 2 * 56 + 6 * 6


def _kv(path):
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_traffic_summary_is_gated_on_the_sources(tmp_path, monkeypatch):
    kv = _kv(bench.TRAFFIC_FILE)
    for key in ("kernel_source_sha256", "input_source_sha256", "traffic_bytes_per_launch",
                "fetch_bytes_per_launch", "write_bytes_per_launch"):
        assert key in kv, key
    t = float(kv["traffic_bytes_per_launch"])
    assert t == pytest.approx(float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"]),
                              rel=1e-5)
    # the same file with the current source hashes is reported, with any
    # other hash it is not
    good = tmp_path / "good.txt"
    text = open(bench.TRAFFIC_FILE).read()
    text = text.replace(kv["kernel_source_sha256"], bench.kernel_source_hash())
    text = text.replace(kv["input_source_sha256"], bench.input_source_hash())
    good.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.stage_a_traffic() == t
    for key in ("kernel_source_sha256", "input_source_sha256"):
        bad = tmp_path / f"bad_{key}.txt"
        h = bench.kernel_source_hash() if key == "kernel_source_sha256" else bench.input_source_hash()
        bad.write_text(text.replace(h, "0" * 64))
        monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
        assert bench.stage_a_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.stage_a_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
