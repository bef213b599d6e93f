"""Host-side parts of bench.py (no GPU): the algorithmic byte models behind
`roofline.frac`, the one-GPU rule, and the source check of the recorded
HBM traffic."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_byte_models_at_c2():
    # N = 1000, S = 2000, m = 4, K = 4, FP64: V = 256,000 B, I' = 998
    b = bench.algorithmic_bytes(1000, 2000, 4, 4, 8)
    assert b["V"] == 256_000
    assert b["post"] == 2 * 998 * 256_000 + 1000 * 2000 + b["P"]
    assert b["pre"] == 3 * 998 * 256_000 + 1000 * 2000 + b["P"]
    assert b["eval"] == b["post"] + b["pre"]
    assert abs(b["eval"] / 1e9 - 1.283) < 0.001      # 1.283 GB per evaluation
    o = bench.onchip_bytes(1000, 2000, 4, 4, 8)
    assert o["post"] == 998 * 256_000 + 1000 * 2000 + b["P"]
    assert o["pre"] - o["post"] == 8 * 1998 * 4 * 125   # one partial per branch and tile
    # FP32 halves the vector bytes, not the tip codes
    b32 = bench.algorithmic_bytes(1000, 2000, 4, 4, 4)
    assert b32["V"] == b["V"] // 2 and b32["tips"] == b["tips"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    # a record for another source is not reported; the committed one is
    # reported only while the source still matches it
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / "traffic.json").write_text(json.dumps({
        "sources_sha256": {"kernels.hip": "0" * 64},
        "C2": {"fp64": {"pre": {"read_bytes": 1, "write_bytes": 2}}}}))
    csrc = tmp_path / "paper_1905_12146_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_text("// another source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record("pre", "fp64", "C2") is None
    import hashlib
    digest = hashlib.sha256(b"// another source\n").hexdigest()
    (fake / "traffic.json").write_text(json.dumps({
        "sources_sha256": {"kernels.hip": digest},
        "C2": {"fp64": {"pre": {"read_bytes": 1, "write_bytes": 2}}}}))
    assert bench.traffic_record("pre", "fp64", "C2") == 3
