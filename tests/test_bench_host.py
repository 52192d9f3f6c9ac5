"""Host-side checks of the benchmark script (no GPU needed)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_reported_only_for_the_profiled_sources(monkeypatch):
    text = open(bench.TRAFFIC_PROFILE).read()
    recorded = re.search(r"source_sha256_16: `([0-9a-f]{16})`", text).group(1)
    per_launch = {k: int(v) for k, v in re.findall(r"hbm_bytes_per_launch (\w+): (\d+)", text)}
    assert set(per_launch) == {"k_shadow", "k_shadow_den"}
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: recorded)
    for k, v in per_launch.items():
        assert bench.profiled_traffic(k) == v > 0
    assert bench.profiled_traffic("k_render") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    for k in per_launch:
        assert bench.profiled_traffic(k) is None


def test_source_hash_covers_both_shadow_sources(tmp_path, monkeypatch):
    # editing either source changes the hash (so stale counters are dropped)
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f))
    h0 = bench.kernel_source_hash()
    for i, f in enumerate(bench.KERNEL_SOURCES):
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        for g in bench.KERNEL_SOURCES:
            gp = tmp_path / g
            gp.parent.mkdir(parents=True, exist_ok=True)
            gp.write_bytes(open(os.path.join(ROOT, g), "rb").read())
        dst.write_bytes(dst.read_bytes() + b"\n")
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        assert bench.kernel_source_hash() != h0, f
        monkeypatch.setattr(bench, "ROOT", ROOT)
