"""The benchmark's contract on the CPU: more than one GPU is refused with a JSON message and
exit status 2 before anything touches a device, and the roofline's HBM traffic is taken from
the committed counter summaries (HBM traffic, VALU instructions) only for the walk sources and
workload size they were measured on."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_profile_figures_follow_the_walk_source(tmp_path, monkeypatch):
    import hashlib
    srcs = [tmp_path / "walk.hip", tmp_path / "common.h"]
    srcs[0].write_bytes(b"// a walk source\n")
    srcs[1].write_bytes(b"// its header\n")
    sha = hashlib.sha256(srcs[0].read_bytes() + srcs[1].read_bytes()).hexdigest()
    summary = tmp_path / "traffic.md"
    summary.write_text("# counters\n\nbench-traffic: kernel=k_walk32 n=1048576 value=2030000000 "
                       f"source-sha256={sha}\n")
    valu = tmp_path / "valu.md"
    valu.write_text(f"bench-valu: kernel=k_walk32 n=1048576 value=1500000000 source-sha256={sha}\n")
    monkeypatch.setattr(bench, "WALK_SOURCES", srcs)
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", summary)
    monkeypatch.setattr(bench, "VALU_SUMMARY", valu)
    assert bench.walk_traffic(1 << 20) == 2030000000
    assert bench.walk_valu(1 << 20) == 1500000000
    assert bench.walk_traffic(1 << 21) is None  # another workload size
    srcs[1].write_bytes(srcs[1].read_bytes() + b"\n")   # any change to the walk sources voids the figures
    assert bench.walk_traffic(1 << 20) is None
    assert bench.walk_valu(1 << 20) is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", tmp_path / "missing.md")
    assert bench.walk_traffic(1 << 20) is None
