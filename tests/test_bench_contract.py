"""The benchmark's contract on the CPU: more than one GPU is refused with a JSON message and
exit status 2 before anything touches a device, and the roofline's HBM traffic is taken from
the committed counter summary only for the walk source and workload size it was measured on."""
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


def test_traffic_follows_the_walk_source(tmp_path, monkeypatch):
    import hashlib
    src = tmp_path / "walk.hip"
    src.write_bytes(b"// a walk source\n")
    summary = tmp_path / "traffic.md"
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary.write_text("# counters\n\nbench-traffic: kernel=k_walk32 n=1048576 bytes=2030000000 "
                       f"source-sha256={sha}\n")
    monkeypatch.setattr(bench, "WALK_SOURCE", src)
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", summary)
    assert bench.walk_traffic(1 << 20) == 2030000000
    assert bench.walk_traffic(1 << 21) is None  # another workload size
    src.write_bytes(src.read_bytes() + b"\n")   # any change to the walk source voids the figure
    assert bench.walk_traffic(1 << 20) is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", tmp_path / "missing.md")
    assert bench.walk_traffic(1 << 20) is None
