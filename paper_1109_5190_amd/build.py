"""Builds libbh.so in-tree with hipcc for gfx950: every HIP source is compiled
to its own object in parallel, then the objects are linked into the shared
library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libbh.so"

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # decision-relevant arithmetic must not be contracted; wanted FMAs are written explicitly
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
NOISE = "is not a recognized feature for this target"


def sources():
    return sorted(str(p) for p in CSRC.glob("*.hip"))


def _jobs():
    try:
        return max(1, int(os.environ.get("MAX_JOBS", "")))
    except ValueError:
        return max(1, min(16, os.cpu_count() or 1))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if NOISE not in l)
    return res.returncode, msg


def build(verbose: bool = False) -> Path:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = [f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    with tempfile.TemporaryDirectory(prefix="bh_build_") as tmpd:
        objs = [str(Path(tmpd) / (Path(s).stem + ".o")) for s in sources()]
        cmds = [[hipcc, *HIPCC_FLAGS, *inc, "-c", s, "-o", o] for s, o in zip(sources(), objs)]
        with ThreadPoolExecutor(max_workers=_jobs()) as ex:
            results = list(ex.map(_run, cmds))
        msgs = []
        for (rc, msg), s in zip(results, sources()):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {s} ({rc}):\n{msg}")
            if msg.strip():
                msgs.append(msg)
        tmp = LIB.with_suffix(".so.tmp")
        rc, msg = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", str(tmp)])
        if rc != 0:
            raise RuntimeError(f"link failed ({rc}):\n{msg}")
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
