"""Known-answer pin of the interaction-set checksum mixer.

The per-body checksum h_i = sum of mix64(node) over accepted cubes plus mix64(n_nodes + j) over
pair partners is what makes "interaction sets equal" checkable; mix64 is the SplitMix64
finalizer of x + 0x9e3779b97f4a7c15.  Its expected values come from the generator's published
outputs (tests/golden/splitmix64_kat.json), not from any implementation here: output k of a
SplitMix64 generator seeded with s is mix64(s + k * gamma).  A changed constant, shift or the
dropped gamma fails these cases.
"""
import json
from pathlib import Path

import numpy as np

import oracle
from tests.gpu_helpers import mix64 as mix64_np

GOLDEN = Path(__file__).resolve().parent / "golden" / "splitmix64_kat.json"
M64 = (1 << 64) - 1


def _cases():
    g = json.loads(GOLDEN.read_text())
    gamma = int(g["gamma"], 16)
    for c in g["cases"]:
        seed = int(c["seed"])
        outs = [int(v, 16) for v in c["out"]] if "out" in c else [int(v) for v in c["out_decimal"]]
        for k, want in enumerate(outs):
            yield (seed + k * gamma) & M64, want


def test_oracle_mix64_known_answers(oracle_lib):
    cases = list(_cases())
    assert len(cases) == 10
    for x, want in cases:
        assert oracle.mix64(x) == want, hex(x)


def test_vectorised_mix64_known_answers():
    xs, wants = zip(*_cases())
    got = mix64_np(np.array(xs, dtype=np.uint64))
    assert [int(v) for v in got] == list(wants)
