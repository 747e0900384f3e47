"""Input generator checks: Philox known answers, Plummer closed forms, cube bounds."""
import json
import math
from pathlib import Path

import numpy as np
import pytest
from scipy import stats

import icgen
import oracle

GOLDEN = Path(__file__).resolve().parent / "golden"


def test_philox_known_answers():
    g = json.loads((GOLDEN / "philox4x32_10_kat.json").read_text())
    for case in g["cases"]:
        ctr = np.array([[int(v, 16) for v in case["ctr"]]], dtype=np.uint32)
        key = [int(v, 16) for v in case["key"]]
        out = icgen.philox4x32_10(ctr, key)[0]
        assert [int(v) for v in out] == [int(v, 16) for v in case["out"]]


def test_uniforms_open_interval_and_counter_based():
    a, b = icgen.uniforms(42, np.arange(100000, dtype=np.uint64), 0, 9)
    assert a.min() > 0.0 and a.max() < 1.0 and b.min() > 0.0 and b.max() < 1.0
    a2, _ = icgen.uniforms(42, np.arange(99990, 100000, dtype=np.uint64), 0, 9)
    assert np.array_equal(a2, a[-10:])                       # index-addressed, order free
    assert abs(a.mean() - 0.5) < 0.005


def test_plummer_radii_follow_mass_profile():
    s = icgen.plummer(20000, 3, com_frame=False)
    r = np.linalg.norm(s.pos, axis=1)
    cut = icgen.PLUMMER_MASS_CUT
    cdf = lambda x: np.minimum((x ** 3 / (1 + x * x) ** 1.5) / cut, 1.0)  # noqa: E731
    assert stats.kstest(r, cdf).pvalue > 1e-3
    # median of the truncated profile solves r^3/(1+r^2)^1.5 = cut/2
    med = 1.0 / math.sqrt((cut / 2) ** (-2.0 / 3.0) - 1.0)
    assert abs(np.median(r) - med) < 0.03 * med
    assert r.max() <= 1.0 / math.sqrt(cut ** (-2.0 / 3.0) - 1.0) + 1e-12


def test_plummer_virial_ratio():
    s = icgen.plummer(4096, 1)
    d = oracle.direct(s.pos, s.mass, eps=0.0)
    K, W = oracle.energy(s.vel, s.mass, d["pot"])
    # Plummer sphere with G = M = a = 1: K = 3 pi / 64, W = -3 pi / 32, Q = K/|W| = 1/2
    assert abs(K / abs(W) - 0.5) < 0.03
    assert abs(K - 3 * math.pi / 64) < 0.1 * 3 * math.pi / 64
    assert abs(W + 3 * math.pi / 32) < 0.1 * 3 * math.pi / 32


def test_plummer_com_frame_and_bulk_motion():
    s = icgen.plummer(5000, 4, centre=(5.0, 0.0, 0.0), bulk_velocity=(-0.3, 0.0, 0.0))
    assert np.allclose((s.mass[:, None] * s.pos).sum(0) / s.mass.sum(), [5.0, 0.0, 0.0], atol=1e-12)
    assert np.allclose((s.mass[:, None] * s.vel).sum(0) / s.mass.sum(), [-0.3, 0.0, 0.0], atol=1e-12)
    assert np.isclose(s.mass.sum(), 1.0)


def test_plummer_speeds_below_escape():
    s = icgen.plummer(20000, 5, com_frame=False)
    r = np.linalg.norm(s.pos, axis=1)
    v = np.linalg.norm(s.vel, axis=1)
    assert np.all(v <= math.sqrt(2.0) * (1 + r * r) ** -0.25 * (1 + 1e-12))
    q = v / (math.sqrt(2.0) * (1 + r * r) ** -0.25)
    # q has density proportional to q^2 (1-q^2)^(7/2): mean B(2, 4.5)/B(1.5, 4.5)
    mean_q = math.exp(math.lgamma(2) + math.lgamma(4.5) - math.lgamma(6.5)
                            - (math.lgamma(1.5) + math.lgamma(4.5) - math.lgamma(6.0)))
    assert abs(q.mean() - mean_q) < 0.01


def test_uniform_cube_bounds():
    s = icgen.uniform_cube(50000, 5)
    assert s.pos.min() >= -1.0 and s.pos.max() <= 1.0
    assert s.mass.min() >= 0.5 / 50000 and s.mass.max() <= 1.5 / 50000
    assert abs(s.mass.sum() - 1.0) < 0.01
    assert np.all(s.vel == 0.0)


def test_workload_recipes():
    inst = icgen.batch_instances(512, 6)
    ns = np.array([n for n, _, _ in inst])
    assert ns.min() >= 1024 and ns.max() <= 262144
    assert 0.6 * 47090 * 512 < ns.sum() < 1.4 * 47090 * 512
    assert {t for _, t, _ in inst} == {0.4, 0.5, 0.7}
    reqs = icgen.request_stream(2000, 200.0, 7)
    t = np.array([r["t"] for r in reqs])
    assert np.all(np.diff(t) >= 0) and abs(t[-1] / 2000 - 1 / 200) < 0.15 / 200
    assert all(1 <= r["steps"] <= 100 for r in reqs)
