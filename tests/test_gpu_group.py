"""GPU parity of the group-criterion variant (BH_GROUP_CRITERION: groups are the
largest cubes of at most 64 bodies) against the oracle's group walk over the same
cube groups: interaction sets equal, forces within the FP64 (1e-10 RMS) and FP32
(2e-6 RMS, 1e-4 max) gates; forests mixing the two criteria equal each simulation
alone."""
import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_helpers import dev, rel_max, rel_rms, u64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bh = pytest.importorskip("paper_1109_5190_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bh.Context(0)
    yield c
    c.sync()


def make(kind, n, seed):
    if kind == "plummer":
        return icgen.plummer(n, seed)
    if kind == "cube":
        return icgen.uniform_cube(n, seed)
    if kind == "duplicates":
        s = icgen.plummer(n, seed)
        pos = np.round(s.pos * 4.0) / 4.0
        pos[: n // 4] = pos[0]
        return icgen.System(pos, s.vel, s.mass)
    return icgen.two_plummer(n // 2, seed, seed + 1)


CASES = [
    ("plummer", 4096, 1, 0.5, 0.01, 1),
    ("plummer", 4096, 1, 1.0, 0.01, 8),
    ("cube", 10001, 5, 0.6, 0.005, 1),        # ragged last walk window
    ("plummer", 20000, 4, 0.8, 0.0, 1),       # unsoftened pairs
    ("two_spheres", 20000, 3, 0.5, 0.005, 2),
    ("duplicates", 5000, 7, 0.6, 0.01, 2),    # a leaf of 1250 coincident bodies
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,n,seed,theta,eps,cap", CASES)
def test_group_walk_parity(ctx, prec, kind, n, seed, theta, eps, cap):
    print(f"[group] {kind} n={n} theta={theta} eps={eps} leaf_cap={cap} {prec}", flush=True)
    s = make(kind, n, seed)
    T = oracle.Tree(s.pos, s.mass, cap)
    ref = T.walk_group(theta, eps, 1.0, starts=T.group_cubes(64))
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(theta, eps, leaf_cap=cap, precision=prec, group=True)).upward()
    r = t.forces_stats(pot=True)
    assert torch.equal(t.forces(), r["acc"])
    assert np.array_equal(r["n_mono"].cpu().numpy(), ref["n_mono"])
    assert np.array_equal(r["n_p2p"].cpu().numpy(), ref["n_p2p"])
    assert np.array_equal(u64(r["hash"]), ref["hash"])
    acc, pot = r["acc"].cpu().numpy(), r["pot"].cpu().numpy()
    if prec == "fp64":
        assert rel_rms(acc, ref["acc"]) <= 1e-10
        assert np.abs(pot - ref["pot"]).max() <= 1e-10 * np.abs(ref["pot"]).max()
    else:
        assert rel_rms(acc, ref["acc"]) <= 2e-6
        assert rel_max(acc, ref["acc"]) <= 1e-4


def test_forest_mixing_criteria_equals_alone(ctx):
    ns = [3000, 5000, 900, 4096]
    seeds = [71, 72, 73, 74]
    cfg = [("fp32", True), ("fp32", False), ("fp64", True), ("fp64", False)]
    plist = [bh.params(0.6, 0.01, precision=p, group=g) for p, g in cfg]
    systems = [icgen.plummer(n, sd) for n, sd in zip(ns, seeds)]
    cat = icgen.concat(*systems)
    fo = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    acc = fo.forces()
    off = 0
    for n, sysm, p in zip(ns, systems, plist):
        t = bh.Tree(ctx, dev(sysm.pos), dev(sysm.mass), p).upward()
        assert torch.equal(acc[off:off + n], t.forces())
        off += n


def test_quad_and_group_are_not_combined(ctx):
    s = icgen.plummer(100, 1)
    with pytest.raises(bh.BHError):
        bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01, quad=True, group=True))
