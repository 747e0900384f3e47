"""GPU parity of the alternative opening radii (BH_OPEN_BMAX, BH_OPEN_OFFSET) against the
oracle's walk with the same radius: interaction sets equal, forces within the FP64 (1e-10 RMS)
and FP32 (2e-6 RMS, 1e-4 max) gates; with the quadrupole; forests mixing radii equal each
simulation alone; the flags' exclusions are refused."""
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


CASES = [
    ("plummer", 4096, 1, 0.5, 0.01, 1),
    ("plummer", 4096, 1, 1.0, 0.01, 1),    # theta 1: the side test accepts cubes holding the body
    ("plummer", 20000, 4, 0.8, 0.0, 1),    # unsoftened
    ("cube", 10001, 5, 0.6, 0.005, 4),
    ("two_spheres", 20000, 3, 0.4, 0.005, 2),
    ("duplicates", 5000, 7, 0.7, 0.01, 2),
    ("plummer", 3000, 2, 0.0, 0.01, 1),    # theta 0: direct summation
]


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


def check(r, ref, prec):
    assert np.array_equal(r["n_mono"].cpu().numpy(), ref["n_mono"])
    assert np.array_equal(r["n_p2p"].cpu().numpy(), ref["n_p2p"])
    assert np.array_equal(u64(r["hash"]), ref["hash"])
    acc = r["acc"].cpu().numpy()
    if prec == "fp64":
        assert rel_rms(acc, ref["acc"]) <= 1e-10
    else:
        assert rel_rms(acc, ref["acc"]) <= 2e-6
        assert rel_max(acc, ref["acc"]) <= 1e-4


@pytest.mark.parametrize("open_", ["bmax", "offset"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,n,seed,theta,eps,cap", CASES)
def test_open_walk_parity(ctx, open_, prec, kind, n, seed, theta, eps, cap):
    print(f"[open] {open_} {kind} n={n} theta={theta} eps={eps} leaf_cap={cap} {prec}", flush=True)
    s = make(kind, n, seed)
    T = oracle.Tree(s.pos, s.mass, cap)
    ref = T.walk(theta, eps, open=open_)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass),
                bh.params(theta, eps, leaf_cap=cap, precision=prec, open=open_)).upward()
    r = t.forces_stats()
    assert torch.equal(t.forces(), r["acc"])
    check(r, ref, prec)
    if theta > 0:
        # the radius changes the sets (it is not silently the side)
        side = T.walk(theta, eps)
        assert not np.array_equal(side["hash"], ref["hash"])


@pytest.mark.parametrize("open_", ["bmax", "offset"])
def test_open_with_quadrupole(ctx, open_):
    s = icgen.plummer(6000, 9)
    ref = oracle.forces(s.pos, s.mass, theta=0.7, eps=0.01, quad=True, open=open_)
    for prec in ("fp64", "fp32"):
        t = bh.Tree(ctx, dev(s.pos), dev(s.mass),
                    bh.params(0.7, 0.01, precision=prec, quad=True, open=open_)).upward()
        check(t.forces_stats(), ref, prec)


def test_forest_mixing_radii_equals_alone(ctx):
    ns = [3000, 5000, 800, 4096, 2500]
    systems = [icgen.plummer(n, 70 + k) for k, n in enumerate(ns)]
    cfg = [("fp32", "bmax"), ("fp64", "offset"), ("fp32", "side"), ("fp64", "bmax"), ("fp32", "offset")]
    plist = [bh.params(0.8, 0.01, precision=p, open=o) for p, o in cfg]
    cat = icgen.concat(*systems)
    fo = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    acc = fo.forces()
    off = 0
    for n, sysm, p in zip(ns, systems, plist):
        t = bh.Tree(ctx, dev(sysm.pos), dev(sysm.mass), p).upward()
        assert torch.equal(acc[off:off + n], t.forces())
        off += n


def test_open_flags_validated(ctx):
    s = icgen.plummer(100, 1)
    for flags in (bh.OPEN_BMAX | bh.OPEN_OFFSET, bh.OPEN_BMAX | bh.GROUP_CRITERION,
                  bh.OPEN_OFFSET | bh.GROUP_CRITERION):
        p = bh.params(0.5, 0.01)
        p.flags = flags
        with pytest.raises(bh.BHError):
            bh.Tree(ctx, dev(s.pos), dev(s.mass), p)
