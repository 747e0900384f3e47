"""Pins of the oracle's alternative opening criteria (the paper lists other ways of
computing the approximation criterion as future work, section 6): r = b_max, the
largest distance from the centre of mass to a corner of the cube, and Barnes'
offset test D > s/theta + delta.  Checked against facts that do not come from
that code: radii worked by hand on dyadic coordinates, the geometric bounds
every cube obeys, an independent pure-Python walk on the pointer octree with the
radii taken from its own cube geometry, a closed-form configuration where the
side test accepts the cube holding the body and the other two do not, theta = 0,
and monotonicity of the interaction count in r.  CPU only."""
import math

import numpy as np
import pytest

import icgen
import oracle
from tests import ptree


def bmax2(lo, L):
    def f(nd, s):
        c0 = [lo[d] + nd.cell[d] * s for d in range(3)]
        e = [max(nd.com[d] - c0[d], c0[d] + s - nd.com[d]) for d in range(3)]
        return e[0] ** 2 + e[1] ** 2 + e[2] ** 2
    return f


def offset2(lo, L, theta):
    def f(nd, s):
        ctr = [lo[d] + (nd.cell[d] + 0.5) * s for d in range(3)]
        delta = math.sqrt(sum((nd.com[d] - ctr[d]) ** 2 for d in range(3)))
        return (s + theta * delta) ** 2
    return f


def test_radii_by_hand(oracle_lib):
    """The root cube is anchored at the per-axis minimum lo = (1/16, 1/8, 1/4) with side 1 (the
    largest extent, 29/32, is below 2^0).  Node 0 is the root, its children the leaves of the two
    particles: (1/16, 1/8, 1/4) at the corner of octant 0 and (31/32, 31/32, 31/32) in octant 7,
    each of side 1/2 with the particle as centre of mass.  All values are exact in binary."""
    pos = np.array([[1 / 16, 1 / 8, 1 / 4], [31 / 32, 31 / 32, 31 / 32]])
    mass = np.array([1.0, 3.0])
    T = oracle.Tree(pos, mass, 1)
    assert T.nn == 3 and T.k == 0 and np.array_equal(T.lo, [1 / 16, 1 / 8, 1 / 4])
    lo = T.lo
    # root: com = (1/16 + 3*31/32, ...)/4 per axis
    com = (pos[0] + 3 * pos[1]) / 4
    e = np.maximum(com - lo, lo + 1.0 - com)
    assert T.open_r2(0.5, "bmax")[0] == (e[0] ** 2 + e[1] ** 2) + e[2] ** 2
    # leaf of particle 0: cube [lo, lo + 1/2)^3, the particle sits at its minimum corner
    assert T.open_r2(0.5, "bmax")[1] == 3 * 0.25
    # leaf of particle 1: cube [lo + 1/2, lo + 1)
    c1 = lo + 0.5
    e1 = np.maximum(pos[1] - c1, c1 + 0.5 - pos[1])
    assert T.open_r2(0.5, "bmax")[2] == (e1[0] ** 2 + e1[1] ** 2) + e1[2] ** 2
    # offset of leaf 0: centre lo + 1/4, particle at lo: delta = sqrt(3)/4
    r = 0.5 + 0.5 * math.sqrt(3 * (1 / 16))
    assert T.open_r2(0.5, "offset")[1] == pytest.approx(r * r, rel=1e-15)
    assert np.array_equal(T.open_r2(0.5, "side"), [1.0, 0.25, 0.25])


def test_offset_three_four_five(oracle_lib):
    """Root [0, 1)^3 (particles at the origin and near (1, 1, 1)); the probe sits in the level-2
    cube [1/4, 1/2)^3, displaced (3/64, 4/64, 0) from its centre 3/8: delta = 5/64 exactly, so the
    offset radius is 1/4 + theta 5/64 and b_max^2 = (1/8 + 3/64)^2 + (1/8 + 4/64)^2 + (1/8)^2."""
    probe = [0.375 + 3 / 64, 0.375 + 4 / 64, 0.375]
    pos = np.array([[0.0, 0.0, 0.0], probe, [0.96875, 0.96875, 0.96875]])
    T = oracle.Tree(pos, np.ones(3), 1)
    assert T.k == 0 and np.array_equal(T.lo, [0.0, 0.0, 0.0])
    ids = [i for i in range(T.nn) if T.count[i] == 1 and T.perm[T.first[i]] == 1]
    assert len(ids) == 1 and T.level[ids[0]] == 2
    r = 0.25 + 0.5 * (5 / 64)
    assert T.open_r2(0.5, "offset")[ids[0]] == r * r
    assert T.open_r2(0.5, "bmax")[ids[0]] == (1 / 8 + 3 / 64) ** 2 + (1 / 8 + 4 / 64) ** 2 + (1 / 8) ** 2


@pytest.mark.parametrize("kind", ["plummer", "cube", "duplicates"])
def test_radius_bounds(oracle_lib, kind):
    """b_max lies between the half diagonal and the full diagonal of the cube (the centre of
    mass is inside the cube); the offset radius lies between s and s (1 + theta sqrt(3)/2).
    Cube corners carry a rounding of the root corner's magnitude, which for level-21 cubes is
    not small against their side: the bounds allow a few units in the last place of it."""
    if kind == "plummer":
        s = icgen.plummer(3000, 3)
    elif kind == "cube":
        s = icgen.uniform_cube(3000, 4)
    else:
        s = icgen.plummer(2000, 5)
        pos = np.round(s.pos * 4.0) / 4.0
        pos[:500] = pos[0]
        s = icgen.System(pos, s.vel, s.mass)
    T = oracle.Tree(s.pos, s.mass, 1)
    side = T.L / 2.0 ** T.level
    tol = 4 * 2.0 ** -52 * (np.abs(T.lo).max() + T.L)
    b = T.open_r2(0.7, "bmax")
    assert np.all(b >= 3 * (side / 2 - tol) ** 2) and np.all(b <= 3 * (side + tol) ** 2)
    o = T.open_r2(0.7, "offset")
    assert np.all(o >= side ** 2) and np.all(o <= (side + 0.7 * math.sqrt(3) * (side / 2 + tol)) ** 2)
    assert np.array_equal(T.open_r2(0.7, "side"), side ** 2)


@pytest.mark.parametrize("open_", ["bmax", "offset"])
@pytest.mark.parametrize("theta", [0.3, 0.6, 1.0])
def test_against_pointer_octree(oracle_lib, open_, theta):
    rng = np.random.default_rng(int(theta * 10) + (0 if open_ == "bmax" else 100))
    n = 60
    pos = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    T = oracle.Tree(pos, mass, 1)
    r = T.walk(theta, 0.02, open=open_)
    root, nodes, lo, L = ptree.build(pos.tolist(), mass.tolist(), 1)
    rad = bmax2(lo, L) if open_ == "bmax" else offset2(lo, L, theta)
    nn = len(nodes)
    assert nn == T.nn
    for i in range(n):
        acc, mono, pairs = ptree.walk(root, nodes, pos.tolist(), mass.tolist(), L, i, theta, 0.02, radius2=rad)
        assert r["n_mono"][i] == len(mono) and r["n_p2p"][i] == len(pairs)
        h = (sum(oracle.mix64(k) for k in mono) + sum(oracle.mix64(nn + j) for j in pairs)) % (1 << 64)
        assert int(r["hash"][i]) == h
        assert np.linalg.norm(r["acc"][i] - acc) <= 1e-12 * np.linalg.norm(acc)


def test_self_containing_cube(oracle_lib):
    """A light body at the corner (0,0,0) of the root cube [0,1)^3 and a heavy cluster near the
    opposite corner: D from the body to the root's centre of mass is about 1.70 > 1, so the side
    test with theta = 1 accepts the root, which holds the body itself.  b_max is the distance
    from that centre of mass to the corner where the body sits, which is D again (the strict
    test fails), and the offset radius 1 + delta exceeds D; both open the root and accept the
    cluster's own cube instead."""
    rng = np.random.default_rng(9)
    cluster = 0.97 + 0.02 * rng.random((10, 3))
    pos = np.vstack([[0.0, 0.0, 0.0], cluster])
    mass = np.concatenate([[1e-3], np.full(10, 1.0)])
    T = oracle.Tree(pos, mass, 1)
    assert T.k == 0 and np.array_equal(T.lo, [0.0, 0.0, 0.0])
    side = T.walk(1.0, 0.0, targets=[0])
    assert side["n_mono"][0] == 1 and side["n_p2p"][0] == 0 and int(side["hash"][0]) == oracle.mix64(0)
    # the smallest cube holding the cluster (single-child cubes above it are removed) is
    # node 2 in preorder; node 1 is the body's leaf
    assert T.count[2] == 10 and T.parent[2] == 0
    for open_ in ("bmax", "offset"):
        r = T.walk(1.0, 0.0, targets=[0], open=open_)
        assert r["n_mono"][0] == 1 and r["n_p2p"][0] == 0 and int(r["hash"][0]) == oracle.mix64(2), open_


@pytest.mark.parametrize("open_", ["bmax", "offset"])
def test_theta_zero_is_direct_sum(oracle_lib, open_):
    s = icgen.plummer(500, 6)
    T = oracle.Tree(s.pos, s.mass, 1)
    r = T.walk(0.0, 0.01, open=open_)
    d = oracle.direct(s.pos, s.mass, eps=0.01)
    assert np.all(r["n_mono"] == 0) and np.all(r["n_p2p"] == s.n - 1)
    assert np.abs(r["acc"] - d["acc"]).max() <= 1e-13 * np.abs(d["acc"]).max()


def test_larger_radius_never_fewer_interactions(oracle_lib):
    """The offset radius is never below the side, so per body the walk opens at least the cubes
    the side test opens: interaction counts do not drop, and here the error against direct
    summation falls."""
    s = icgen.plummer(3000, 8)
    T = oracle.Tree(s.pos, s.mass, 1)
    a, b = T.walk(0.7, 0.01), T.walk(0.7, 0.01, open="offset")
    assert np.all(b["n_mono"] + b["n_p2p"] >= a["n_mono"] + a["n_p2p"])
    d = oracle.direct(s.pos, s.mass, eps=0.01)["acc"]

    def err(x):
        return math.sqrt(((x - d) ** 2).sum() / (d ** 2).sum())

    assert err(b["acc"]) < err(a["acc"])
