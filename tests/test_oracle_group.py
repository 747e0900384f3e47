"""Pins of the oracle's group-criterion walk (a cube is accepted for a whole group
of bodies when it passes against the group's bounding box) against facts that do not
come from that code: the per-body walk it must equal for groups of one, an independent
pure-Python group walk on the pointer octree (groups of key-consecutive bodies, and the
library's groups: the largest cubes of at most 64 bodies, whose partition the pointer
octree also reproduces), the per-body criterion every accepted cube must also pass,
direct summation at theta = 0, the accuracy ordering it implies, and the bounded work
of cube groups on separated systems.  CPU only."""
import math

import numpy as np
import pytest

import icgen
import oracle
from tests import ptree


def test_groups_of_one_are_the_per_body_walk(oracle_lib):
    s = icgen.plummer(3000, 17)
    T = oracle.Tree(s.pos, s.mass, 1)
    for theta in (0.4, 0.7, 1.0):
        a = T.walk(theta, 0.01)
        b = T.walk_group(theta, 0.01, group=1)
        for k in ("n_mono", "n_p2p", "hash"):
            assert np.array_equal(a[k], b[k]), (theta, k)
        # the same terms summed in another order (cubes first, then pairs)
        assert np.abs(a["acc"] - b["acc"]).max() <= 1e-13 * np.abs(a["acc"]).max()
        assert np.abs(a["pot"] - b["pot"]).max() <= 1e-13 * np.abs(a["pot"]).max()


def py_group_walk(pos, mass, theta, eps, group=None, cap=None):
    """Group criterion on the pointer octree (no keys): groups of `group` consecutive bodies in
    the depth-first leaf order (one body per leaf), or (cap) the largest cubes of at most cap
    bodies, a leaf of more than cap bodies cut into runs of cap."""
    root, nodes, lo, L = ptree.build(pos, mass, 1)
    if cap is None:
        order = [i for nd in nodes if not nd.children for i in nd.ids]
        groups = [order[g0:g0 + group] for g0 in range(0, len(order), group)]
    else:
        groups = []

        def collect(nd):
            if len(nd.ids) <= cap:
                groups.append([i for leaf in leaves_of(nd) for i in leaf.ids])
            elif not nd.children:
                groups.extend(nd.ids[k:k + cap] for k in range(0, len(nd.ids), cap))
            else:
                for c in nd.children:
                    collect(c)

        def leaves_of(nd):
            return [nd] if not nd.children else [x for c in nd.children for x in leaves_of(c)]

        collect(root)
    out = {}
    for members in groups:
        blo = [min(pos[i][d] for i in members) for d in range(3)]
        bhi = [max(pos[i][d] for i in members) for d in range(3)]
        mono, leaves = [], []

        def visit(nd):
            dd = [max(0.0, blo[d] - nd.com[d], nd.com[d] - bhi[d]) for d in range(3)]
            D2 = dd[0] ** 2 + dd[1] ** 2 + dd[2] ** 2
            s = L / 2 ** nd.level
            if s * s < theta * theta * D2:
                mono.append(nd)
            elif not nd.children:
                leaves.append(nd)
            else:
                for c in nd.children:
                    visit(c)

        visit(root)
        for i in members:
            pairs = [j for nd in leaves for j in nd.ids if j != i]
            out[i] = ([nd.pre for nd in mono], pairs, mono)
    return out, nodes, groups


@pytest.mark.parametrize("group", [4, 16, 64])
def test_against_pointer_octree(oracle_lib, group):
    rng = np.random.default_rng(group)
    n = 300
    pos = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    T = oracle.Tree(pos, mass, 1)
    r = T.walk_group(0.6, 0.02, group=group)
    ref, nodes, _ = py_group_walk(pos.tolist(), mass.tolist(), 0.6, 0.02, group)
    nn = len(nodes)
    for i in range(n):
        mono_ids, pairs, mono_nodes = ref[i]
        assert r["n_mono"][i] == len(mono_ids) and r["n_p2p"][i] == len(pairs)
        h = (sum(oracle.mix64(k) for k in mono_ids) + sum(oracle.mix64(nn + j) for j in pairs)) % (1 << 64)
        assert int(r["hash"][i]) == h
        # every cube accepted for the group also passes the per-body test of each member
        for nd in mono_nodes:
            D2 = sum((nd.com[d] - pos[i][d]) ** 2 for d in range(3))
            assert (T.L / 2 ** nd.level) ** 2 < 0.36 * D2


def test_theta_zero_is_direct_sum(oracle_lib):
    s = icgen.plummer(1500, 8)
    T = oracle.Tree(s.pos, s.mass, 1)
    g = T.walk_group(0.0, 0.01, group=64)
    d = oracle.direct(s.pos, s.mass, eps=0.01)
    assert np.all(g["n_mono"] == 0) and np.all(g["n_p2p"] == s.n - 1)
    num = np.sqrt(((g["acc"] - d["acc"]) ** 2).sum() / (d["acc"] ** 2).sum())
    assert num <= 1e-13


def test_group_criterion_is_more_accurate(oracle_lib):
    s = icgen.plummer(6000, 9)
    T = oracle.Tree(s.pos, s.mass, 1)
    d = oracle.direct(s.pos, s.mass, eps=0.01)["acc"]
    err = lambda a: math.sqrt(((a - d) ** 2).sum() / (d ** 2).sum())
    per_body = T.walk(0.7, 0.01)
    grp = T.walk_group(0.7, 0.01, group=64)
    assert err(grp["acc"]) < err(per_body["acc"])
    assert grp["n_mono"].sum() + grp["n_p2p"].sum() > per_body["n_mono"].sum() + per_body["n_p2p"].sum()


def _clustered(n, seed):
    """Two distant Plummer-like clumps plus a few far strays and a knot of coincident bodies."""
    rng = np.random.default_rng(seed)
    pos = rng.normal(scale=0.3, size=(n, 3))
    pos[: n // 2, 0] += 6.0
    pos[n // 2:, 0] -= 6.0
    pos[:5] = rng.uniform(-20, 20, size=(5, 3))
    pos[10:90] = pos[10]
    mass = rng.uniform(0.5, 1.5, n)
    return pos, mass


@pytest.mark.parametrize("cap", [1, 8, 64])
def test_cube_groups_against_pointer_octree(oracle_lib, cap):
    """The groups of the library's group criterion, the largest cubes of at most cap bodies
    (oversized coincident leaves cut into runs), and the walk over them, against the pointer
    octree: the same partition of the bodies and the same interaction sets."""
    n = 400
    pos, mass = _clustered(n, cap)
    T = oracle.Tree(pos, mass, 1)
    starts = T.group_cubes(cap)
    ref, nodes, groups = py_group_walk(pos.tolist(), mass.tolist(), 0.6, 0.02, cap=cap)
    perm = T.perm.astype(np.int64)
    mine = [sorted(perm[starts[g]:starts[g + 1]].tolist()) for g in range(len(starts) - 1)]
    assert mine == [sorted(g) for g in groups]
    assert all(len(g) <= cap for g in groups)
    r = T.walk_group(0.6, 0.02, starts=starts)
    nn = len(nodes)
    for i in range(n):
        mono_ids, pairs, _ = ref[i]
        assert r["n_mono"][i] == len(mono_ids) and r["n_p2p"][i] == len(pairs)
        h = (sum(oracle.mix64(k) for k in mono_ids) + sum(oracle.mix64(nn + j) for j in pairs)) % (1 << 64)
        assert int(r["hash"][i]) == h


def test_cube_groups_of_one_are_the_per_body_walk(oracle_lib):
    s = icgen.plummer(2000, 19)
    T = oracle.Tree(s.pos, s.mass, 1)
    a = T.walk(0.6, 0.01)
    b = T.walk_group(0.6, 0.01, starts=T.group_cubes(1))
    for k in ("n_mono", "n_p2p", "hash"):
        assert np.array_equal(a[k], b[k]), k


def test_cube_groups_bound_the_work_of_separated_systems(oracle_lib):
    """Two distant spheres: key-consecutive groups of 64 that straddle the gap take almost
    every cube of the other sphere apart (work of order N per body); groups that never leave
    a cube of at most 64 bodies keep every body's work close to the per-body walk's."""
    s = icgen.two_plummer(8192, 3, 4)
    T = oracle.Tree(s.pos, s.mass, 1)
    per_body = T.walk(0.5, 0.005)
    pb = per_body["n_mono"] + per_body["n_p2p"]
    key = T.walk_group(0.5, 0.005, group=64)
    cube = T.walk_group(0.5, 0.005, starts=T.group_cubes(64))
    wk, wc = key["n_mono"] + key["n_p2p"], cube["n_mono"] + cube["n_p2p"]
    assert wk.max() > 0.5 * s.n
    assert wc.max() < 4 * pb.max()
    assert wc.sum() < 2 * pb.sum()
    # every group cube holds at most 64 bodies and is a cube of the tree
    st = T.group_cubes(64)
    assert np.diff(st).max() <= 64 and st[0] == 0 and st[-1] == s.n
