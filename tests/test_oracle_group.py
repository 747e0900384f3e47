"""Pins of the oracle's group-criterion walk (a cube is accepted for a
whole group of key-consecutive bodies when it passes against the group's bounding
box) against facts that do not come from that code: the per-body walk it must
equal for groups of one, an independent pure-Python group walk on the pointer
octree, the per-body criterion every accepted cube must also pass, direct
summation at theta = 0, and the accuracy ordering it implies.  CPU only."""
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


def py_group_walk(pos, mass, theta, eps, group):
    """Group criterion on the pointer octree (no keys): bodies ordered by the depth-first
    leaf order (one body per leaf), groups of `group` consecutive bodies."""
    root, nodes, lo, L = ptree.build(pos, mass, 1)
    order = [nd.ids[0] for nd in nodes if not nd.children]
    out = {}
    for g0 in range(0, len(order), group):
        members = order[g0:g0 + group]
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
    return out, nodes


@pytest.mark.parametrize("group", [4, 16, 64])
def test_against_pointer_octree(oracle_lib, group):
    rng = np.random.default_rng(group)
    n = 300
    pos = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    T = oracle.Tree(pos, mass, 1)
    r = T.walk_group(0.6, 0.02, group=group)
    ref, nodes = py_group_walk(pos.tolist(), mass.tolist(), 0.6, 0.02, group)
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
