"""Pins of the CPU oracle against facts that do not come from the oracle itself:
hand-worked key cases, an independent pointer octree, closed forms, direct
summation, brute force, invariants and the paper's Fig. 2 example.
Runs on the CPU only."""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import icgen
import oracle
from tests import ptree

GOLDEN = Path(__file__).resolve().parent / "golden"


# ----------------------------------------------------------------- keys ---

def deinterleave(key):
    q = [0, 0, 0]
    for b in range(21):
        q[0] |= ((key >> (3 * b + 2)) & 1) << b
        q[1] |= ((key >> (3 * b + 1)) & 1) << b
        q[2] |= ((key >> (3 * b)) & 1) << b
    return tuple(q)


def test_key_hand_cases(oracle_lib):
    g = json.loads((GOLDEN / "morton_keys.json").read_text())
    for case in g["cases"]:
        assert oracle.interleave(*case["q"]) == int(case["key"], 16), case


def test_key_roundtrip_and_level_order(oracle_lib):
    rng = np.random.default_rng(11)
    qs = rng.integers(0, 2 ** 21, size=(400, 3))
    keys = [oracle.interleave(int(a), int(b), int(c)) for a, b, c in qs]
    for (a, b, c), k in zip(qs, keys):
        assert deinterleave(k) == (a, b, c)
        assert k < 2 ** 63
    # key order == lexicographic order of the per-level octant digits (x is the MSB of each digit)
    def digits(q):
        return tuple(4 * ((q[0] >> (20 - l)) & 1) + 2 * ((q[1] >> (20 - l)) & 1) + ((q[2] >> (20 - l)) & 1)
                     for l in range(21))
    by_key = sorted(range(len(keys)), key=lambda i: keys[i])
    by_digits = sorted(range(len(keys)), key=lambda i: digits(tuple(int(v) for v in qs[i])))
    assert by_key == by_digits


def test_root_cube_cases(oracle_lib):
    g = json.loads((GOLDEN / "root_cube.json").read_text())
    for case in g["cases"]:
        pos = np.array(case["pos"], dtype=np.float64)
        lo, k = oracle.root_cube(pos)
        assert 2.0 ** k == case["L"], case
        assert np.array_equal(lo, pos.min(axis=0))


def test_keys_from_positions_match_independent_quantisation(oracle_lib):
    s = icgen.plummer(3000, 5)
    lo, k = oracle.root_cube(s.pos)
    L = 2.0 ** k
    ext = (s.pos.max(0) - s.pos.min(0)).max()
    assert ext < L <= 2 * ext
    keys = oracle.keys(s.pos, lo, k)
    off = s.pos - lo                      # same IEEE subtraction
    q = np.floor(off * 2.0 ** (21 - k)).astype(np.int64)
    assert q.min() >= 0 and q.max() < 2 ** 21
    for i in range(0, 3000, 7):
        assert deinterleave(int(keys[i])) == tuple(int(v) for v in q[i])


def test_order_is_key_then_index(oracle_lib):
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 50, size=5000).astype(np.uint64)     # many ties
    perm = oracle.order(keys)
    ref = np.lexsort((np.arange(5000), keys))
    assert np.array_equal(perm.astype(np.int64), ref)


# ----------------------------------------------------------------- tree ---

def oracle_node_list(T):
    out = []
    for n in range(T.nn):
        lvl = int(T.level[n])
        ids = sorted(int(i) for i in T.perm[T.first[n]:T.first[n] + T.count[n]])
        cell = deinterleave(int(T.keys[T.first[n]]) >> (3 * (21 - lvl)) << (3 * (21 - lvl)))
        cell = tuple(c >> (21 - lvl) for c in cell)
        out.append((lvl, cell, tuple(ids), int(T.parent[n])))
    return out


def ptree_node_list(nodes):
    parent = {}
    for nd in nodes:
        for c in nd.children:
            parent[c.pre] = nd.pre
    return [(nd.level, nd.cell, tuple(sorted(nd.ids)), parent.get(nd.pre, -1)) for nd in nodes]


def inputs_for(kind, n, seed):
    if kind == "uniform":
        return icgen.uniform_cube(n, seed)
    if kind == "plummer":
        return icgen.plummer(n, seed)
    if kind == "duplicates":
        s = icgen.plummer(n, seed)
        pos = np.round(s.pos * 4.0) / 4.0                 # heavy coincidence
        pos[: n // 4] = pos[0]                            # a block of identical points
        return icgen.System(pos, s.vel, s.mass)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "plummer", "duplicates"])
@pytest.mark.parametrize("leaf_cap", [1, 4, 16])
def test_topology_matches_pointer_octree(oracle_lib, kind, leaf_cap):
    s = inputs_for(kind, 1500, 21)
    T = oracle.Tree(s.pos, s.mass, leaf_cap)
    root, nodes, lo, L = ptree.build(s.pos, s.mass, leaf_cap)
    assert L == T.L and np.array_equal(np.array(lo), T.lo)
    assert oracle_node_list(T) == ptree_node_list(nodes)


@pytest.mark.parametrize("leaf_cap", [1, 3, 8])
def test_tree_invariants(oracle_lib, leaf_cap):
    s = inputs_for("duplicates", 2500, 4)
    T = oracle.Tree(s.pos, s.mass, leaf_cap)
    assert T.level[0] >= 0 and T.parent[0] == -1 and T.first[0] == 0 and T.count[0] == T.n
    kids = {n: [] for n in range(T.nn)}
    for n in range(1, T.nn):
        p = int(T.parent[n])
        assert 0 <= p < n                                 # preorder: parent first
        assert T.level[n] > T.level[p]
        kids[p].append(n)
    for n in range(T.nn):
        lvl = int(T.level[n])
        f, c = int(T.first[n]), int(T.count[n])
        pref = T.keys[f:f + c] >> np.uint64(3 * (21 - lvl))
        assert np.all(pref == pref[0])                    # the cube holds its particles
        if kids[n]:
            assert len(kids[n]) >= 2 and T.nchild[n] == len(kids[n])
            # children partition the parent range in ascending order
            pos_ = f
            for ch in kids[n]:
                assert T.first[ch] == pos_
                pos_ += int(T.count[ch])
            assert pos_ == f + c
            assert c > leaf_cap
        else:
            assert c <= leaf_cap or lvl == 21


def test_tree_edge_cases(oracle_lib):
    one = oracle.Tree(np.array([[0.5, -1.0, 2.0]]), np.array([1.0]), 1)
    assert one.nn == 1 and one.level[0] == 0 and one.count[0] == 1 and one.k == 0
    same = oracle.Tree(np.tile([[1.0, 2.0, 3.0]], (10, 1)), np.full(10, 0.1), 1)
    assert same.nn == 1 and same.level[0] == 21 and same.count[0] == 10 and same.L == 1.0
    few = oracle.Tree(icgen.plummer(12, 1).pos, np.full(12, 1 / 12), 16)
    assert few.nn == 1 and few.level[0] == 0 and few.count[0] == 12
    two = oracle.Tree(np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]), np.array([0.5, 0.5]), 1)
    # ext = 1 -> L = 2; the two points sit in octants 0 and 7 of the root
    assert two.nn == 3 and list(two.level) == [0, 1, 1] and two.L == 2.0


# --------------------------------------------------------------- upward ---

def test_upward_mass_and_centre(oracle_lib):
    s = icgen.plummer(3000, 8)
    s.mass[:] = np.linspace(0.5, 1.5, 3000) / 3000
    T = oracle.Tree(s.pos, s.mass, 1)
    u = np.finfo(float).eps
    assert abs(T.M[0] - math.fsum(s.mass)) <= 3000 * u * math.fsum(s.mass)
    gcom = np.array([math.fsum(s.mass * s.pos[:, d]) for d in range(3)]) / math.fsum(s.mass)
    scale = np.abs(s.pos).max()
    assert np.all(np.abs(T.com[0] - gcom) <= 3000 * u * scale)
    leaves = np.where((T.nchild == 0) & (T.count == 1))[0]
    for n in leaves[:200]:
        j = int(T.perm[T.first[n]])
        m = s.mass[j]
        assert T.M[n] == m
        assert np.array_equal(T.com[n], (m * s.pos[j]) / m)
    # every internal node: M is the sum over its particles (any order, to round-off)
    for n in range(0, T.nn, 13):
        ids = T.perm[T.first[n]:T.first[n] + T.count[n]]
        assert abs(T.M[n] - math.fsum(s.mass[ids])) <= len(ids) * u * T.M[n]


# ----------------------------------------------------------------- walk ---

def rel_rms(a, b):
    return math.sqrt(((a - b) ** 2).sum() / (b ** 2).sum())


@pytest.mark.parametrize("leaf_cap", [1, 8])
def test_theta_zero_is_direct_sum(oracle_lib, leaf_cap):
    s = icgen.plummer(2048, 2)
    T = oracle.Tree(s.pos, s.mass, leaf_cap)
    r = T.walk(theta=0.0, eps=0.01)
    d = oracle.direct(s.pos, s.mass, eps=0.01)
    assert rel_rms(r["acc"], d["acc"]) <= 1e-13
    assert rel_rms(r["pot"][:, None], d["pot"][:, None]) <= 1e-13
    assert np.all(r["n_mono"] == 0) and np.all(r["n_p2p"] == 2047)
    mixes = np.array([oracle.mix64(T.nn + j) for j in range(2048)], dtype=np.uint64)
    total = np.uint64(0)
    with np.errstate(over="ignore"):
        for v in mixes:
            total = total + v
        for i in range(0, 2048, 97):
            assert r["hash"][i] == total - mixes[i]


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7, 1.0])
@pytest.mark.parametrize("n,leaf_cap", [(64, 1), (64, 4), (40, 1)])
def test_brute_force_textbook_walk(oracle_lib, theta, n, leaf_cap):
    s = icgen.plummer(n, 100 + n)
    T = oracle.Tree(s.pos, s.mass, leaf_cap)
    root, nodes, lo, L = ptree.build(s.pos, s.mass, leaf_cap)
    assert oracle_node_list(T) == ptree_node_list(nodes)
    r = T.walk(theta=theta, eps=0.01)
    for i in range(n):
        acc, mono, pairs = ptree.walk(root, nodes, s.pos, s.mass, L, i, theta, 0.01)
        assert r["n_mono"][i] == len(mono) and r["n_p2p"][i] == len(pairs)
        h = sum(oracle.mix64(m) for m in mono) + sum(oracle.mix64(T.nn + j) for j in pairs)
        assert int(r["hash"][i]) == h % 2 ** 64
        assert np.allclose(r["acc"][i], acc, rtol=1e-12, atol=1e-14 * np.abs(acc).max())


def test_two_body_closed_form(oracle_lib):
    pos = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.2]])
    mass = np.array([2.0, 5.0])
    eps, G = 0.1, 1.5
    r = oracle.forces(pos, mass, theta=0.5, eps=eps, G=G)
    d = pos[1] - pos[0]
    r2 = d @ d + eps * eps
    assert np.allclose(r["acc"][0], G * mass[1] * d / r2 ** 1.5, rtol=1e-15)
    assert np.allclose(r["acc"][1], -G * mass[0] * d / r2 ** 1.5, rtol=1e-15)
    assert np.allclose(r["pot"], [-G * mass[1] / math.sqrt(r2), -G * mass[0] / math.sqrt(r2)], rtol=1e-15)


def test_single_particle_feels_nothing(oracle_lib):
    r = oracle.forces(np.array([[1.0, 2.0, 3.0]]), np.array([1.0]), theta=0.7, eps=0.0)
    assert np.all(r["acc"] == 0.0) and r["n_mono"][0] == 0 and r["n_p2p"][0] == 0 and r["hash"][0] == 0


def test_symmetric_cube_corners_cancel(oracle_lib):
    c = np.array([[x, y, z] for x in (-1.0, 1.0) for y in (-1.0, 1.0) for z in (-1.0, 1.0)])
    pos = np.vstack([[0.0, 0.0, 0.0], c])
    mass = np.ones(9)
    for theta in (0.0, 0.5, 1.0):
        r = oracle.forces(pos, mass, theta=theta, eps=0.05)
        assert np.abs(r["acc"][0]).max() <= 1e-15


def test_fig2_worked_example(oracle_lib):
    """Paper Fig. 2: P3 and P4 collapse into one node, so P1 needs two inputs (P2 and N2)."""
    g = json.loads((GOLDEN / "fig2_example.json").read_text())
    pos = np.array(g["pos"])
    mass = np.array(g["mass"])
    T = oracle.Tree(pos, mass, 1)
    r = T.walk(theta=g["theta"], eps=g["eps"])
    # N2: the node holding exactly P3 and P4
    n2 = [n for n in range(T.nn) if sorted(T.perm[T.first[n]:T.first[n] + T.count[n]]) == [2, 3]]
    assert len(n2) == 1
    n2 = n2[0]
    assert T.level[n2] == g["n2_level"]
    for i in (0, 1):
        other = 1 - i
        assert r["n_mono"][i] == 1 and r["n_p2p"][i] == 1
        assert int(r["hash"][i]) == (oracle.mix64(n2) + oracle.mix64(T.nn + other)) % 2 ** 64
        want = np.zeros(3)
        for y, m in ((pos[other], mass[other]), (T.com[n2], T.M[n2])):
            d = y - pos[i]
            r2 = d @ d + g["eps"] ** 2
            want += m * d / r2 ** 1.5
        assert np.allclose(r["acc"][i], want, rtol=1e-14)


def test_momentum_conserved_at_theta_zero(oracle_lib):
    s = icgen.plummer(1024, 9)
    s.mass[:] = np.linspace(0.2, 1.8, 1024) / 1024
    r = oracle.forces(s.pos, s.mass, theta=0.0, eps=0.01)
    P = (s.mass[:, None] * r["acc"]).sum(0)
    scale = (s.mass * np.linalg.norm(r["acc"], axis=1)).sum()
    assert np.abs(P).max() <= 64 * np.finfo(float).eps * scale


def test_approximation_improves_as_theta_shrinks(oracle_lib):
    s = icgen.plummer(4096, 1)
    T = oracle.Tree(s.pos, s.mass, 1)
    d = oracle.direct(s.pos, s.mass, eps=0.01)
    errs = [rel_rms(T.walk(theta=t, eps=0.01)["acc"], d["acc"]) for t in (1.0, 0.7, 0.5, 0.3)]
    assert errs[2] < 5e-2
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    counts = [T.walk(theta=t, eps=0.01)["n_mono"].mean() for t in (1.0, 0.7, 0.5, 0.3)]
    assert counts == sorted(counts)


# ------------------------------------------------------------ integrator ---

def test_kdk_time_reversible(oracle_lib):
    s = icgen.plummer(256, 12)
    x1, v1, a1, _ = oracle.kdk(s.pos, s.vel, s.mass, dt=1e-3, nsteps=5, theta=0.0, eps=0.01)
    x2, v2, a2, _ = oracle.kdk(x1, v1, s.mass, dt=-1e-3, nsteps=5, theta=0.0, eps=0.01, acc=a1)
    assert np.abs(x2 - s.pos).max() <= 1e-12 * np.abs(s.pos).max()
    assert np.abs(v2 - s.vel).max() <= 1e-11 * np.abs(s.vel).max()


def test_kdk_energy_error_second_order(oracle_lib):
    s = icgen.plummer(128, 13)
    d0 = oracle.direct(s.pos, s.mass, eps=0.05)
    E0 = sum(oracle.energy(s.vel, s.mass, d0["pot"]))
    errs = []
    for dt, n in ((4e-3, 25), (2e-3, 50)):
        x, v, a, pot = oracle.kdk(s.pos, s.vel, s.mass, dt=dt, nsteps=n, theta=0.0, eps=0.05)
        errs.append(abs(sum(oracle.energy(v, s.mass, pot)) - E0))
    ratio = errs[0] / errs[1]
    assert 2.5 < ratio < 6.0, (errs, ratio)


def test_kdk_one_step_by_hand(oracle_lib):
    s = icgen.plummer(64, 14)
    a0 = oracle.forces(s.pos, s.mass, theta=0.5, eps=0.01)["acc"]
    dt = 1e-3
    v_half = s.vel + (0.5 * dt) * a0
    x1 = s.pos + dt * v_half
    a1 = oracle.forces(x1, s.mass, theta=0.5, eps=0.01)["acc"]
    v1 = v_half + (0.5 * dt) * a1
    x, v, a, _ = oracle.kdk(s.pos, s.vel, s.mass, dt=dt, nsteps=1, theta=0.5, eps=0.01)
    assert np.array_equal(x, x1) and np.array_equal(v, v1) and np.array_equal(a, a1)
