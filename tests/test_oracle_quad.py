"""Pins of the oracle's quadrupole option (the multipole extension the paper names
as future work, section 6) against facts that do not come from the oracle: hand
moments, translation invariance, the convergence order of the expansion against
direct summation, the force as minus the gradient of the potential, and the
vanishing quadrupole of a cube of equal masses.  CPU only."""
import numpy as np
import pytest

import oracle


def node_of_root(T):
    return 0


def test_moments_by_hand(oracle_lib):
    # two masses of 2 at (1 +- 0.5, 3, -2): S = diag(2 * 2 * 0.25, 0, 0) about the centre
    pos = np.array([[0.5, 3.0, -2.0], [1.5, 3.0, -2.0]])
    T = oracle.Tree(pos, np.array([2.0, 2.0]), 1)
    S = T.moments()
    assert np.array_equal(T.com[0], [1.0, 3.0, -2.0])
    assert np.array_equal(S[0], [1.0, 0, 0, 0, 0, 0])
    # one-particle leaves have no second moment
    assert np.all(S[T.nchild == 0] == 0.0)
    # a cross: masses 1 at +-e_x, +-e_y (centre 0): S = diag(2, 2, 0); off-diagonals 0
    pos = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
    T = oracle.Tree(pos, np.ones(4), 1)
    assert np.allclose(T.moments()[0], [2.0, 2.0, 0, 0, 0, 0], atol=1e-15)
    # a tilted pair: masses 1 at +-(1, 1, 0): S_xy = 2
    pos = np.array([[1.0, 1.0, 0.0], [-1.0, -1.0, 0.0]])
    T = oracle.Tree(pos, np.ones(2), 1)
    assert np.allclose(T.moments()[0], [2.0, 2.0, 0, 2.0, 0, 0], atol=1e-15)


def test_moments_translation_invariant(oracle_lib):
    rng = np.random.default_rng(3)
    pos = rng.normal(size=(300, 3))
    mass = rng.uniform(0.5, 1.5, 300)
    S0 = oracle.Tree(pos, mass, 4).moments()[0]
    S1 = oracle.Tree(pos + np.array([1000.0, -77.0, 3.5]), mass, 4).moments()[0]
    assert np.allclose(S0, S1, rtol=1e-9, atol=1e-9 * np.abs(S0).max())


def far_cluster(b, seed=5, k=200, D=20.0):
    """k unit-ish masses within radius b of the origin, plus one light target at D on a skew axis."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(k, 3))
    u = u / np.linalg.norm(u, axis=1, keepdims=True) * rng.uniform(0, 1, (k, 1)) ** (1 / 3)
    pos = np.vstack([b * u, D * np.array([[0.8, 0.5, 0.33166247903554]])])
    mass = np.concatenate([rng.uniform(0.5, 1.5, k), [1e-9]])
    return pos, mass


@pytest.mark.parametrize("eps", [0.0, 0.3, 5.0])
def test_expansion_order_against_direct(oracle_lib, eps):
    """At a far target the cluster is one accepted cube: the monopole error falls as (b/D)^2,
    with the quadrupole as (b/D)^3, and the quadrupole is far more accurate."""
    errs = {False: [], True: []}
    for b in (1.0, 0.5, 0.25):
        pos, mass = far_cluster(b)
        tgt = np.array([len(mass) - 1], dtype=np.int64)
        ref = oracle.direct(pos, mass, eps=eps, targets=tgt)
        T = oracle.Tree(pos, mass, 1)
        for q in (False, True):
            r = T.walk(0.9, eps, 1.0, tgt, quad=q)
            assert r["n_mono"][0] >= 1 and r["n_p2p"][0] == 0     # the cluster is taken as cubes
            errs[q].append(np.linalg.norm(r["acc"][0] - ref["acc"][0]) / np.linalg.norm(ref["acc"][0]))
    m, q = np.array(errs[False]), np.array(errs[True])
    assert np.all(q < m / 10)
    # halving b: monopole error / 4, quadrupole error / 8 (within a factor 1.6)
    assert np.all((m[:-1] / m[1:] > 4 / 1.6) & (m[:-1] / m[1:] < 4 * 1.6))
    assert np.all((q[:-1] / q[1:] > 8 / 1.6) & (q[:-1] / q[1:] < 8 * 1.6))


def test_quad_force_is_minus_gradient_of_potential(oracle_lib):
    pos, mass = far_cluster(1.0, D=6.0)
    i = len(mass) - 1
    T = oracle.Tree(pos, mass, 1)
    a = T.walk(0.9, 0.2, 1.0, np.array([i], dtype=np.int64), quad=True)["acc"][0]
    h = 1e-5
    g = np.zeros(3)
    for k in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += h
        pm[i, k] -= h
        fp = oracle.Tree(pp, mass, 1).walk(0.9, 0.2, 1.0, np.array([i], dtype=np.int64), quad=True)["pot"][0]
        fm = oracle.Tree(pm, mass, 1).walk(0.9, 0.2, 1.0, np.array([i], dtype=np.int64), quad=True)["pot"][0]
        g[k] = (fp - fm) / (2 * h)
    assert np.allclose(a, -g, rtol=1e-6, atol=1e-9 * np.abs(a).max())


def test_cube_of_equal_masses_has_no_quadrupole(oracle_lib):
    # 8 equal masses at the corners of a cube: isotropic second moments, so with eps = 0 the
    # quadrupole term vanishes and quad == monopole at a far target
    c = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], dtype=float)
    pos = np.vstack([c * 0.5, [[15.0, 4.0, -7.0]]])
    mass = np.concatenate([np.ones(8), [1e-9]])
    T = oracle.Tree(pos, mass, 1)
    S = T.moments()[0]
    tgt = np.array([8], dtype=np.int64)
    r0 = T.walk(0.9, 0.0, 1.0, tgt, quad=False)
    r1 = T.walk(0.9, 0.0, 1.0, tgt, quad=True)
    assert r0["n_mono"][0] >= 1
    assert np.allclose(r1["acc"], r0["acc"], rtol=1e-14, atol=0)


def test_theta_zero_ignores_quad(oracle_lib):
    rng = np.random.default_rng(9)
    pos = rng.normal(size=(500, 3))
    mass = rng.uniform(0.5, 1.5, 500)
    T = oracle.Tree(pos, mass, 1)
    r0 = T.walk(0.0, 0.05, 1.0, quad=False)
    r1 = T.walk(0.0, 0.05, 1.0, quad=True)
    assert np.array_equal(r0["acc"], r1["acc"]) and np.array_equal(r0["pot"], r1["pot"])
