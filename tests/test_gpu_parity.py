"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same
seeded inputs.  Keys, order, topology, masses and centres of mass bit-exact;
forces within the FP64 (1e-10 RMS) and FP32 (2e-6 RMS, 1e-4 max) gates with
per-body interaction counts and set checksums equal."""
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


def system(kind, n, seed):
    if kind == "plummer":
        return icgen.plummer(n, seed)
    if kind == "uniform":
        return icgen.uniform_cube(n, seed)
    if kind == "duplicates":
        s = icgen.plummer(n, seed)
        pos = np.round(s.pos * 4.0) / 4.0
        pos[: n // 4] = pos[0]
        return icgen.System(pos, s.vel, s.mass)
    if kind == "coincident":
        return icgen.System(np.tile([[0.25, -1.5, 3.0]], (n, 1)), np.zeros((n, 3)), np.full(n, 1.0 / n))
    if kind == "two_spheres":
        h = n // 2
        return icgen.two_plummer(h, seed, seed + 1)
    raise ValueError(kind)


TREE_CASES = [
    ("plummer", 4096, 1, 1),      # the small workload: one tile
    ("plummer", 4096, 1, 16),
    ("uniform", 10001, 5, 1),     # three tiles with a ragged tail
    ("duplicates", 5000, 7, 1),
    ("duplicates", 5000, 7, 8),
    ("two_spheres", 9000, 3, 4),
    ("plummer", 1, 2, 1),
    ("plummer", 2, 2, 1),
    ("coincident", 3, 0, 1),
    ("coincident", 700, 0, 16),
    ("plummer", 64, 9, 64),       # whole system in one leaf
    ("plummer", 65, 9, 64),
]


@pytest.mark.parametrize("kind,n,seed,leaf_cap", TREE_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tree_bit_exact(ctx, kind, n, seed, leaf_cap, prec):
    print(f"[tree] {kind} n={n} seed={seed} leaf_cap={leaf_cap} {prec}", flush=True)
    s = system(kind, n, seed)
    T = oracle.Tree(s.pos, s.mass, leaf_cap)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01, leaf_cap=leaf_cap, precision=prec)).upward()
    ex = t.export()
    ctx.sync()
    assert ex["n_nodes"] == T.nn
    assert ex["k"] == T.k and np.array_equal(np.array(ex["lo"]), T.lo)
    assert np.array_equal(u64(ex["keys"]), T.keys)
    assert np.array_equal(ex["perm"].cpu().numpy().astype(np.uint32), T.perm)
    assert np.array_equal(ex["level"].cpu().numpy(), T.level)
    assert np.array_equal(ex["first"].cpu().numpy().astype(np.uint32), T.first)
    assert np.array_equal(ex["count"].cpu().numpy().astype(np.uint32), T.count)
    assert np.array_equal(ex["parent"].cpu().numpy(), T.parent)
    assert np.array_equal(ex["M"].cpu().numpy(), T.M)           # bit-exact FP64
    assert np.array_equal(ex["com"].cpu().numpy(), T.com)


WALK_CASES = [
    ("plummer", 4096, 1, 0.5, 0.01, 1),
    ("plummer", 4096, 1, 0.5, 0.01, 16),
    ("plummer", 4096, 1, 0.3, 0.01, 1),
    ("plummer", 4096, 1, 0.7, 0.01, 1),
    ("plummer", 20000, 4, 1.0, 0.0, 1),   # unsoftened: close pairs dominate the error norm
    ("plummer", 4096, 1, 1.0, 0.01, 1),
    ("uniform", 20001, 5, 0.5, 0.005, 1),
    ("two_spheres", 20000, 3, 0.5, 0.005, 4),
    ("duplicates", 5000, 7, 0.6, 0.01, 2),
]


@pytest.mark.parametrize("kind,n,seed,theta,eps,leaf_cap", WALK_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_walk_parity(ctx, kind, n, seed, theta, eps, leaf_cap, prec):
    print(f"[walk] {kind} n={n} theta={theta} leaf_cap={leaf_cap} {prec}", flush=True)
    s = system(kind, n, seed)
    ref = oracle.forces(s.pos, s.mass, theta=theta, eps=eps, leaf_cap=leaf_cap)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(theta, eps, leaf_cap=leaf_cap, precision=prec)).upward()
    r = t.forces_stats(pot=True)
    ctx.sync()
    assert np.array_equal(r["n_mono"].cpu().numpy(), ref["n_mono"])
    assert np.array_equal(r["n_p2p"].cpu().numpy(), ref["n_p2p"])
    assert np.array_equal(u64(r["hash"]), ref["hash"])
    acc = r["acc"].cpu().numpy()
    pot = r["pot"].cpu().numpy()
    if prec == "fp64":
        assert rel_rms(acc, ref["acc"]) <= 1e-10
        assert rel_rms(pot[:, None], ref["pot"][:, None]) <= 1e-10
    else:
        assert rel_rms(acc, ref["acc"]) <= 2e-6
        assert rel_max(acc, ref["acc"]) <= 1e-4
        assert rel_rms(pot[:, None], ref["pot"][:, None]) <= 2e-6
    tot = r["totals"]
    assert tot["n_mono"] == ref["n_mono"].sum() and tot["n_p2p"] == ref["n_p2p"].sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_theta_zero_is_direct_sum(ctx, prec):
    s = icgen.plummer(3000, 4)
    d = oracle.direct(s.pos, s.mass, eps=0.01)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.0, 0.01, precision=prec)).upward()
    r = t.forces_stats()
    ctx.sync()
    assert np.all(r["n_p2p"].cpu().numpy() == 2999) and np.all(r["n_mono"].cpu().numpy() == 0)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert rel_rms(r["acc"].cpu().numpy(), d["acc"]) <= tol


def test_fp64_pair_term_accuracy(ctx):
    """FP64 pair terms against the closed form m d / |d|^3 for single pairs at separations over 40
    binades (a forest of 256 two-body simulations, theta = 0, no softening).  The walk corrects
    the force factor of the hardware reciprocal square root estimate y to first order in its
    residual, m y^3 (1 + 3e/2) with e = 1 - x y^2, which leaves 7.5 times the square of the
    estimate's relative error (below 2^-24, so about 2.7e-14) plus a few roundings; an error in
    the correction would leave the estimate's own error, of order 1e-8."""
    rng = np.random.default_rng(11)
    K = 256
    pos = np.zeros((2 * K, 3))
    for s in range(K):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        pos[2 * s + 1] = d * np.ldexp(1.0 + rng.random(), -20 + (40 * s) // K)   # the other body at the origin
    mass = np.tile([0.5, 0.25], K)
    plist = [bh.params(0.0, 0.0, precision="fp64") for _ in range(K)]
    forest = bh.Forest(ctx, [2] * K, plist, dev(pos), dev(np.zeros_like(pos)), dev(mass))
    acc = forest.forces().cpu().numpy()
    ctx.sync()
    P = pos.astype(np.longdouble)
    d = P[1::2] - P[0::2]
    r2 = (d * d).sum(axis=1)
    r3 = (r2 * np.sqrt(r2))[:, None]
    ref = np.empty((2 * K, 3), dtype=np.longdouble)
    ref[0::2] = 0.25 * d / r3
    ref[1::2] = -0.5 * d / r3
    err = np.sqrt(((acc - ref) ** 2).sum(axis=1)) / np.sqrt((ref ** 2).sum(axis=1))
    assert float(err.max()) <= 5e-14


def test_forces_plain_equals_stats_variant(ctx):
    s = icgen.plummer(4096, 1)
    for prec in ("fp64", "fp32"):
        t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01, precision=prec)).upward()
        a = t.forces()
        r = t.forces_stats()
        ctx.sync()
        assert torch.equal(a, r["acc"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rebuild_equals_fresh_tree(ctx, prec):
    """bh_rebuild in the workspace of a tree built on other positions (a different root cube and
    node count) gives the fresh build's tree and forces bit for bit, and the oracle's tree."""
    a, b = icgen.plummer(6000, 21), icgen.uniform_cube(6000, 22)
    p = bh.params(0.6, 0.01, precision=prec)
    t = bh.Tree(ctx, dev(a.pos), dev(a.mass), p).upward()
    t.forces()
    pos_b, mass_b = dev(b.pos), dev(b.mass)
    t.rebuild(pos_b, mass_b).upward()
    fresh = bh.Tree(ctx, pos_b, mass_b, p).upward()
    ex, ef = t.export(), fresh.export()
    ctx.sync()
    T = oracle.Tree(b.pos, b.mass, 1)
    assert ex["n_nodes"] == ef["n_nodes"] == T.nn
    for k in ("keys", "perm", "level", "first", "count", "parent", "M", "com"):
        assert torch.equal(ex[k], ef[k]), k
    assert np.array_equal(ex["com"].cpu().numpy(), T.com)
    assert torch.equal(t.forces(), fresh.forces())
