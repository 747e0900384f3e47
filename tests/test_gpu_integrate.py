"""GPU: KDK steps, energies, forests (batched simulations), graph replay and
device-side initial conditions, against the oracle and against each other."""
import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_helpers import dev, rel_max, rel_rms

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


def test_kdk_c1_fp64_matches_oracle(ctx):
    """Small workload: Plummer 4096, one force evaluation + one KDK step, dt = 1e-3."""
    s = icgen.plummer(4096, 1)
    pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
    sim = bh.Sim(ctx, pos, vel, mass, bh.params(0.5, 0.01, precision="fp64"))
    sim.step(1, 1e-3)
    ctx.sync()
    x, v, a, _ = oracle.kdk(s.pos, s.vel, s.mass, 1e-3, 1, theta=0.5, eps=0.01)
    assert np.abs(pos.cpu().numpy() - x).max() <= 1e-13 * np.abs(x).max()
    assert np.abs(vel.cpu().numpy() - v).max() <= 1e-12 * np.abs(v).max()
    assert rel_rms(sim.acc.cpu().numpy(), a) <= 1e-10
    # and against direct summation at the new positions (approximation error, reported bound)
    d = oracle.direct(x, s.mass, eps=0.01)
    assert rel_rms(sim.acc.cpu().numpy(), d["acc"]) < 5e-2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_multi_step_parity(ctx, prec, tol):
    """10 KDK steps with a rebuild every step; forces compared with the oracle's own trajectory."""
    s = icgen.plummer(20000, 2)
    pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
    sim = bh.Sim(ctx, pos, vel, mass, bh.params(0.5, 0.005, precision=prec))
    xo, vo, ao = s.pos, s.vel, None
    for k in range(2):
        sim.step(5, 1e-4)
        ctx.sync()
        xo, vo, ao, _ = oracle.kdk(xo, vo, s.mass, 1e-4, 5, theta=0.5, eps=0.005, acc=ao)
        acc = sim.acc.cpu().numpy()
        assert rel_rms(acc, ao) <= tol, (k, rel_rms(acc, ao))
        if prec == "fp32":
            assert rel_max(acc, ao) <= 1e-4
        assert np.abs(pos.cpu().numpy() - xo).max() <= 1e-9


def test_energy_matches_oracle(ctx):
    s = icgen.plummer(4096, 1)
    sim = bh.Sim(ctx, dev(s.pos), dev(s.vel), dev(s.mass), bh.params(0.5, 0.01, precision="fp64"))
    K, W = sim.energy()
    r = oracle.forces(s.pos, s.mass, theta=0.5, eps=0.01)
    Ko, Wo = oracle.energy(s.vel, s.mass, r["pot"])
    assert abs(K - Ko) <= 1e-13 * abs(Ko) and abs(W - Wo) <= 1e-10 * abs(Wo)
    assert abs(K / abs(W) - 0.5) < 0.03


def make_forest_inputs(ns, seeds):
    systems = [icgen.plummer(n, sd) for n, sd in zip(ns, seeds)]
    return systems, icgen.concat(*systems)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forest_equals_standalone(ctx, prec):
    """Each simulation's result inside a forest is bit-identical to running it alone."""
    ns = [1000, 4096, 70, 13000, 1, 5000]
    seeds = [11, 12, 13, 14, 15, 16]
    thetas = [0.4, 0.5, 0.7, 0.5, 0.5, 0.4]
    plist = [bh.params(t, 0.01, leaf_cap=1 if i % 2 else 8, precision=prec) for i, t in enumerate(thetas)]
    systems, cat = make_forest_inputs(ns, seeds)
    fpos, fvel, fmass = dev(cat.pos), dev(cat.vel), dev(cat.mass)
    forest = bh.Forest(ctx, ns, plist, fpos, fvel, fmass)
    forest.step(3, [1e-3] * len(ns))
    ctx.sync()
    off = 0
    for i, (n, sysm) in enumerate(zip(ns, systems)):
        p, v, m = dev(sysm.pos), dev(sysm.vel), dev(sysm.mass)
        sim = bh.Sim(ctx, p, v, m, plist[i])
        sim.step(3, 1e-3)
        ctx.sync()
        assert torch.equal(fpos[off:off + n], p), i
        assert torch.equal(fvel[off:off + n], v), i
        assert torch.equal(forest.acc[off:off + n], sim.acc), i
        off += n


def test_forest_forces_match_oracle(ctx):
    ns = [3000, 257, 9000]
    seeds = [21, 22, 23]
    plist = [bh.params(0.5, 0.01, leaf_cap=c, precision="fp64") for c in (1, 4, 16)]
    systems, cat = make_forest_inputs(ns, seeds)
    forest = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    acc = forest.forces().cpu().numpy()
    off = 0
    for n, sysm, c in zip(ns, systems, (1, 4, 16)):
        ref = oracle.forces(sysm.pos, sysm.mass, theta=0.5, eps=0.01, leaf_cap=c)
        assert rel_rms(acc[off:off + n], ref["acc"]) <= 1e-10
        off += n


def test_forest_graph_replay_equals_eager(ctx):
    """A step recorded as a HIP graph and replayed gives the eager result on every replay."""
    ns = [2000, 3000, 64]
    plist = [bh.params(0.5, 0.01, precision="fp32") for _ in ns]
    systems, cat = make_forest_inputs(ns, [31, 32, 33])
    ga = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    ea = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    for rep in range(4):
        ga.step_graph(1, 1e-3)
        ea.step(1, 1e-3)
        ctx.sync()
        # eager work between replays
        _ = (ea.pos * 2.0).sum().item()
        assert torch.equal(ga.pos, ea.pos), rep
        assert torch.equal(ga.vel, ea.vel), rep
        assert torch.equal(ga.acc, ea.acc), rep


@pytest.mark.parametrize("kind", [0, 1])
def test_device_initial_conditions_match_generator(ctx, kind):
    n, seed = 50000, 77
    pos, vel, mass = bh.ic_generate(ctx, kind, n, seed)
    ctx.sync()
    ref = icgen.plummer(n, seed) if kind == 0 else icgen.uniform_cube(n, seed)
    assert np.allclose(pos.cpu().numpy(), ref.pos, rtol=1e-12, atol=1e-12)
    assert np.allclose(vel.cpu().numpy(), ref.vel, rtol=1e-12, atol=1e-12)
    assert np.allclose(mass.cpu().numpy(), ref.mass, rtol=1e-15, atol=0)


def test_autotune_changes_no_result(ctx):
    """The walk's launch shape is chosen by timing; every shape gives the same bits."""
    ns = [3000, 700, 12000, 64]
    plist = [bh.params(0.5, 0.01, precision=pr) for pr in ("fp32", "fp64", "fp32", "fp64")]
    systems, cat = make_forest_inputs(ns, [41, 42, 43, 44])
    fo = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    ref = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    a0 = fo.forces().clone()
    shape, ms = fo.autotune()
    assert shape in bh.TUNE_SHAPES and sorted(ms) == sorted(bh.TUNE_SHAPES) and all(v > 0 for v in ms.values())
    assert torch.equal(fo.acc, a0)          # the last timed shape
    assert torch.equal(fo.forces(), a0)     # the chosen shape
    fo.step_graph(2, 1e-3)
    ref.step(2, 1e-3)
    ctx.sync()
    assert torch.equal(fo.pos, ref.pos) and torch.equal(fo.acc, ref.acc)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_split_and_resumed_runs_are_bit_identical(ctx, prec):
    """Checkpoint and resume: a simulation views caller memory, so its state is (pos, vel); six
    steps in one call, three + three calls on one simulation (the fused kick-kick between steps
    against a closing and an opening kick), and three steps, a copy of (pos, vel) into new
    tensors and three steps of a new simulation all give the same bits (the first force
    evaluation of the resumed run is the walk the first run did at the same positions)."""
    s = icgen.plummer(12000, 19)
    p = bh.params(0.5, 0.01, precision=prec)
    runs = []
    for split in ("one", "two", "resume"):
        pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
        sim = bh.Sim(ctx, pos, vel, mass, p)
        if split == "one":
            sim.step(6, 1e-3)
        else:
            sim.step(3, 1e-3)
            if split == "resume":
                pos, vel = pos.clone(), vel.clone()
                sim.close()
                sim = bh.Sim(ctx, pos, vel, mass, p)
            sim.step(3, 1e-3)
        ctx.sync()
        runs.append((pos, vel, sim.acc))
    for k in (1, 2):
        for a, b in zip(runs[0], runs[k]):
            assert torch.equal(a, b), k
