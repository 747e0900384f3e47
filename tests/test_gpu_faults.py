"""GPU: device fault reporting and recovery, and the boundary's outputs.

- A non-finite position or mass is reported as BH_E_DEVICE at the next
  synchronising call, the report clears the fault word, and the same tree
  rebuilt from clean inputs walks again and matches the oracle.
- A server iteration whose state blows up (a request with an absurd time step)
  fails that iteration's requests only: a request submitted afterwards runs to
  completion with the same bits as alone.
- bh_tree_export's node count and per-body checksums (and bh_stats.t_ms).
- Quadrupole moments with massless particles: ancestors of a massless child stay
  finite and the walk matches the oracle's quadrupole walk.
- bh_ic_generate refuses a missing or short workspace.
"""
import time

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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("where", ["position", "mass", "inf"])
def test_non_finite_input_reported_then_tree_recovers(ctx, prec, where):
    print(f"[faults] non-finite {where} {prec}", flush=True)
    s = icgen.plummer(3000, 11)
    pos, mass = dev(s.pos), dev(s.mass)
    bad_pos, bad_mass = pos.clone(), mass.clone()
    if where == "position":
        bad_pos[1234, 1] = float("nan")
    elif where == "mass":
        bad_mass[77] = float("nan")
    else:
        bad_pos[5, 0] = float("inf")
    p = bh.params(0.5, 0.01, precision=prec)
    t = bh.Tree(ctx, bad_pos, bad_mass, p).upward()
    t.forces()
    with pytest.raises(bh.BHError) as ei:
        ctx.sync()
    assert ei.value.status == bh.E_DEVICE
    ctx.sync()   # the report cleared the fault word
    t.rebuild(pos, mass).upward()
    r = t.forces_stats()
    ctx.sync()
    ref = oracle.forces(s.pos, s.mass, theta=0.5, eps=0.01)
    assert np.array_equal(r["n_mono"].cpu().numpy(), ref["n_mono"])
    assert np.array_equal(u64(r["hash"]), ref["hash"])
    assert rel_rms(r["acc"].cpu().numpy(), ref["acc"]) <= (1e-10 if prec == "fp64" else 2e-6)
    assert r["totals"]["t_ms"] > 0.0


def test_non_finite_state_in_a_simulation_is_reported(ctx):
    s = icgen.plummer(2048, 12)
    pos, vel, mass = dev(s.pos), dev(s.vel), dev(s.mass)
    sim = bh.Sim(ctx, pos, vel, mass, bh.params(0.5, 0.01, precision="fp32"))
    sim.step(1, 1e-3)
    ctx.sync()
    vel[9, 2] = float("nan")          # drifts into a position on the next step
    sim.step(2, 1e-3)
    with pytest.raises(bh.BHError) as ei:
        ctx.sync()
    assert ei.value.status == bh.E_DEVICE


def _wait(sv, rid, timeout=120.0):
    t0 = time.time()
    while True:
        r = sv.poll(rid)
        if r["state"] in ("done", "failed", "cancelled"):
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"request {rid} stuck in {r}")
        time.sleep(0.001)


def test_server_recovers_after_a_failed_iteration(ctx):
    sv = bh.Server(ctx, 1 << 30, max_slots=8, max_resident=1 << 18)
    p = bh.params(0.5, 0.01, precision="fp32")
    good = (4096, 3, 0, 501)
    rid = sv.submit(*good, p, 1e-3)
    r_alone = _wait(sv, rid)
    assert r_alone["state"] == "done"
    alone = sv.fetch(rid, good[0])
    # the absurd step size drives positions to infinity after one step: the next
    # iteration's build flags them and that iteration's requests fail
    bad = sv.submit(3000, 4, 1, 502, p, 1e300)
    r_bad = _wait(sv, bad)
    assert r_bad["state"] == "failed", r_bad
    rid2 = sv.submit(*good, p, 1e-3)
    r2 = _wait(sv, rid2)
    assert r2["state"] == "done", r2
    again = sv.fetch(rid2, good[0])
    assert torch.equal(alone[0], again[0]) and torch.equal(alone[1], again[1])
    assert r2["K"] == r_alone["K"] and r2["W"] == r_alone["W"]
    sv.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("group", [False, True])
def test_export_node_count_and_checksums(ctx, prec, group):
    s = icgen.plummer(5000, 13)
    p = bh.params(0.6, 0.01, precision=prec, group=group)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), p).upward()
    ex = t.export(with_hash=True)
    st = t.forces_stats()
    ctx.sync()
    T = oracle.Tree(s.pos, s.mass, 1)
    assert ex["n_nodes"] == T.nn
    ref = T.walk_group(0.6, 0.01, 1.0, starts=T.group_cubes(64)) if group else T.walk(0.6, 0.01)
    assert np.array_equal(u64(ex["isect_hash"]), ref["hash"])
    assert torch.equal(ex["isect_hash"], st["hash"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_quadrupole_with_massless_particles(ctx, prec):
    s = icgen.plummer(6000, 14)
    mass = s.mass.copy()
    rng = np.random.default_rng(3)
    mass[rng.choice(s.n, 300, replace=False)] = 0.0     # single massless bodies and a few massless cubes
    T = oracle.Tree(s.pos, mass, 1)
    ref = T.walk(0.6, 0.01, quad=True)
    p = bh.params(0.6, 0.01, precision=prec, quad=True)
    t = bh.Tree(ctx, dev(s.pos), dev(mass), p).upward()
    r = t.forces_stats()
    ctx.sync()
    acc = r["acc"].cpu().numpy()
    assert np.isfinite(acc).all()
    assert np.array_equal(r["n_mono"].cpu().numpy(), ref["n_mono"])
    assert np.array_equal(u64(r["hash"]), ref["hash"])
    if prec == "fp64":
        assert rel_rms(acc, ref["acc"]) <= 1e-10
    else:
        assert rel_rms(acc, ref["acc"]) <= 2e-6 and rel_max(acc, ref["acc"]) <= 1e-4


def test_ic_generate_needs_its_workspace(ctx):
    import ctypes as C
    n = 1000
    pos = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    vel = torch.empty_like(pos)
    mass = torch.empty(n, dtype=torch.float64, device="cuda")
    L = bh.lib()
    nb = L.bh_ic_workspace_bytes()
    _raw, ws = bh.workspace(nb, pos.device)
    args = (ctx.h, 0, n, 7, 1.0, 1.0, bh._ptr(pos), bh._ptr(vel), bh._ptr(mass))
    assert L.bh_ic_generate(*args, None, nb) == bh.E_INVAL
    assert L.bh_ic_generate(*args, bh._ptr(ws), nb - 8) == bh.E_NOMEM
    assert L.bh_ic_generate(*args, C.c_void_p(ws.data_ptr() + 8), nb) == bh.E_INVAL
    assert L.bh_ic_generate(*args, bh._ptr(ws), nb) == bh.OK
    ctx.sync()
    assert torch.isfinite(pos).all() and torch.isfinite(vel).all()


def test_handles_refuse_another_context(ctx):
    """A tree, simulation or forest belongs to the context it was created on: a call that passes
    another context is refused (BH_E_INVAL) and changes nothing; its own context still works."""
    s = icgen.plummer(2000, 15)
    p = bh.params(0.5, 0.01, precision="fp32")
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), p).upward()
    a = t.forces().clone()
    other = bh.Context(0)
    acc = torch.zeros_like(a)
    st = bh.lib().bh_forces(other.h, t.h, bh._ptr(acc), None)
    assert st == bh.E_INVAL
    assert "another context" in bh.lib().bh_last_error().decode()
    assert torch.count_nonzero(acc) == 0
    sim = bh.Sim(ctx, dev(s.pos), dev(s.vel), dev(s.mass), p)
    assert bh.lib().bh_step(other.h, sim.h, 1, bh.C.c_double(1e-3)) == bh.E_INVAL
    sim.step(1, 1e-3)
    ctx.sync()
    assert torch.equal(t.forces(), a)
    other.sync()

