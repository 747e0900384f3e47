"""GPU: the continuous-batching server.  Each request's result is the same alone
and in the mix (bit for bit), equals a plain simulation from the same device
initial conditions, and admission/cancel/error paths behave."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bh = pytest.importorskip("paper_1109_5190_amd")

GiB = 1 << 30


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bh.Context(0)
    yield c
    c.sync()


def wait(sv, rid, timeout=60.0):
    t0 = time.time()
    while True:
        r = sv.poll(rid)
        if r["state"] in ("done", "failed", "cancelled"):
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"request {rid} stuck in {r}")
        time.sleep(0.001)


REQS = [  # (n, steps, kind, seed, theta, precision)
    (3000, 5, 0, 101, 0.5, "fp32"),
    (20000, 3, 1, 102, 0.7, "fp64"),
    (64, 7, 0, 103, 0.4, "fp32"),
    (9000, 1, 0, 104, 0.5, "fp64"),
    (1, 4, 1, 105, 0.5, "fp32"),
    (15000, 6, 0, 106, 0.5, "fp32"),
    (5000, 0, 1, 107, 0.5, "fp64"),
    (12000, 2, 0, 108, 0.5, "fp32"),
]


def submit(sv, req, dt=1e-3):
    n, steps, kind, seed, theta, prec = req
    return sv.submit(n, steps, kind, seed, bh.params(theta, 0.01, precision=prec), dt)


def test_alone_equals_mix_and_equals_plain_simulation(ctx):
    sv = bh.Server(ctx, 2 * GiB, max_slots=16, max_resident=1 << 20)
    alone = []
    for req in REQS:
        rid = submit(sv, req)
        r = wait(sv, rid)
        assert r["state"] == "done", r
        alone.append((sv.fetch(rid, req[0]), r))
    # all at once, plus staggered arrivals while others run
    ids = [submit(sv, req) for req in REQS[:5]]
    time.sleep(0.01)
    ids += [submit(sv, req) for req in REQS[5:]]
    mixed = []
    for rid, req in zip(ids, REQS):
        r = wait(sv, rid)
        assert r["state"] == "done", r
        mixed.append((sv.fetch(rid, req[0]), r))
    for k, (((pa, va), ra), ((pm, vm), rm)) in enumerate(zip(alone, mixed)):
        assert torch.equal(pa, pm), k
        assert torch.equal(va, vm), k
        assert ra["K"] == rm["K"] and ra["W"] == rm["W"], k
        assert ra["steps_done"] == REQS[k][1]
    sv.close()
    # the same request through bh_sim from the same device initial conditions
    for k in (0, 1, 3):
        n, steps, kind, seed, theta, prec = REQS[k]
        pos, vel, mass = bh.ic_generate(ctx, kind, n, seed)
        sim = bh.Sim(ctx, pos, vel, mass, bh.params(theta, 0.01, precision=prec))
        sim.step(steps, 1e-3)
        K, W = sim.energy()
        ctx.sync()
        (pa, va), ra = alone[k]
        assert torch.equal(pos, pa) and torch.equal(vel, va), k
        assert abs(K - ra["K"]) <= 1e-14 * abs(K) and abs(W - ra["W"]) <= 1e-12 * abs(W), k


def test_admission_limits_queue_and_reject(ctx):
    # a small arena: the tree workspace for 40k resident particles plus room for ~2 requests of 10k
    sv = bh.Server(ctx, 64 << 20, max_slots=2, max_resident=40000)
    with pytest.raises(bh.BHError) as e:
        sv.submit(50000, 1, 0, 1, bh.params(), 1e-3)     # above the particle cap: never fits
    assert e.value.status == bh.E_NOMEM
    ids = [sv.submit(10000, 3, 0, 200 + k, bh.params(precision="fp32"), 1e-3, release=True) for k in range(6)]
    res = [wait(sv, rid) for rid in ids]
    assert all(r["state"] == "done" for r in res)
    admits = sorted(r["t_admit"] for r in res)
    # at most two resident at a time: the third admission waits for a completion
    dones = sorted(r["t_done"] for r in res)
    assert admits[2] >= dones[0] - 1e-6
    with pytest.raises(bh.BHError):
        sv.fetch(ids[0], 10000)                             # released at completion
    sv.close()


def test_cancel(ctx):
    sv = bh.Server(ctx, 512 << 20, max_slots=1, max_resident=1 << 18)
    a = sv.submit(100000, 50, 0, 1, bh.params(precision="fp32"), 1e-3)
    b = sv.submit(1000, 2, 0, 2, bh.params(), 1e-3)
    sv.cancel(b)          # still queued behind a
    sv.cancel(a)          # running
    ra, rb = wait(sv, a), wait(sv, b)
    assert rb["state"] == "cancelled"
    assert ra["state"] in ("cancelled", "done")
    c = sv.submit(1000, 2, 0, 3, bh.params(), 1e-3)
    assert wait(sv, c)["state"] == "done"
    sv.close()


VARIANT_REQS = [  # (n, steps, kind, seed, theta, precision, option)
    (4000, 3, 0, 201, 0.6, "fp32", dict(quad=True)),
    (6000, 2, 1, 202, 0.8, "fp64", dict(open="bmax")),
    (3000, 4, 0, 203, 0.7, "fp32", dict(open="offset")),
    (5000, 2, 0, 204, 0.5, "fp64", dict(group=True)),
    (2500, 3, 1, 205, 0.6, "fp64", dict(quad=True, open="offset")),
]


def test_options_alone_equal_mix_and_plain_simulation(ctx):
    """Requests with the quadrupole, the alternative radii and the group criterion, mixed with
    each other in one forest iteration, give the bits they give alone and under bh_sim."""
    def sub(sv, req):
        n, steps, kind, seed, theta, prec, opt = req
        return sv.submit(n, steps, kind, seed, bh.params(theta, 0.01, precision=prec, **opt), 1e-3)

    sv = bh.Server(ctx, 2 * GiB, max_slots=16, max_resident=1 << 20)
    alone = []
    for req in VARIANT_REQS:
        rid = sub(sv, req)
        assert wait(sv, rid)["state"] == "done"
        alone.append(sv.fetch(rid, req[0]))
    ids = [sub(sv, req) for req in VARIANT_REQS]
    for k, (rid, req) in enumerate(zip(ids, VARIANT_REQS)):
        assert wait(sv, rid)["state"] == "done"
        pm, vm = sv.fetch(rid, req[0])
        assert torch.equal(alone[k][0], pm) and torch.equal(alone[k][1], vm), k
    sv.close()
    for k, (n, steps, kind, seed, theta, prec, opt) in enumerate(VARIANT_REQS):
        pos, vel, mass = bh.ic_generate(ctx, kind, n, seed)
        sim = bh.Sim(ctx, pos, vel, mass, bh.params(theta, 0.01, precision=prec, **opt))
        sim.step(steps, 1e-3)
        ctx.sync()
        assert torch.equal(pos, alone[k][0]) and torch.equal(vel, alone[k][1]), k


def test_fetch_while_another_request_runs(ctx):
    """A finished request is fetched while a long one is still resident: the copy does not wait
    for the long request, and the fetched state equals the same request served alone."""
    sv = bh.Server(ctx, 2 * GiB, max_slots=8, max_resident=1 << 20)
    req = (3000, 3, 0, 301, 0.5, "fp32")
    rid = submit(sv, req)
    assert wait(sv, rid)["state"] == "done"
    ref_pos, ref_vel = sv.fetch(rid, req[0])
    long_id = sv.submit(200000, 400, 1, 302, bh.params(0.5, 0.01, precision="fp64"), 1e-4)
    rid2 = submit(sv, req)
    assert wait(sv, rid2)["state"] == "done"
    pos, vel = sv.fetch(rid2, req[0])
    assert sv.poll(long_id)["state"] == "running"
    assert torch.equal(pos, ref_pos) and torch.equal(vel, ref_vel)
    with pytest.raises(bh.BHError):
        sv.fetch(rid2, req[0])   # released by the first fetch
    sv.cancel(long_id)
    assert wait(sv, long_id, timeout=120.0)["state"] == "cancelled"
    del sv

