"""GPU: walk launch shapes.  The grid form (1, 2, 4 or 8 wavefronts per workgroup) and the
persistent form (resident workgroups taking 64-body groups from a counter) give the same
bits for every walk variant of both precisions, with and without the potential, in a
forest, a tree (whole range and sub-ranges), a simulation and a replayed step graph; the
autotuner's timings, its cache and the BH_TUNE_CACHE file."""
import json
import os

import pytest

import icgen
from tests.gpu_helpers import dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
bh = pytest.importorskip("paper_1109_5190_amd")

SHAPES = bh.TUNE_SHAPES


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bh.Context(0)
    yield c
    c.sync()


def _all_variants():
    """One simulation per walk variant (each a counter slot of the persistent form)."""
    spec = [  # n, precision, quad, group, eps
        (3000, "fp32", False, False, 0.01), (700, "fp32", True, False, 0.01), (5000, "fp32", False, False, 0.0),
        (64, "fp32", True, False, 0.0), (2100, "fp32", False, True, 0.01), (900, "fp32", False, True, 0.0),
        (1500, "fp64", False, False, 0.01), (4100, "fp64", True, False, 0.01), (333, "fp64", False, True, 0.01),
        (1, "fp64", False, False, 0.0), (2500, "fp64", False, False, 0.0),
    ]
    ns = [s[0] for s in spec]
    plist = [bh.params(0.6, eps, precision=pr, quad=q, group=g) for _, pr, q, g, eps in spec]
    systems = [icgen.plummer(n, 100 + i) for i, n in enumerate(ns)]
    return ns, plist, icgen.concat(*systems)


def test_forest_every_variant_every_shape(ctx):
    print("[shapes] forest of every walk variant", flush=True)
    ns, plist, cat = _all_variants()
    fo = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    pot = torch.empty(sum(ns), dtype=torch.float64, device="cuda")
    fo.set_walk_shape(4)
    ref_a = fo.forces(pot).clone()
    ref_p = pot.clone()
    ctx.sync()
    assert torch.isfinite(ref_a).all()
    for sh in SHAPES:
        print(f"[shapes] forest shape {bh.shape_name(sh)}", flush=True)
        fo.set_walk_shape(sh)
        pot.fill_(float("nan"))
        a = fo.forces(pot)
        ctx.sync()
        assert torch.equal(a, ref_a), bh.shape_name(sh)
        assert torch.equal(pot, ref_p), bh.shape_name(sh)
        a = fo.forces()          # without the potential
        ctx.sync()
        assert torch.equal(a, ref_a), bh.shape_name(sh)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tree_shapes_whole_and_ranges(ctx, prec):
    print(f"[shapes] tree {prec}", flush=True)
    s = icgen.plummer(70001, 7)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.005, precision=prec)).upward()
    ref, ref_pot = t.forces(pot=True)
    for sh in (1 | bh.WALK_PERSISTENT, 4 | bh.WALK_PERSISTENT, 8 | bh.WALK_PERSISTENT, 2):
        t.set_walk_shape(sh)
        a, p = t.forces(pot=True)
        whole = t.forces_range(0, s.n)
        part = t.forces_range(0, 1000)
        part = t.forces_range(1000, s.n - 1000, acc=part)
        ctx.sync()
        assert torch.equal(a, ref) and torch.equal(p, ref_pot), bh.shape_name(sh)
        assert torch.equal(whole, ref) and torch.equal(part, ref), bh.shape_name(sh)


def test_invalid_shapes_are_refused(ctx):
    s = icgen.plummer(500, 8)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01)).upward()
    for sh in (0, 3, 16, 0x200, 0x100, -4):
        with pytest.raises(bh.BHError) as ei:
            t.set_walk_shape(sh)
        assert ei.value.status == bh.E_INVAL


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_persistent_sim_and_step_graph(ctx, prec):
    """A simulation and a replayed step graph in the persistent form equal eager grid-form steps."""
    print(f"[shapes] persistent steps and graph {prec}", flush=True)
    ns = [3000, 700, 12000, 64]
    plist = [bh.params(0.5, 0.01, precision=prec)] * 4
    systems = [icgen.plummer(n, 40 + i) for i, n in enumerate(ns)]
    cat = icgen.concat(*systems)
    a = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    b = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    a.set_walk_shape(4 | bh.WALK_PERSISTENT)
    for k in range(3):
        a.step_graph(2, 1e-3)
        b.step(2, 1e-3)
        scratch = torch.randn(1 << 16, device="cuda").sum()   # eager work between the replays
        ctx.sync()
        assert torch.isfinite(scratch)
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel) and torch.equal(a.acc, b.acc), k
    s = systems[2]
    p1, v1, m1 = dev(s.pos), dev(s.vel), dev(s.mass)
    p2, v2 = p1.clone(), v1.clone()
    s1 = bh.Sim(ctx, p1, v1, m1, plist[0])
    s2 = bh.Sim(ctx, p2, v2, m1, plist[0])
    s1.set_walk_shape(1 | bh.WALK_PERSISTENT)
    s1.step(3, 1e-3)
    s2.step(3, 1e-3)
    ctx.sync()
    assert torch.equal(p1, p2) and torch.equal(v1, v2) and torch.equal(s1.acc, s2.acc)


def test_autotune_timings_cache_and_file(ctx, tmp_path):
    print("[shapes] autotune", flush=True)
    bh.tune_cache_clear()
    ns = [3000, 700, 12000, 64]
    plist = [bh.params(0.5, 0.01, precision=pr) for pr in ("fp32", "fp64", "fp32", "fp64")]
    systems = [icgen.plummer(n, 41 + i) for i, n in enumerate(ns)]
    cat = icgen.concat(*systems)
    fo = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    ref = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    a0 = fo.forces().clone()
    path = tmp_path / "tune.json"
    os.environ["BH_TUNE_CACHE"] = str(path)
    try:
        shape, ms = fo.autotune()
    finally:
        del os.environ["BH_TUNE_CACHE"]
    assert shape in SHAPES and sorted(ms) == sorted(SHAPES) and all(v > 0 for v in ms.values())
    assert ms[shape] == min(ms.values())
    assert torch.equal(fo.acc, a0)            # refreshed by the chosen shape's walk
    assert torch.equal(fo.forces(), a0)
    assert bh.tune_cache_size() == 1
    doc = json.loads(path.read_text())        # written back by the timed call
    (e,) = doc["entries"]
    assert e["shape"] == shape and e["n_log2"] == 13 and e["sims_log2"] == 2 and e["precision"] == "mixed"
    assert e["theta"] == 0.5 and e["device"].startswith("gfx")
    # a forest with the same key takes the cached shape without timing
    other = bh.Forest(ctx, ns, plist, dev(cat.pos), dev(cat.vel), dev(cat.mass))
    s2, ms2 = other.autotune(cached=True)
    assert s2 == shape and all(v == -1.0 for v in ms2.values())
    assert torch.equal(other.acc, a0)
    fo.step_graph(2, 1e-3)
    ref.step(2, 1e-3)
    ctx.sync()
    assert torch.equal(fo.pos, ref.pos) and torch.equal(fo.acc, ref.acc)
    # the file loads back into an emptied cache
    bh.tune_cache_clear()
    bh.tune_cache_load(path)
    assert bh.tune_cache_size() == 1
    bh.tune_cache_clear()
