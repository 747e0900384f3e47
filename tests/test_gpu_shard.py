"""One GPU's target share (bh_forces_range) and the cost-balanced split of the targets
(bh_shard_bounds).  A range walk writes the full walk's bits on the rows of its bodies and
leaves every other row as it was, for each kind of tree; the per-body work output is each
group's wavefront work spread evenly and sums to the walk's wavefront totals; the ranges of a
split together give the full walk; the split equals the cost-zone definition (smallest rank r
with G P(r) >= j T) evaluated with numpy from the same costs, over ragged sizes and more than
1024 chunks."""
import numpy as np
import pytest

import icgen
from tests.costzones import cost_zones, group_zones
from tests.gpu_helpers import dev

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


VARIANTS = {
    "fp32": dict(precision="fp32"),
    "fp64": dict(precision="fp64"),
    "fp32-quad": dict(precision="fp32", quad=True),
    "fp64-quad": dict(precision="fp64", quad=True),
    "fp32-group": dict(precision="fp32", group=True),
    "fp64-group": dict(precision="fp64", group=True),
    "fp32-bmax": dict(precision="fp32", open="bmax"),
    "fp64-offset": dict(precision="fp64", open="offset"),
}
RANGES = [(0, None), (0, 1), (5, 100), (64, 64), (130, 1000), (None, 37), (1000, 0), (63, 2)]


def nan_like(n, cols=None):
    shape = (n,) if cols is None else (n, cols)
    return torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")


# every tree variant softened, and the unsoftened walks of both precisions
CASES = [(v, 0.01) for v in VARIANTS] + [("fp32", 0.0), ("fp64", 0.0)]


@pytest.mark.parametrize("var,eps", CASES)
def test_range_rows_are_the_full_walks(ctx, var, eps):
    n = 5000
    print(f"[range] {var} eps={eps} n={n}", flush=True)
    s = icgen.plummer(n, 11)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.6, eps, **VARIANTS[var])).upward()
    full, pfull = t.forces(pot=True)
    st = t.forces_stats()
    ng = (n + 63) // 64
    wfull = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    gfull = torch.full((ng,), -1, dtype=torch.int64, device="cuda")
    t.forces_range(0, n, None, None, None, None, wfull, gfull)
    perm = t.export(with_mass=False)["perm"].long()
    for first, count in RANGES:
        first = n - 37 if first is None else first
        count = n - first if count is None else count
        rows = perm[first:first + count]
        other = torch.ones(n, dtype=torch.bool, device="cuda")
        other[rows] = False
        acc, pot = nan_like(n, 3), nan_like(n)
        t.forces_range(first, count, acc, pot)
        assert torch.equal(acc[rows], full[rows]) and torch.equal(pot[rows], pfull[rows]), (first, count)
        assert torch.isnan(acc[other]).all() and torch.isnan(pot[other]).all(), (first, count)
        # the counting walk over the same range
        acc2 = nan_like(n, 3)
        nm, np_, wk = (torch.full((n,), -1, dtype=torch.int64, device="cuda") for _ in range(3))
        gw = torch.full((ng,), -1, dtype=torch.int64, device="cuda")
        t.forces_range(first, count, acc2, None, nm, np_, wk, gw)
        g0, g1 = first // 64, (first + count + 63) // 64 if count else first // 64   # groups the range meets
        assert torch.equal(gw[g0:g1], gfull[g0:g1]) and (gw[:g0] == -1).all() and (gw[g1:] == -1).all()
        assert torch.equal(acc2[rows], st["acc"][rows])
        assert torch.equal(nm[rows], st["n_mono"][rows]) and torch.equal(np_[rows], st["n_p2p"][rows])
        assert torch.equal(wk[rows], wfull[rows])
        assert (nm[other] == -1).all() and (np_[other] == -1).all() and (wk[other] == -1).all()
        assert torch.isnan(acc2[other]).all()


@pytest.mark.parametrize("var", ["fp32", "fp64", "fp32-group", "fp64-group", "fp32-quad"])
def test_work_is_the_groups_wavefront_work(ctx, var):
    """Each 64-body group's work W (children tested plus pair iterations of its shared
    traversal) spread evenly over its bodies; with one particle per leaf every opened leaf is
    one pair iteration, so the FP32 walks' totals give sum W = wavefront visits + opened leaves."""
    n = 6000
    s = icgen.plummer(n, 17)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.6, 0.01, **VARIANTS[var])).upward()
    wk = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    gw = torch.full(((n + 63) // 64,), -1, dtype=torch.int64, device="cuda")
    t.forces_range(0, n, None, None, None, None, wk, gw)
    perm = t.export(with_mass=False)["perm"].long()
    ws = wk[perm].cpu().numpy()
    assert ws.min() >= 0
    W = []
    for g in range(0, n, 64):
        v = ws[g:g + 64]
        c, Wg = len(v), int(v.sum())
        k = np.arange(c)
        assert np.array_equal(v, (Wg * (k + 1)) // c - (Wg * k) // c), g
        W.append(Wg)
    assert min(W) > 0
    assert np.array_equal(gw.cpu().numpy(), np.array(W))
    if var.startswith("fp32"):
        tot = t.forces_stats()["totals"]
        assert sum(W) == tot["wave_visits"] + tot["wave_leaves"]


@pytest.mark.parametrize("G", [1, 2, 3, 8, 64, 1000])
def test_bounds_are_the_cost_zones(ctx, G):
    n = 20000   # 20 chunks of 1024 and a ragged tail
    s = icgen.plummer(n, 12)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01, precision="fp32")).upward()
    st = t.forces_stats()
    perm = t.export(with_mass=False)["perm"].long().cpu().numpy()
    nm, np_ = st["n_mono"], st["n_p2p"]
    cost = (1 + nm.cpu().numpy() + np_.cpu().numpy())[perm]
    b = t.shard_bounds(G, nm, np_).cpu().numpy()
    assert np.array_equal(b, cost_zones(cost, G))
    assert b[0] == 0 and b[-1] == n and np.all(np.diff(b) >= 0)
    P = np.concatenate([[0], np.cumsum(cost)])
    share = P[b[1:]] - P[b[:-1]]
    assert share.max() <= P[-1] / G + cost.max()
    # one count array, and none (equal counts: ceil(j n / G))
    c1 = (1 + nm.cpu().numpy())[perm]
    assert np.array_equal(t.shard_bounds(G, nm, None).cpu().numpy(), cost_zones(c1, G))
    wk = torch.empty(n, dtype=torch.int64, device="cuda")
    gw = torch.empty((n + 63) // 64, dtype=torch.int64, device="cuda")
    t.forces_range(0, n, None, None, None, None, wk, gw)
    cw = (1 + wk.cpu().numpy())[perm]
    assert np.array_equal(t.shard_bounds(G, wk).cpu().numpy(), cost_zones(cw, G))
    bg = t.shard_bounds_groups(G, gw).cpu().numpy()
    assert np.array_equal(bg, group_zones(gw.cpu().numpy(), n, G))
    assert np.all((bg[:-1] % 64 == 0) | (bg[:-1] == n)) and bg[-1] == n
    eq = np.array([-(-j * n // G) for j in range(G + 1)], dtype=np.int64)
    assert np.array_equal(t.shard_bounds(G).cpu().numpy(), eq)


def test_bounds_over_many_chunks(ctx):
    """1,100,001 bodies: 1075 chunks, so the chunk scan takes two rounds; arbitrary counts."""
    n = 1_100_001
    s = icgen.uniform_cube(n, 13)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01, precision="fp32")).upward()
    rng = np.random.default_rng(14)
    nm = rng.integers(0, 3000, n)
    np_ = rng.integers(0, 200, n)
    perm = t.export(with_mass=False)["perm"].long().cpu().numpy()
    cost = (1 + nm + np_)[perm]
    gc = rng.integers(0, 100000, (n + 63) // 64)
    for G in (2, 8, 4096):
        b = t.shard_bounds(G, torch.tensor(nm, dtype=torch.int64, device="cuda"),
                           torch.tensor(np_, dtype=torch.int64, device="cuda")).cpu().numpy()
        assert np.array_equal(b, cost_zones(cost, G)), G
        bg = t.shard_bounds_groups(G, torch.tensor(gc, dtype=torch.int64, device="cuda")).cpu().numpy()
        assert np.array_equal(bg, group_zones(gc, n, G)), G


def test_shards_cover_the_full_walk(ctx):
    n = 1 << 16
    s = icgen.plummer(n, 15)
    for prec in ("fp32", "fp64"):
        t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.005, precision=prec)).upward()
        st = t.forces_stats()
        wk = torch.empty(n, dtype=torch.int64, device="cuda")
        gw = torch.empty(n // 64, dtype=torch.int64, device="cuda")
        t.forces_range(0, n, None, None, None, None, wk, gw)
        for b in (t.shard_bounds(8, st["n_mono"], st["n_p2p"]), t.shard_bounds(8, wk), t.shard_bounds_groups(8, gw)):
            b = b.cpu().tolist()
            acc = nan_like(n, 3)
            for j in range(8):
                t.forces_range(b[j], b[j + 1] - b[j], acc)
            assert torch.equal(acc, st["acc"]), prec


def test_arguments_validated(ctx):
    s = icgen.plummer(300, 16)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(0.5, 0.01))
    with pytest.raises(bh.BHError):
        t.forces_range(0, 10)                   # before bh_upward
    with pytest.raises(bh.BHError):
        t.shard_bounds(4)
    t.upward()
    for first, count in ((-1, 5), (0, -1), (299, 2), (301, 0)):
        with pytest.raises(bh.BHError):
            t.forces_range(first, count)
    for G in (0, -3, 65537):
        with pytest.raises(bh.BHError):
            t.shard_bounds(G)
    gw = torch.zeros(5, dtype=torch.int64, device="cuda")
    for G in (0, 65537):
        with pytest.raises(bh.BHError):
            t.shard_bounds_groups(G, gw)
    with pytest.raises(bh.BHError):
        t.shard_bounds_groups(4, None)
    acc = t.forces_range(300, 0)                # empty range at the end: nothing written
    assert torch.isnan(acc).all()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130])
def test_tiny_trees(ctx, n):
    """Trees of one partial group up to a few groups; every single-body range, and splits with
    more ranges than bodies (empty ranges where a boundary repeats)."""
    print(f"[tiny] n={n}", flush=True)
    s = icgen.plummer(max(n, 2), 18)
    pos, mass = s.pos[:n], s.mass[:n]
    for prec in ("fp32", "fp64"):
        t = bh.Tree(ctx, dev(pos), dev(mass), bh.params(0.5, 0.01, precision=prec)).upward()
        st = t.forces_stats()
        perm = t.export(with_mass=False)["perm"].long()
        acc = nan_like(n, 3)
        for r in range(n):
            t.forces_range(r, 1, acc)
            assert torch.equal(acc[perm[r]], st["acc"][perm[r]]), (prec, r)
        assert torch.equal(acc, st["acc"])
        wk = torch.empty(n, dtype=torch.int64, device="cuda")
        gw = torch.empty((n + 63) // 64, dtype=torch.int64, device="cuda")
        t.forces_range(0, n, None, None, None, None, wk, gw)
        ps = perm.cpu().numpy()
        for G in (1, 3, 2 * n + 1):
            b = t.shard_bounds(G, wk).cpu().numpy()
            assert np.array_equal(b, cost_zones((1 + wk.cpu().numpy())[ps], G)), (prec, G)
            bg = t.shard_bounds_groups(G, gw).cpu().numpy()
            assert np.array_equal(bg, group_zones(gw.cpu().numpy(), n, G)), (prec, G)
            for bb in (b, bg):
                acc2 = nan_like(n, 3)
                for j in range(G):
                    t.forces_range(int(bb[j]), int(bb[j + 1] - bb[j]), acc2)
                assert torch.equal(acc2, st["acc"]), (prec, G)
