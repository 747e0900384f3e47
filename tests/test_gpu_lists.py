"""Two-phase force stage (bh_lists_build, bh_lists_forces), both precisions: the evaluated
lists give the single-pass walk's forces bit for bit, and the lists themselves, decoded per body, are the
oracle's interaction sets (counts and checksums); buffer sizing and refusals."""
import ctypes as C

import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_helpers import dev, mix64

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


def make(kind, n, seed):
    if kind == "plummer":
        return icgen.plummer(n, seed)
    if kind == "cube":
        return icgen.uniform_cube(n, seed)
    if kind == "duplicates":
        s = icgen.plummer(n, seed)
        pos = np.round(s.pos * 4.0) / 4.0
        pos[: n // 4] = pos[0]
        return icgen.System(pos, s.vel, s.mass)
    if kind == "coincident":
        return icgen.System(np.tile([[0.25, -1.5, 3.0]], (n, 1)), np.zeros((n, 3)), np.full(n, 1.0 / n))
    return icgen.two_plummer(n // 2, seed, seed + 1)


CASES = [
    ("plummer", 4096, 1, 0.5, 0.01, 1, "side"),
    ("plummer", 20000, 4, 1.0, 0.0, 1, "side"),     # unsoftened pairs
    ("duplicates", 5000, 7, 0.6, 0.01, 2, "side"),
    ("coincident", 1250, 0, 0.5, 0.01, 1, "side"),  # one leaf of 1250 particles at the depth limit
    ("cube", 10001, 5, 0.7, 0.005, 4, "bmax"),
    ("two_spheres", 20000, 3, 0.5, 0.005, 1, "offset"),
]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("kind,n,seed,theta,eps,cap,open_", CASES)
def test_lists_give_the_walks_bits(ctx, kind, n, seed, theta, eps, cap, open_, prec):
    print(f"[lists] {kind} n={n} theta={theta} eps={eps} leaf_cap={cap} {open_} {prec}", flush=True)
    s = make(kind, n, seed)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass),
                bh.params(theta, eps, leaf_cap=cap, precision=prec, open=open_)).upward()
    a, p = t.forces(pot=True)
    t.lists_build()
    b, q = t.lists_forces(pot=True)
    assert torch.equal(a, b) and torch.equal(p, q)
    assert torch.equal(t.lists_forces(), a)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("kind,n,seed,theta,eps", [("plummer", 6000, 9, 0.7, 0.01), ("plummer", 20000, 4, 1.0, 0.0),
                                                   ("cube", 8000, 5, 0.6, 0.005)])
def test_lists_with_quadrupole(ctx, kind, n, seed, theta, eps, prec):
    """Quadrupole trees: the replay adds the walk's quadrupole term (and, in FP32, its FP64 lanes
    for bodies close to a cube) in the same order, so the bits are the walk's."""
    s = make(kind, n, seed)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(theta, eps, precision=prec, quad=True)).upward()
    a, p = t.forces(pot=True)
    t.lists_build()
    b, q = t.lists_forces(pot=True)
    assert torch.equal(a, b) and torch.equal(p, q)


def up256(v):
    return (v + 255) & ~255


def layout(G, Cn):
    head = 256 * 256
    count = up256(head + 4 * G)
    nxt = up256(count + 4 * G)
    ent = up256(nxt + 4 * Cn)
    return head, count, nxt, ent, ent + 16 * 64 * Cn


def chunks_for(G, nbytes):
    fixed = layout(G, 0)[4]
    if nbytes <= fixed + 256:
        return 0
    c = (nbytes - fixed - 256) // (4 + 16 * 64)
    while c > 0 and layout(G, c)[4] > nbytes:
        c -= 1
    return c


def decode(buf, n):
    """Per body (original index): accepted node ids and pair partners (original indices)."""
    raw = buf.cpu().numpy()
    G = (n + 63) // 64
    Cn = chunks_for(G, raw.size)
    ho, co, no, eo, _ = layout(G, Cn)
    head = np.frombuffer(raw, np.uint32, G, ho)
    count = np.frombuffer(raw, np.uint32, G, co)
    nxt = np.frombuffer(raw, np.uint32, Cn, no)
    ent = np.frombuffer(raw, np.uint32, 64 * Cn * 4, eo).reshape(-1, 4)
    out = []
    for g in range(G):
        rows, ch, k = [], int(head[g]), 0
        while k < count[g]:
            m = min(64, int(count[g]) - k)
            rows.append(ent[64 * ch: 64 * ch + m])
            k += m
            ch = int(nxt[ch])
        out.append(np.concatenate(rows))
    return out


@pytest.mark.parametrize("kind,n,seed,theta,cap,prec", [("plummer", 4096, 2, 0.6, 4, "fp32"),
                                                        ("duplicates", 3000, 8, 0.8, 1, "fp32"),
                                                        ("plummer", 4096, 2, 0.6, 4, "fp64")])
def test_lists_are_the_oracle_sets(ctx, kind, n, seed, theta, cap, prec):
    s = make(kind, n, seed)
    ref = oracle.Tree(s.pos, s.mass, cap).walk(theta, 0.01)
    t = bh.Tree(ctx, dev(s.pos), dev(s.mass), bh.params(theta, 0.01, leaf_cap=cap, precision=prec)).upward()
    ex = t.export(with_mass=False)
    perm = ex["perm"].cpu().numpy().astype(np.int64)
    nn = ex["n_nodes"]
    lists = decode(t.lists_build(), n)
    n_mono = np.zeros(n, np.int64)
    n_p2p = np.zeros(n, np.int64)
    h = np.zeros(n, np.uint64)
    with np.errstate(over="ignore"):
        for g, e in enumerate(lists):
            a, b = e[:, 0].astype(np.int64), e[:, 1].astype(np.int64)
            mask = e[:, 2].astype(np.uint64) | (e[:, 3].astype(np.uint64) << np.uint64(32))
            start = a != 0xFFFFFFFF
            leaf = start & (b >= 0x80000000)
            mono = start & (b < 0x80000000)
            for k in range(min(64, n - 64 * g)):
                rank = 64 * g + k
                i = perm[rank]
                bit = ((mask >> np.uint64(k)) & np.uint64(1)).astype(bool)
                mk = mono & bit
                n_mono[i] = mk.sum()
                h[i] += mix64(b[mk]).sum(dtype=np.uint64)
                for a0, cnt in zip(a[leaf & bit], b[leaf & bit] & 0x7FFFFFFF):
                    ranks = np.arange(a0, a0 + cnt)
                    ranks = ranks[ranks != rank]
                    n_p2p[i] += ranks.size
                    h[i] += mix64(nn + perm[ranks]).sum(dtype=np.uint64)
    assert np.array_equal(n_mono, ref["n_mono"])
    assert np.array_equal(n_p2p, ref["n_p2p"])
    assert np.array_equal(h, ref["hash"])


def test_buffer_sizing_and_validity(ctx):
    s = icgen.plummer(5000, 3)
    pos, mass = dev(s.pos), dev(s.mass)
    t = bh.Tree(ctx, pos, mass, bh.params(0.5, 0.01, precision="fp32")).upward()
    with pytest.raises(bh.BHError):
        t.lists_forces()                       # nothing built yet
    raw, small = bh.workspace(256 * 1024, pos.device)   # the tables fit, the lists do not
    need = C.c_size_t(0)
    st = bh.lib().bh_lists_build(ctx.h, t.h, C.c_void_p(small.data_ptr()), small.numel(), C.byref(need))
    assert st == bh.E_NOMEM and need.value > small.numel()
    raw2, fit = bh.workspace(need.value, pos.device)
    need2 = C.c_size_t(0)
    st = bh.lib().bh_lists_build(ctx.h, t.h, C.c_void_p(fit.data_ptr()), fit.numel(), C.byref(need2))
    assert st == bh.OK and need2.value == need.value
    t._lists = (raw2, fit)
    assert torch.equal(t.lists_forces(), t.forces())
    t.rebuild(pos, mass).upward()              # lists belong to the tree they were built on
    with pytest.raises(bh.BHError):
        t.lists_forces()


def test_unsupported_trees_refused(ctx):
    s = icgen.plummer(2000, 4)
    for p in (bh.params(0.5, 0.01, precision="fp32", group=True), bh.params(0.5, 0.01, precision="fp64", group=True)):
        t = bh.Tree(ctx, dev(s.pos), dev(s.mass), p).upward()
        with pytest.raises(bh.BHError):
            t.lists_build()
