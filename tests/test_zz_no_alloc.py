"""GPU: bh_ic_generate_static, the entry point that allocates nothing, gives
bh_ic_generate's outputs bit for bit, on two calls in a row (the second with a
smaller n, so the static scratch holds the previous call's contents), for both
initial-condition kinds; its argument checks match."""
import pytest

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


def _bufs(n):
    pos = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
    return pos, torch.full_like(pos, float("nan")), torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")


def _static(ctx, kind, n, seed, a=1.0, M=1.0):
    pos, vel, mass = _bufs(n)
    st = bh.lib().bh_ic_generate_static(ctx.h, kind, n, seed, a, M, bh._ptr(pos), bh._ptr(vel), bh._ptr(mass))
    assert st == bh.OK, bh.lib().bh_last_error()
    return pos, vel, mass


@pytest.mark.parametrize("kind", [0, 1])
def test_static_equals_workspace_variant(ctx, kind):
    for n, seed in ((200001, 31), (4097, 32)):   # the second call is smaller
        print(f"[no-alloc] kind={kind} n={n} seed={seed}", flush=True)
        ref = bh.ic_generate(ctx, kind, n, seed, a=1.5, M=2.0)
        got = _static(ctx, kind, n, seed, a=1.5, M=2.0)
        ctx.sync()
        for r, g in zip(ref, got):
            assert torch.equal(r, g)
        assert torch.isfinite(got[0]).all() and torch.isfinite(got[1]).all()


def test_static_argument_checks(ctx):
    L = bh.lib()
    pos, vel, mass = _bufs(16)
    p = (bh._ptr(pos), bh._ptr(vel), bh._ptr(mass))
    assert L.bh_ic_generate_static(None, 0, 16, 1, 1.0, 1.0, *p) == bh.E_INVAL
    assert L.bh_ic_generate_static(ctx.h, 2, 16, 1, 1.0, 1.0, *p) == bh.E_INVAL
    assert L.bh_ic_generate_static(ctx.h, 0, 0, 1, 1.0, 1.0, *p) == bh.E_INVAL
    assert L.bh_ic_generate_static(ctx.h, 0, 1 << 30, 1, 1.0, 1.0, *p) == bh.E_INVAL
    assert b"n out of range" in L.bh_last_error()
    assert L.bh_ic_generate_static(ctx.h, 0, 16, 1, -1.0, 1.0, *p) == bh.E_INVAL
    assert L.bh_ic_generate_static(ctx.h, 0, 16, 1, 1.0, 1.0, None, p[1], p[2]) == bh.E_INVAL
    ctx.sync()
