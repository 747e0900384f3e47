"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point include/bh.h declares, the Python binding covers exactly those names,
host-only calls (sizes, validation, errors) behave without a GPU."""
import ctypes as C
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "bh.h"


def declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def bh():
    import paper_1109_5190_amd as m
    if not m.LIB_PATH.exists():
        from paper_1109_5190_amd import build
        build.build()
    return m


def test_library_exports_every_declared_symbol(bh):
    out = subprocess.run(["nm", "-D", "--defined-only", str(bh.LIB_PATH)], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (bh_[a-z_0-9]+)$", out, flags=re.M))
    missing = [s for s in declared() if s not in exported]
    assert not missing, missing


def test_binding_names_match_header(bh):
    assert sorted(bh.exported_symbols()) == declared()
    bh.lib()   # binds every signature; raises if a symbol is absent


def test_version_and_error_strings(bh):
    L = bh.lib()
    assert L.bh_version().decode().startswith("bh-mi355x")
    assert isinstance(L.bh_last_error(), bytes)


def test_workspace_planning_without_gpu(bh):
    L = bh.lib()
    p64 = bh.params(precision="fp64")
    p32 = bh.params(precision="fp32")
    sizes = [L.bh_workspace_bytes(n, C.byref(p64)) for n in (1, 4096, 1 << 20)]
    assert all(s > 0 for s in sizes) and sizes[0] < sizes[1] < sizes[2]
    # roughly linear in n, a few hundred bytes per particle
    assert 150 < sizes[2] / (1 << 20) < 600
    assert L.bh_workspace_bytes(1 << 20, C.byref(p32)) > 0
    assert L.bh_sim_workspace_bytes(4096, C.byref(p32)) == L.bh_workspace_bytes(4096, C.byref(p32))
    ns = (C.c_int64 * 3)(1000, 1, 70000)
    ps = (bh.Params * 3)(p32, p64, p32)
    assert L.bh_forest_workspace_bytes(3, ns, ps) >= L.bh_workspace_bytes(71001, C.byref(p32))


@pytest.mark.parametrize("kw", [dict(theta=-0.1), dict(eps=-1.0), dict(leaf_cap=0), dict(leaf_cap=65),
                                dict(theta=float("nan")), dict(G=float("inf"))])
def test_invalid_parameters_rejected(bh, kw):
    L = bh.lib()
    args = dict(theta=0.5, eps=0.01, G=1.0, leaf_cap=1)
    args.update(kw)
    p = bh.params(**args)
    assert L.bh_workspace_bytes(1000, C.byref(p)) == 0
    assert L.bh_workspace_bytes(0, C.byref(bh.params())) == 0


def test_null_arguments_are_errors_not_crashes(bh):
    L = bh.lib()
    assert L.bh_build(None, 10, None, None, None, None, 0, None) == bh.E_INVAL
    assert L.bh_upward(None, None) == bh.E_INVAL
    assert L.bh_forces(None, None, None, None) == bh.E_INVAL
    assert L.bh_step(None, None, 1, 1e-3) == bh.E_INVAL
    assert L.bh_server_submit(None, None, None) == bh.E_INVAL
    assert L.bh_ctx_sync(None) == bh.E_INVAL
    assert L.bh_tree_free(None, None) == bh.OK


def test_context_without_device_reports_error(bh):
    L = bh.lib()
    h = C.c_void_p()
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    st = L.bh_ctx_create(0, None, C.byref(h))
    assert st in (bh.E_DEVICE, bh.E_INVAL)
    assert L.bh_last_error()


@pytest.mark.parametrize("flags", [2 | 4, 8 | 16, 8 | 4, 16 | 4, 1 << 7, 1 << 31])
def test_flag_combinations_rejected_on_the_host(bh, flags):
    """Options that exclude each other (quadrupole and group criterion; the two opening radii;
    a radius other than the side with the group criterion) and unknown bits are refused by the
    host-side parameter check, without a device."""
    p = bh.params(0.5, 0.01)
    p.flags = flags
    assert bh.lib().bh_workspace_bytes(1000, C.byref(p)) == 0


@pytest.mark.parametrize("flags", [0, 2, 4, 8, 16, 2 | 8, 2 | 16, 1])
def test_flag_combinations_accepted_on_the_host(bh, flags):
    p = bh.params(0.5, 0.01)
    p.flags = flags
    assert bh.lib().bh_workspace_bytes(1000, C.byref(p)) > 0
