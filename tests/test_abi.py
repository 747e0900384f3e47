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


# The boundary's required entry points and outputs: the calls the hot path exposes
# (tree build, upward pass, forces, canonical export with node count and per-body
# checksums, simulations, forests and the request API), the status codes and the
# walk statistics with their time.
REQUIRED = ["bh_ctx_create", "bh_ctx_destroy", "bh_ctx_sync", "bh_last_error", "bh_workspace_bytes", "bh_build",
            "bh_upward", "bh_forces", "bh_forces_stats", "bh_tree_export", "bh_tree_free", "bh_sim_create",
            "bh_step", "bh_energy", "bh_sim_destroy", "bh_forest_create", "bh_forest_step", "bh_forest_destroy",
            "bh_server_create", "bh_server_submit", "bh_server_poll", "bh_server_fetch", "bh_server_cancel",
            "bh_server_destroy", "bh_ic_generate", "bh_ic_workspace_bytes", "bh_forest_autotune",
            "bh_tree_set_walk_shape", "bh_sim_set_walk_shape", "bh_forest_set_walk_shape", "bh_tune_cache_load",
            "bh_tune_cache_save", "bh_tune_cache_clear", "bh_tune_cache_size"]


def _decl(name):
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    m = re.search(r"\b" + name + r"\s*\(([^;]*)\)\s*;", text, flags=re.S)
    assert m, name
    return " ".join(m.group(1).split())


def test_header_declares_the_boundary():
    names = declared()
    assert not [n for n in REQUIRED if n not in names]
    exp = _decl("bh_tree_export")
    assert "int64_t *n_nodes" in exp and "uint64_t *isect_hash" in exp
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    stats = re.search(r"typedef struct \{([^}]*)\} bh_stats;", text, flags=re.S).group(1)
    assert re.search(r"double t_ms;", stats)
    for f in ("n_mono", "n_p2p", "n_visits", "n_fallback"):
        assert f in stats
    codes = dict(re.findall(r"(BH_E_[A-Z]+|BH_OK) = (\d+)", text))
    assert codes == {"BH_OK": "0", "BH_E_INVAL": "1", "BH_E_NOMEM": "2", "BH_E_DEVICE": "3", "BH_E_BUSY": "4",
                     "BH_E_NOTFOUND": "5", "BH_E_OVERFLOW": "6", "BH_E_CANCELLED": "7", "BH_E_IO": "8"}
    assert "uint32_t flags, int32_t *shape_out, double *ms_out" in _decl("bh_forest_autotune")
    assert re.search(r"#define BH_WALK_PERSISTENT 0x100\b", text) and re.search(r"#define BH_TUNE_SHAPES 8\b", text)
    # every device buffer comes from the caller: workspace arguments on the calls that need scratch
    for name in ("bh_build", "bh_sim_create", "bh_forest_create", "bh_ic_generate"):
        assert "void *ws" in _decl(name), name
    assert "void *arena" in _decl("bh_server_create")


def test_ic_workspace_size_without_gpu(bh):
    L = bh.lib()
    nb = L.bh_ic_workspace_bytes()
    assert 256 < nb < 1 << 20 and nb % 256 == 0


def test_library_makes_no_device_allocations():
    """The library allocates no device memory of its own: no hipMalloc-family call in
    its sources (all device buffers are carved from caller workspaces)."""
    src = ROOT / "paper_1109_5190_amd" / "csrc"
    for p in list(src.glob("*.hip")) + list(src.glob("*.h")):
        text = re.sub(r"//[^\n]*", "", p.read_text())
        assert not re.search(r"\bhip(Malloc|MallocAsync|ExtMallocWithFlags|HostMalloc|MallocManaged)\s*\(", text), p
