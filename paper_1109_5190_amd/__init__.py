"""Thin Python binding of libbh.so, the MI355X Barnes-Hut library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (workspaces, inputs, outputs)
and the HIP stream (the current torch stream).  The names follow the C ABI
in include/bh.h without the `bh_` prefix.

Loading fails loudly when libbh.so has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libbh.so"

OK, E_INVAL, E_NOMEM, E_DEVICE, E_BUSY, E_NOTFOUND, E_OVERFLOW, E_CANCELLED, E_IO = range(9)
FP64, FP32 = 0, 1


class BHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bh status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("eps", C.c_double), ("G", C.c_double), ("leaf_cap", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("reserved", C.c_uint32)]


QUADRUPOLE = 2
GROUP_CRITERION = 4
OPEN_BMAX = 8
OPEN_OFFSET = 16
OPEN = {"side": 0, "bmax": OPEN_BMAX, "offset": OPEN_OFFSET}

WALK_PERSISTENT = 0x100
TUNE_CACHED = 1
# the autotuner's shapes, in the order of its timings: wavefronts per workgroup, grid then persistent form
TUNE_SHAPES = (1, 2, 4, 8, 1 | WALK_PERSISTENT, 2 | WALK_PERSISTENT, 4 | WALK_PERSISTENT, 8 | WALK_PERSISTENT)


def shape_name(shape):
    """'4' for four wavefronts per workgroup, '4p' for the persistent form."""
    return f"{shape & 0xff}{'p' if shape & WALK_PERSISTENT else ''}"


def params(theta=0.5, eps=0.01, G=1.0, leaf_cap=1, precision="fp64", quad=False, group=False,
           open="side") -> Params:
    """open: opening radius of the test r^2 < theta^2 D^2: "side" (the cube side), "bmax"
    (BH_OPEN_BMAX) or "offset" (BH_OPEN_OFFSET)."""
    prec = {"fp64": FP64, "fp32": FP32, FP64: FP64, FP32: FP32}[precision]
    flags = (QUADRUPOLE if quad else 0) | (GROUP_CRITERION if group else 0) | OPEN[open]
    return Params(float(theta), float(eps), float(G), int(leaf_cap), prec, flags, 0)


class Stats(C.Structure):
    _fields_ = [("n_mono", C.c_uint64), ("n_p2p", C.c_uint64), ("n_visits", C.c_uint64),
                ("n_fallback", C.c_uint64), ("wave_visits", C.c_uint64), ("wave_entries", C.c_uint64),
                ("wave_accepts", C.c_uint64), ("wave_leaves", C.c_uint64), ("t_ms", C.c_double)]


class Request(C.Structure):
    _fields_ = [("n", C.c_int64), ("steps", C.c_int32), ("ic_kind", C.c_int32), ("seed", C.c_uint64),
                ("p", Params), ("dt", C.c_double)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("steps_done", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("K", C.c_double), ("W", C.c_double)]


_VP = C.c_void_p
_SIGS = {
    "bh_last_error": ([], C.c_char_p),
    "bh_version": ([], C.c_char_p),
    "bh_ctx_create": ([C.c_int, _VP, C.POINTER(_VP)], C.c_int),
    "bh_ctx_destroy": ([_VP], C.c_int),
    "bh_ctx_sync": ([_VP], C.c_int),
    "bh_workspace_bytes": ([C.c_int64, C.POINTER(Params)], C.c_size_t),
    "bh_build": ([_VP, C.c_int64, _VP, _VP, C.POINTER(Params), _VP, C.c_size_t, C.POINTER(_VP)], C.c_int),
    "bh_rebuild": ([_VP, _VP, _VP, _VP], C.c_int),
    "bh_upward": ([_VP, _VP], C.c_int),
    "bh_lists_build": ([_VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
    "bh_lists_forces": ([_VP, _VP, _VP, _VP, _VP], C.c_int),
    "bh_forces": ([_VP, _VP, _VP, _VP], C.c_int),
    "bh_forces_stats": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(Stats)], C.c_int),
    "bh_forces_range": ([_VP, _VP, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP], C.c_int),
    "bh_shard_bounds": ([_VP, _VP, _VP, _VP, C.c_int32, _VP], C.c_int),
    "bh_shard_bounds_groups": ([_VP, _VP, _VP, C.c_int32, _VP], C.c_int),
    "bh_tree_info": ([_VP, _VP, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int32)], C.c_int),
    "bh_tree_export": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_int64), _VP], C.c_int),
    "bh_tree_free": ([_VP, _VP], C.c_int),
    "bh_sim_workspace_bytes": ([C.c_int64, C.POINTER(Params)], C.c_size_t),
    "bh_sim_create": ([_VP, C.c_int64, _VP, _VP, _VP, _VP, C.POINTER(Params), _VP, C.c_size_t, C.POINTER(_VP)],
                      C.c_int),
    "bh_step": ([_VP, _VP, C.c_int32, C.c_double], C.c_int),
    "bh_energy": ([_VP, _VP, C.POINTER(C.c_double)], C.c_int),
    "bh_sim_destroy": ([_VP, _VP], C.c_int),
    "bh_forest_workspace_bytes": ([C.c_int32, C.POINTER(C.c_int64), C.POINTER(Params)], C.c_size_t),
    "bh_forest_create": ([_VP, C.c_int32, C.POINTER(C.c_int64), C.POINTER(Params), _VP, _VP, _VP, _VP, _VP,
                          C.c_size_t, C.POINTER(_VP)], C.c_int),
    "bh_forest_step": ([_VP, _VP, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "bh_forest_forces": ([_VP, _VP, _VP], C.c_int),
    "bh_forest_step_graph": ([_VP, _VP, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "bh_forest_autotune": ([_VP, _VP, C.c_uint32, C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
    "bh_tree_set_walk_shape": ([_VP, _VP, C.c_int32], C.c_int),
    "bh_sim_set_walk_shape": ([_VP, _VP, C.c_int32], C.c_int),
    "bh_forest_set_walk_shape": ([_VP, _VP, C.c_int32], C.c_int),
    "bh_tune_cache_load": ([C.c_char_p], C.c_int),
    "bh_tune_cache_save": ([C.c_char_p], C.c_int),
    "bh_tune_cache_clear": ([], C.c_int),
    "bh_tune_cache_size": ([], C.c_int64),
    "bh_forest_energy": ([_VP, _VP, C.POINTER(C.c_double)], C.c_int),
    "bh_forest_destroy": ([_VP, _VP], C.c_int),
    "bh_ic_workspace_bytes": ([], C.c_size_t),
    "bh_ic_generate_static": ([_VP, C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_double, _VP, _VP, _VP],
                              C.c_int),
    "bh_ic_generate": ([_VP, C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_double, _VP, _VP, _VP, _VP,
                        C.c_size_t], C.c_int),
    "bh_server_create": ([_VP, _VP, C.c_size_t, C.c_int32, C.c_int64, C.POINTER(_VP)], C.c_int),
    "bh_server_submit": ([_VP, C.POINTER(Request), C.POINTER(C.c_uint64)], C.c_int),
    "bh_server_poll": ([_VP, C.c_uint64, C.POINTER(Result)], C.c_int),
    "bh_server_fetch": ([_VP, C.c_uint64, _VP, _VP], C.c_int),
    "bh_server_cancel": ([_VP, C.c_uint64], C.c_int),
    "bh_server_now": ([_VP], C.c_double),
    "bh_server_destroy": ([_VP], C.c_int),
}

_lib = None


def lib():
    """The loaded libbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1109_5190_amd.build` "
                              "(there is no CPU fallback)")
        L = C.CDLL(str(LIB_PATH))
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _check(status):
    if status != OK:
        raise BHError(status, lib().bh_last_error().decode())


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else _VP(t.data_ptr())


def _need(t, n, cols, dtype_name="float64"):
    torch = _torch()
    dt = getattr(torch, dtype_name)
    if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} CUDA tensor")
    shape = (n, cols) if cols else (n,)
    if tuple(t.shape) != shape:
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")


def workspace(nbytes, device):
    """A 256-byte aligned device byte buffer of at least nbytes (torch-owned)."""
    torch = _torch()
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:]


class Context:
    """bh_ctx bound to a device and the current torch stream."""

    def __init__(self, device=0, stream=None):
        torch = _torch()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = _VP()
        _check(lib().bh_ctx_create(self.device.index or 0, _VP(s.cuda_stream), C.byref(h)))
        self.h = h

    def sync(self):
        _check(lib().bh_ctx_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().bh_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(n, p: Params) -> int:
    return int(lib().bh_workspace_bytes(int(n), C.byref(p)))


class Tree:
    """bh_build / bh_upward / bh_forces over device tensors pos (n,3) and mass (n,)."""

    def __init__(self, ctx: Context, pos, mass, p: Params):
        n = int(mass.shape[0])
        _need(pos, n, 3)
        _need(mass, n, 0)
        self.ctx, self.n, self.p = ctx, n, p
        self.pos, self.mass = pos, mass
        nb = workspace_bytes(n, p)
        if nb == 0:
            raise BHError(E_INVAL, "invalid parameters")
        self._raw, self.ws = workspace(nb, pos.device)
        h = _VP()
        _check(lib().bh_build(ctx.h, n, _ptr(pos), _ptr(mass), C.byref(p), _ptr(self.ws), nb, C.byref(h)))
        self.h = h

    def rebuild(self, pos, mass):
        """bh_rebuild: the same tree and workspace, new positions and masses of the n particles."""
        _need(pos, self.n, 3)
        _need(mass, self.n, 0)
        self.pos, self.mass = pos, mass
        _check(lib().bh_rebuild(self.ctx.h, self.h, _ptr(pos), _ptr(mass)))
        return self

    def upward(self):
        _check(lib().bh_upward(self.ctx.h, self.h))
        return self

    def lists_build(self, nbytes=None, reuse=False):
        """bh_lists_build into a torch-owned buffer (grown to the size the call reports if it is
        too small; reuse=True writes into the buffer of the last call).  Returns the buffer
        (uint8, 256-byte aligned view), kept for lists_forces."""
        nbytes = int(nbytes or 4096 * (self.n // 64 + 1) * 16 + (1 << 20))
        for attempt in range(2):
            if reuse and attempt == 0 and getattr(self, "_lists", None):
                raw, buf = self._lists
            else:
                raw, buf = workspace(nbytes, self.pos.device)
            need = C.c_size_t(0)
            st = lib().bh_lists_build(self.ctx.h, self.h, _ptr(buf), buf.numel(), C.byref(need))
            if st == OK:
                self._lists = (raw, buf)
                return buf
            if st != E_NOMEM:
                _check(st)
            nbytes = int(need.value) + 256
        _check(st)

    def lists_forces(self, acc=None, pot=False):
        """bh_lists_forces over the buffer of the last lists_build."""
        torch = _torch()
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float64, device=self.pos.device)
        ph = torch.empty(self.n, dtype=torch.float64, device=self.pos.device) if pot else None
        buf = self._lists[1] if getattr(self, "_lists", None) else None
        _check(lib().bh_lists_forces(self.ctx.h, self.h, _ptr(buf), _ptr(acc), _ptr(ph)))
        return (acc, ph) if pot else acc

    def forces(self, acc=None, pot=False):
        torch = _torch()
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float64, device=self.pos.device)
        ph = torch.empty(self.n, dtype=torch.float64, device=self.pos.device) if pot else None
        _check(lib().bh_forces(self.ctx.h, self.h, _ptr(acc), _ptr(ph)))
        return (acc, ph) if pot else acc

    def forces_stats(self, pot=False):
        torch = _torch()
        dev = self.pos.device
        acc = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        ph = torch.empty(self.n, dtype=torch.float64, device=dev) if pot else None
        nm = torch.empty(self.n, dtype=torch.int64, device=dev)
        np_ = torch.empty(self.n, dtype=torch.int64, device=dev)
        hs = torch.empty(self.n, dtype=torch.int64, device=dev)
        st = Stats()
        _check(lib().bh_forces_stats(self.ctx.h, self.h, _ptr(acc), _ptr(ph), _ptr(nm), _ptr(np_), _ptr(hs),
                                     C.byref(st)))
        totals = {k: int(getattr(st, k)) for k, _ in Stats._fields_ if k != "t_ms"}
        totals["t_ms"] = float(st.t_ms)
        return dict(acc=acc, pot=ph, n_mono=nm, n_p2p=np_, hash=hs, totals=totals)

    def forces_range(self, first, count, acc=None, pot=None, n_mono=None, n_p2p=None, work=None, group_work=None):
        """bh_forces_range: rows of the bodies of sorted ranks [first, first + count) in acc (and pot,
        n_mono, n_p2p, work when given; group_work per 64-body group); the other rows keep their
        contents.  Returns acc."""
        torch = _torch()
        if acc is None:
            acc = torch.full((self.n, 3), float("nan"), dtype=torch.float64, device=self.pos.device)
        _check(lib().bh_forces_range(self.ctx.h, self.h, int(first), int(count), _ptr(acc), _ptr(pot),
                                     _ptr(n_mono), _ptr(n_p2p), _ptr(work), _ptr(group_work)))
        return acc

    def shard_bounds(self, G, cost_a=None, cost_b=None):
        """bh_shard_bounds: G + 1 int64 range starts (device) for body costs 1 + cost_a + cost_b."""
        torch = _torch()
        b = torch.empty(max(int(G) + 1, 1), dtype=torch.int64, device=self.pos.device)   # G < 1: the call refuses it
        _check(lib().bh_shard_bounds(self.ctx.h, self.h, _ptr(cost_a), _ptr(cost_b), int(G), _ptr(b)))
        return b

    def shard_bounds_groups(self, G, group_work):
        """bh_shard_bounds_groups: G + 1 int64 range starts (device) on 64-body group boundaries."""
        torch = _torch()
        b = torch.empty(max(int(G) + 1, 1), dtype=torch.int64, device=self.pos.device)   # G < 1: the call refuses it
        _check(lib().bh_shard_bounds_groups(self.ctx.h, self.h, _ptr(group_work), int(G), _ptr(b)))
        return b

    def set_walk_shape(self, shape):
        """Wavefronts per workgroup (1, 2, 4, 8), | WALK_PERSISTENT for the persistent form."""
        _check(lib().bh_tree_set_walk_shape(self.ctx.h, self.h, int(shape)))
        return self

    def info(self):
        nn = C.c_int64()
        lo = (C.c_double * 3)()
        k = C.c_int32()
        _check(lib().bh_tree_info(self.ctx.h, self.h, C.byref(nn), lo, C.byref(k)))
        return int(nn.value), [lo[0], lo[1], lo[2]], int(k.value)

    def export(self, with_mass=True, with_hash=False):
        """bh_tree_export: keys, perm and the node arrays (device tensors), the node count,
        and with_hash the per-body interaction-set checksums (needs upward())."""
        torch = _torch()
        nn, lo, k = self.info()
        dev = self.pos.device
        out = dict(
            keys=torch.empty(self.n, dtype=torch.int64, device=dev),
            perm=torch.empty(self.n, dtype=torch.int32, device=dev),
            level=torch.empty(nn, dtype=torch.int32, device=dev),
            first=torch.empty(nn, dtype=torch.int32, device=dev),
            count=torch.empty(nn, dtype=torch.int32, device=dev),
            parent=torch.empty(nn, dtype=torch.int32, device=dev),
            M=torch.empty(nn, dtype=torch.float64, device=dev) if with_mass else None,
            com=torch.empty((nn, 3), dtype=torch.float64, device=dev) if with_mass else None,
            isect_hash=torch.empty(self.n, dtype=torch.int64, device=dev) if with_hash else None,
        )
        nno = C.c_int64(-1)
        _check(lib().bh_tree_export(self.ctx.h, self.h, _ptr(out["keys"]), _ptr(out["perm"]), _ptr(out["level"]),
                                    _ptr(out["first"]), _ptr(out["count"]), _ptr(out["parent"]), _ptr(out["M"]),
                                    _ptr(out["com"]), C.byref(nno), _ptr(out["isect_hash"])))
        if int(nno.value) != nn:
            raise BHError(E_DEVICE, f"node count changed between bh_tree_info ({nn}) and bh_tree_export ({nno.value})")
        out.update(n_nodes=nn, lo=lo, k=k)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().bh_tree_free(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim:
    """bh_sim: KDK leapfrog with a tree rebuild every step, state updated in place."""

    def __init__(self, ctx: Context, pos, vel, mass, p: Params, acc=None):
        torch = _torch()
        n = int(mass.shape[0])
        for t, c in ((pos, 3), (vel, 3)):
            _need(t, n, c)
        _need(mass, n, 0)
        self.acc = acc if acc is not None else torch.zeros((n, 3), dtype=torch.float64, device=pos.device)
        self.ctx, self.n, self.p = ctx, n, p
        self.pos, self.vel, self.mass = pos, vel, mass
        nb = int(lib().bh_sim_workspace_bytes(n, C.byref(p)))
        self._raw, self.ws = workspace(nb, pos.device)
        h = _VP()
        _check(lib().bh_sim_create(ctx.h, n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(self.acc), C.byref(p),
                                   _ptr(self.ws), nb, C.byref(h)))
        self.h = h

    def step(self, nsteps, dt):
        _check(lib().bh_step(self.ctx.h, self.h, int(nsteps), float(dt)))

    def set_walk_shape(self, shape):
        _check(lib().bh_sim_set_walk_shape(self.ctx.h, self.h, int(shape)))

    def energy(self):
        kw = (C.c_double * 2)()
        _check(lib().bh_energy(self.ctx.h, self.h, kw))
        return kw[0], kw[1]

    def close(self):
        if getattr(self, "h", None):
            lib().bh_sim_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Forest:
    """bh_forest: many simulations, concatenated rows, one launch sequence per step."""

    def __init__(self, ctx: Context, ns, plist, pos, vel, mass, acc=None):
        torch = _torch()
        self.ns = [int(v) for v in ns]
        n = sum(self.ns)
        for t, c in ((pos, 3), (vel, 3)):
            _need(t, n, c)
        _need(mass, n, 0)
        self.ctx, self.n = ctx, n
        self.pos, self.vel, self.mass = pos, vel, mass
        self.acc = acc if acc is not None else torch.zeros((n, 3), dtype=torch.float64, device=pos.device)
        k = len(self.ns)
        self._n = (C.c_int64 * k)(*self.ns)
        self._p = (Params * k)(*plist)
        nb = int(lib().bh_forest_workspace_bytes(k, self._n, self._p))
        if nb == 0:
            raise BHError(E_INVAL, "invalid forest parameters")
        self._raw, self.ws = workspace(nb, pos.device)
        h = _VP()
        _check(lib().bh_forest_create(ctx.h, k, self._n, self._p, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(self.acc),
                                      _ptr(self.ws), nb, C.byref(h)))
        self.h = h

    def _dt(self, dt):
        k = len(self.ns)
        if not hasattr(dt, "__len__"):
            dt = [float(dt)] * k
        return (C.c_double * k)(*[float(v) for v in dt])

    def step(self, nsteps, dt):
        _check(lib().bh_forest_step(self.ctx.h, self.h, int(nsteps), self._dt(dt)))

    def step_graph(self, nsteps, dt):
        _check(lib().bh_forest_step_graph(self.ctx.h, self.h, int(nsteps), self._dt(dt)))

    def autotune(self, cached=False):
        """Times the walk in every launch shape (TUNE_SHAPES) at the current positions and keeps
        the fastest; cached: take the tuning cache's shape for this forest's key when it has one
        (timings then -1).  Returns (shape, {shape: ms})."""
        w = C.c_int32()
        ms = (C.c_double * len(TUNE_SHAPES))()
        _check(lib().bh_forest_autotune(self.ctx.h, self.h, TUNE_CACHED if cached else 0, C.byref(w), ms))
        return int(w.value), {k: float(ms[i]) for i, k in enumerate(TUNE_SHAPES)}

    def set_walk_shape(self, shape):
        _check(lib().bh_forest_set_walk_shape(self.ctx.h, self.h, int(shape)))

    def forces(self, pot=None):
        _check(lib().bh_forest_forces(self.ctx.h, self.h, _ptr(pot)))
        return self.acc

    def energy(self):
        k = len(self.ns)
        out = (C.c_double * (2 * k))()
        _check(lib().bh_forest_energy(self.ctx.h, self.h, out))
        return [(out[2 * s], out[2 * s + 1]) for s in range(k)]

    def close(self):
        if getattr(self, "h", None):
            lib().bh_forest_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


REQ_RELEASE = 1
STATE_NAMES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class Server:
    """bh_server: continuous batching of simulation requests on its own thread and stream."""

    def __init__(self, ctx: Context, arena_bytes, max_slots=64, max_resident=1 << 24):
        self.ctx = ctx
        self._raw, self.arena = workspace(int(arena_bytes), ctx.device)
        h = _VP()
        _check(lib().bh_server_create(ctx.h, _ptr(self.arena), int(arena_bytes), int(max_slots), int(max_resident),
                                      C.byref(h)))
        self.h = h

    def submit(self, n, steps, ic_kind, seed, p: Params, dt, release=False):
        pp = Params(p.theta, p.eps, p.G, p.leaf_cap, p.precision, (p.flags | REQ_RELEASE) if release else p.flags, 0)
        r = Request(int(n), int(steps), int(ic_kind), int(seed) & 0xFFFFFFFFFFFFFFFF, pp, float(dt))
        rid = C.c_uint64()
        _check(lib().bh_server_submit(self.h, C.byref(r), C.byref(rid)))
        return int(rid.value)

    def poll(self, rid):
        res = Result()
        st = lib().bh_server_poll(self.h, C.c_uint64(rid), C.byref(res))
        if st not in (OK, E_BUSY, E_CANCELLED, E_DEVICE):
            _check(st)
        return dict(state=STATE_NAMES.get(res.state, res.state), steps_done=res.steps_done, t_submit=res.t_submit,
                    t_admit=res.t_admit, t_done=res.t_done, K=res.K, W=res.W)

    def fetch(self, rid, n):
        torch = _torch()
        pos = torch.empty((n, 3), dtype=torch.float64, device=self.ctx.device)
        vel = torch.empty((n, 3), dtype=torch.float64, device=self.ctx.device)
        # the copies run on the server's own stream: torch's pending work on these blocks first
        torch.cuda.current_stream(pos.device).synchronize()
        _check(lib().bh_server_fetch(self.h, C.c_uint64(rid), _ptr(pos), _ptr(vel)))
        return pos, vel

    def cancel(self, rid):
        _check(lib().bh_server_cancel(self.h, C.c_uint64(rid)))

    def now(self):
        return float(lib().bh_server_now(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().bh_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ic_workspace_bytes():
    return int(lib().bh_ic_workspace_bytes())


def ic_generate(ctx: Context, kind, n, seed, a=1.0, M=1.0):
    """Device-side Plummer (kind 0) or uniform cube (kind 1) initial conditions."""
    torch = _torch()
    dev = ctx.device
    pos = torch.empty((n, 3), dtype=torch.float64, device=dev)
    vel = torch.empty((n, 3), dtype=torch.float64, device=dev)
    mass = torch.empty(n, dtype=torch.float64, device=dev)
    nb = ic_workspace_bytes()
    _raw, ws = workspace(nb, dev)
    _check(lib().bh_ic_generate(ctx.h, int(kind), int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, float(a), float(M),
                                _ptr(pos), _ptr(vel), _ptr(mass), _ptr(ws), nb))
    return pos, vel, mass


def tune_cache_load(path):
    """bh_tune_cache_load: merges the JSON tuning cache at `path` into the process's cache."""
    _check(lib().bh_tune_cache_load(str(path).encode()))


def tune_cache_save(path):
    _check(lib().bh_tune_cache_save(str(path).encode()))


def tune_cache_clear():
    _check(lib().bh_tune_cache_clear())


def tune_cache_size():
    return int(lib().bh_tune_cache_size())
