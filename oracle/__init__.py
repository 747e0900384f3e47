"""ctypes front end of the plain-C Barnes-Hut oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg.  The product library never imports,
links or runs anything in this directory.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB = HERE / "liboracle.so"
SRC = [HERE / "bh_oracle.c"]

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C")


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("eps", C.c_double), ("G", C.c_double), ("leaf_cap", C.c_int32),
                ("quad", C.c_int32), ("open", C.c_int32)]


def build(force: bool = True) -> Path:
    """Compile liboracle.so with gcc (FP64, no contraction, OpenMP for the walk loops)."""
    if force or not LIB.exists():
        tmp = LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", str(tmp)] + [str(s) for s in SRC] + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        L.or_root_cube.argtypes = [C.c_int64, _f64p, _f64p, C.POINTER(C.c_int32)]
        L.or_interleave.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_interleave.restype = C.c_uint64
        L.or_keys.argtypes = [C.c_int64, _f64p, _f64p, C.c_int32, _u64p]
        L.or_order.argtypes = [C.c_int64, _u64p, _u32p]
        L.or_tree_create.argtypes = [C.c_int64, _f64p, _f64p, C.c_int32]
        L.or_tree_create.restype = C.c_void_p
        L.or_tree_destroy.argtypes = [C.c_void_p]
        L.or_tree_nn.argtypes = [C.c_void_p]
        L.or_tree_nn.restype = C.c_int64
        L.or_tree_moments.argtypes = [C.c_void_p, _f64p]
        L.or_tree_walk_group.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int32, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.or_tree_walk_group_ranges.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int64, _i64p, C.c_int64,
                                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p, C.c_int]
        L.or_tree_group_cubes.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
        L.or_tree_group_cubes.restype = C.c_int64
        L.or_tree_export.argtypes = [C.c_void_p, _f64p, C.POINTER(C.c_int32), _u64p, _u32p, _i32p,
                                     _u32p, _u32p, _i32p, _i32p, _f64p, _f64p]
        opt = lambda t: C.c_void_p  # noqa: E731  (nullable array arguments)
        L.or_tree_walk.argtypes = [C.c_void_p, _f64p, C.POINTER(Params), C.c_int64, C.c_void_p,
                                   opt(0), opt(0), opt(0), opt(0), opt(0), C.c_int]
        L.or_forces.argtypes = [C.c_int64, _f64p, _f64p, C.POINTER(Params), C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.or_direct.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_double, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int]
        L.or_kdk.argtypes = [C.c_int64, _f64p, _f64p, _f64p, C.POINTER(Params), C.c_double, C.c_int32,
                             _f64p, C.c_int32, C.c_void_p, C.c_int]
        L.or_energy.argtypes = [C.c_int64, _f64p, _f64p, C.c_void_p, _f64p]
        L.or_open_r2.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int32]
        L.or_open_r2.restype = C.c_double
        L.or_mix64.argtypes = [C.c_uint64]
        L.or_mix64.restype = C.c_uint64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def mix64(x: int) -> int:
    return int(lib().or_mix64(C.c_uint64(int(x) & 0xFFFFFFFFFFFFFFFF)))


def interleave(qx: int, qy: int, qz: int) -> int:
    return int(lib().or_interleave(qx, qy, qz))


def root_cube(pos):
    pos = _f64(pos, (-1, 3))
    lo = np.zeros(3)
    k = C.c_int32()
    lib().or_root_cube(pos.shape[0], pos, lo, C.byref(k))
    return lo, int(k.value)


def keys(pos, lo, k):
    pos = _f64(pos, (-1, 3))
    out = np.zeros(pos.shape[0], dtype=np.uint64)
    lib().or_keys(pos.shape[0], pos, _f64(lo), int(k), out)
    return out


def order(keys_):
    keys_ = np.ascontiguousarray(keys_, dtype=np.uint64)
    perm = np.zeros(keys_.shape[0], dtype=np.uint32)
    lib().or_order(keys_.shape[0], keys_, perm)
    return perm


OPEN = {"side": 0, "bmax": 1, "offset": 2}


def params(theta=0.5, eps=0.01, G=1.0, leaf_cap=1, quad=False, open="side"):
    """open: the opening radius r of r^2 < theta^2 D^2 ("side", "bmax" or "offset")."""
    return Params(float(theta), float(eps), float(G), int(leaf_cap), int(bool(quad)), OPEN[open])


class Tree:
    """Oracle tree over (pos, mass): keys, order, canonical nodes, M and com."""

    def __init__(self, pos, mass, leaf_cap=1):
        self.pos = _f64(pos, (-1, 3))
        self.mass = _f64(mass)
        self.n = self.pos.shape[0]
        h = lib().or_tree_create(self.n, self.pos, self.mass, int(leaf_cap))
        if not h:
            raise ValueError("oracle tree build failed")
        self._h = h
        nn = lib().or_tree_nn(h)
        self.nn = nn
        self.lo = np.zeros(3)
        k = C.c_int32()
        self.keys = np.zeros(self.n, np.uint64)
        self.perm = np.zeros(self.n, np.uint32)
        self.level = np.zeros(nn, np.int32)
        self.first = np.zeros(nn, np.uint32)
        self.count = np.zeros(nn, np.uint32)
        self.parent = np.zeros(nn, np.int32)
        self.nchild = np.zeros(nn, np.int32)
        self.M = np.zeros(nn)
        self.com = np.zeros((nn, 3))
        lib().or_tree_export(h, self.lo, C.byref(k), self.keys, self.perm, self.level, self.first,
                             self.count, self.parent, self.nchild, self.M, self.com)
        self.k = int(k.value)
        self.L = 2.0 ** self.k

    def moments(self):
        """Second moments about each node's centre of mass (nn x 6: xx yy zz xy xz yz)."""
        out = np.zeros((self.nn, 6))
        lib().or_tree_moments(self._h, out)
        return out

    def open_r2(self, theta, open):
        """r^2 of every node under the opening variant `open` (see or_open_r2)."""
        p = params(theta, 0.0, 1.0, 1, False, open)
        return np.array([lib().or_open_r2(self._h, C.byref(p), i) for i in range(self.nn)])

    def walk(self, theta=0.5, eps=0.01, G=1.0, targets=None, nthreads=0, quad=False, open="side"):
        p = params(theta, eps, G, 1, quad, open)
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
        nt = self.n if t is None else t.shape[0]
        acc = np.zeros((nt, 3))
        pot = np.zeros(nt)
        nm = np.zeros(nt, np.int64)
        np_ = np.zeros(nt, np.int64)
        hs = np.zeros(nt, np.uint64)
        rc = lib().or_tree_walk(self._h, self.pos, C.byref(p), nt, _ptr(t), _ptr(acc), _ptr(pot),
                                _ptr(nm), _ptr(np_), _ptr(hs), int(nthreads))
        if rc:
            raise ValueError("oracle walk rejected its arguments")
        return dict(acc=acc, pot=pot, n_mono=nm, n_p2p=np_, hash=hs)

    def group_cubes(self, cap=64):
        """Start ranks of the cube-based groups (largest cubes holding at most cap bodies), n at the end."""
        ng = lib().or_tree_group_cubes(self._h, int(cap), None)
        if ng < 1:
            raise ValueError("bad group cap")
        starts = np.zeros(ng + 1, np.int64)
        lib().or_tree_group_cubes(self._h, int(cap), starts.ctypes.data_as(C.c_void_p))
        return starts

    def walk_group(self, theta=0.5, eps=0.01, G=1.0, group=64, targets=None, nthreads=0, starts=None):
        """Group-criterion variant: one interaction list per group of key-consecutive bodies,
        `group` at a time, or the groups given by their start ranks (`starts`, n at the end)."""
        p = params(theta, eps, G, 1)
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
        nt = self.n if t is None else t.shape[0]
        acc = np.zeros((nt, 3))
        pot = np.zeros(nt)
        nm = np.zeros(nt, np.int64)
        np_ = np.zeros(nt, np.int64)
        hs = np.zeros(nt, np.uint64)
        if starts is None:
            rc = lib().or_tree_walk_group(self._h, C.byref(p), int(group), nt, _ptr(t), _ptr(acc), _ptr(pot),
                                          _ptr(nm), _ptr(np_), _ptr(hs), int(nthreads))
        else:
            st = np.ascontiguousarray(starts, dtype=np.int64)
            rc = lib().or_tree_walk_group_ranges(self._h, C.byref(p), st.shape[0] - 1, st, nt, _ptr(t), _ptr(acc),
                                                 _ptr(pot), _ptr(nm), _ptr(np_), _ptr(hs), int(nthreads))
        if rc:
            raise ValueError("oracle group walk rejected its arguments")
        return dict(acc=acc, pot=pot, n_mono=nm, n_p2p=np_, hash=hs)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_tree_destroy(h)
            self._h = None


def forces(pos, mass, theta=0.5, eps=0.01, G=1.0, leaf_cap=1, targets=None, nthreads=0, quad=False,
           open="side"):
    t = Tree(pos, mass, leaf_cap)
    return t.walk(theta, eps, G, targets, nthreads, quad, open)


def direct(pos, mass, eps=0.01, G=1.0, targets=None, nthreads=0):
    pos = _f64(pos, (-1, 3))
    mass = _f64(mass)
    t = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = pos.shape[0] if t is None else t.shape[0]
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    lib().or_direct(pos.shape[0], pos, mass, float(eps), float(G), nt, _ptr(t), _ptr(acc), _ptr(pot),
                    int(nthreads))
    return dict(acc=acc, pot=pot)


def kdk(pos, vel, mass, dt, nsteps, theta=0.5, eps=0.01, G=1.0, leaf_cap=1, acc=None, nthreads=0, quad=False,
        open="side"):
    """Returns (pos, vel, acc, pot) after nsteps leapfrog steps (copies; inputs untouched)."""
    pos = _f64(pos, (-1, 3)).copy()
    vel = _f64(vel, (-1, 3)).copy()
    mass = _f64(mass)
    have = acc is not None
    a = _f64(acc, (-1, 3)).copy() if have else np.zeros_like(pos)
    pot = np.zeros(pos.shape[0])
    p = params(theta, eps, G, leaf_cap, quad, open)
    rc = lib().or_kdk(pos.shape[0], pos, vel, mass, C.byref(p), float(dt), int(nsteps), a, int(have),
                      _ptr(pot), int(nthreads))
    if rc:
        raise ValueError("oracle kdk failed")
    return pos, vel, a, pot


def energy(vel, mass, pot):
    vel = _f64(vel, (-1, 3))
    mass = _f64(mass)
    pot = _f64(pot)
    out = np.zeros(2)
    lib().or_energy(mass.shape[0], vel, mass, _ptr(pot), out)
    return float(out[0]), float(out[1])
