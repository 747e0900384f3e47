"""Seeded synthetic initial conditions for Barnes-Hut N-body runs.

This module is the one place where inputs are made.  It is shared by the
CPU oracle side and the GPU side of every test and benchmark, and it holds
none of the Barnes-Hut arithmetic (no keys, no tree, no forces): only
random numbers and the classical initial-condition transforms.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
generator: every draw is a pure function of (counter, key), so particle i's
values never depend on how many particles are drawn or in what order.

Counter layout used everywhere below (ctr = 4 x uint32, key = 2 x uint32):
    key = (seed & 0xffffffff, seed >> 32)
    ctr = (i & 0xffffffff, i >> 32, call, tag)
where i is the particle index, `call` numbers the Philox calls made for
that particle, and `tag` separates generators (PLUMMER_TAG, CUBE_TAG, ...).
Each call yields four 32-bit words, i.e. two uniforms in (0, 1) of 53 bits:
    u(a, b) = ((a >> 5) * 2**26 + (b >> 6) + 0.5) * 2**-53.

The paper's inputs were Plummer spheres (section 4, experimental set-up),
made by a program from an online course that is not available; the Plummer
sampler here follows the published Aarseth-Henon-Wielen (1974) recipe.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint32(0x9E3779B9)
PHILOX_W1 = np.uint32(0xBB67AE85)

PLUMMER_TAG = 1
CUBE_TAG = 2
SEED_TAG = 3
ARRIVAL_TAG = 4

#: Plummer radius cut, as an enclosed-mass fraction (keeps the bounding box and
#: the 2**-21 Morton grid resolution sane: r_max = 38.7 a instead of ~1e3 a).
PLUMMER_MASS_CUT = 0.999

_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.  ctr: (n, 4) uint32, key: 2 uint32 -> (n, 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint32).reshape(-1, 4)
    x0 = c[:, 0].astype(np.uint64)
    x1 = c[:, 1].astype(np.uint32)
    x2 = c[:, 2].astype(np.uint64)
    x3 = c[:, 3].astype(np.uint32)
    k0 = np.uint32(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint32(int(key[1]) & 0xFFFFFFFF)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            p0 = PHILOX_M0 * x0          # 64-bit products of 32-bit words
            p1 = PHILOX_M1 * x2
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            n0 = hi1 ^ x1 ^ k0
            n1 = lo1
            n2 = hi0 ^ x3 ^ k1
            n3 = lo0
            x0, x1, x2, x3 = n0.astype(np.uint64), n1, n2.astype(np.uint64), n3
            if rnd != 9:
                k0 = np.uint32((int(k0) + int(PHILOX_W0)) & 0xFFFFFFFF)
                k1 = np.uint32((int(k1) + int(PHILOX_W1)) & 0xFFFFFFFF)
    out = np.empty((c.shape[0], 4), dtype=np.uint32)
    out[:, 0] = x0.astype(np.uint32)
    out[:, 1] = x1
    out[:, 2] = x2.astype(np.uint32)
    out[:, 3] = x3
    return out


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def _ctr(idx: np.ndarray, call: int, tag: int) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    c = np.empty((idx.shape[0], 4), dtype=np.uint32)
    c[:, 0] = (idx & _MASK32).astype(np.uint32)
    c[:, 1] = (idx >> np.uint64(32)).astype(np.uint32)
    c[:, 2] = np.uint32(call)
    c[:, 3] = np.uint32(tag)
    return c


def u53(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Two 32-bit words -> a double in (0, 1) with 53 random bits (never 0 or 1)."""
    hi = (a.astype(np.uint64) >> np.uint64(5)).astype(np.float64)
    lo = (b.astype(np.uint64) >> np.uint64(6)).astype(np.float64)
    return (hi * 67108864.0 + lo + 0.5) * (2.0 ** -53)


def uniforms(seed: int, idx: np.ndarray, call: int, tag: int):
    """Two uniform doubles per index from one Philox call."""
    w = philox4x32_10(_ctr(idx, call, tag), _key(seed))
    return u53(w[:, 0], w[:, 1]), u53(w[:, 2], w[:, 3])


@dataclass
class System:
    pos: np.ndarray   # (n, 3) float64, row-major
    vel: np.ndarray   # (n, 3) float64
    mass: np.ndarray  # (n,) float64

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def _com_shift(pos, vel, mass):
    mt = mass.sum()
    pos -= (mass[:, None] * pos).sum(axis=0) / mt
    vel -= (mass[:, None] * vel).sum(axis=0) / mt


def plummer(n: int, seed: int, a: float = 1.0, total_mass: float = 1.0, G: float = 1.0,
            mass_cut: float = PLUMMER_MASS_CUT, centre=(0.0, 0.0, 0.0),
            bulk_velocity=(0.0, 0.0, 0.0), com_frame: bool = True) -> System:
    """Plummer sphere by the Aarseth-Henon-Wielen (1974) method.

    Radius from the inverted cumulative mass M(r)/M = r^3/(1+r^2)^(3/2) with
    the mass fraction drawn uniformly in (0, mass_cut); isotropic position;
    speed q * v_esc(r) with v_esc = sqrt(2GM/a) (1+r^2)^(-1/4) and q drawn by
    von Neumann rejection from g(q) = q^2 (1-q^2)^(7/2) under the bound 0.1;
    isotropic velocity; then shift to the zero-momentum, zero-dipole frame of
    the sphere, then place it at `centre` moving with `bulk_velocity`.
    Equal masses total_mass / n.
    """
    n = int(n)
    idx = np.arange(n, dtype=np.uint64)
    x1, x2 = uniforms(seed, idx, 0, PLUMMER_TAG)
    x3, x6 = uniforms(seed, idx, 1, PLUMMER_TAG)
    x7, _ = uniforms(seed, idx, 2, PLUMMER_TAG)
    frac = mass_cut * x1
    r = 1.0 / np.sqrt(frac ** (-2.0 / 3.0) - 1.0)
    z = (1.0 - 2.0 * x2) * r
    rho = np.sqrt(np.maximum(r * r - z * z, 0.0))
    phi = 2.0 * math.pi * x3
    pos = np.empty((n, 3))
    pos[:, 0] = rho * np.cos(phi)
    pos[:, 1] = rho * np.sin(phi)
    pos[:, 2] = z
    # speed fraction q by rejection; attempt k uses Philox call 3 + k
    q = np.zeros(n)
    todo = np.arange(n)
    call = 3
    while todo.size:
        x4, x5 = uniforms(seed, idx[todo], call, PLUMMER_TAG)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q[todo[ok]] = x4[ok]
        todo = todo[~ok]
        call += 1
        if call > 3 + 400:
            raise RuntimeError("Plummer speed rejection did not converge")
    v = q * math.sqrt(2.0 * G * total_mass / a) * (1.0 + r * r) ** (-0.25)
    vz = (1.0 - 2.0 * x6) * v
    vrho = np.sqrt(np.maximum(v * v - vz * vz, 0.0))
    psi = 2.0 * math.pi * x7
    vel = np.empty((n, 3))
    vel[:, 0] = vrho * np.cos(psi)
    vel[:, 1] = vrho * np.sin(psi)
    vel[:, 2] = vz
    pos *= a
    mass = np.full(n, total_mass / n)
    if com_frame:
        _com_shift(pos, vel, mass)
    pos += np.asarray(centre, dtype=np.float64)
    vel += np.asarray(bulk_velocity, dtype=np.float64)
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass)


def uniform_cube(n: int, seed: int, half: float = 1.0, mlo: float = 0.5, mhi: float = 1.5) -> System:
    """Positions uniform in [-half, half]^3, masses uniform in [mlo, mhi]/n, at rest."""
    n = int(n)
    idx = np.arange(n, dtype=np.uint64)
    u0, u1 = uniforms(seed, idx, 0, CUBE_TAG)
    u2, u3 = uniforms(seed, idx, 1, CUBE_TAG)
    pos = np.empty((n, 3))
    pos[:, 0] = (2.0 * u0 - 1.0) * half
    pos[:, 1] = (2.0 * u1 - 1.0) * half
    pos[:, 2] = (2.0 * u2 - 1.0) * half
    mass = (mlo + (mhi - mlo) * u3) / n
    return System(np.ascontiguousarray(pos), np.zeros((n, 3)), mass)


def concat(*systems: System) -> System:
    return System(np.concatenate([s.pos for s in systems]),
                  np.concatenate([s.vel for s in systems]),
                  np.concatenate([s.mass for s in systems]))


def two_plummer(n_each: int, seed_a: int, seed_b: int, sep: float = 5.0, speed: float = 0.3) -> System:
    """Two unit-mass Plummer spheres at +-(sep,0,0) approaching each other at -+(speed,0,0)."""
    a = plummer(n_each, seed_a, centre=(sep, 0.0, 0.0), bulk_velocity=(-speed, 0.0, 0.0))
    b = plummer(n_each, seed_b, centre=(-sep, 0.0, 0.0), bulk_velocity=(speed, 0.0, 0.0))
    return concat(a, b)


def derived_seeds(master: int, count: int, tag: int = SEED_TAG) -> np.ndarray:
    """`count` 64-bit seeds from one master seed."""
    w = philox4x32_10(_ctr(np.arange(count, dtype=np.uint64), 0, tag), _key(master))
    return (w[:, 0].astype(np.uint64) | (w[:, 1].astype(np.uint64) << np.uint64(32)))


def batch_instances(count: int = 512, master_seed: int = 6, nmin: int = 1024, nmax: int = 262144,
                    thetas=(0.4, 0.5, 0.7)):
    """Batch workload: per instance N log-uniform in [nmin, nmax], theta drawn from `thetas`,
    its own seed.  Returns a list of (n, theta, seed)."""
    idx = np.arange(count, dtype=np.uint64)
    ua, ub = uniforms(master_seed, idx, 0, SEED_TAG)
    seeds = derived_seeds(master_seed, count, tag=SEED_TAG + 16)
    ns = np.rint(np.exp(math.log(nmin) + ua * (math.log(nmax) - math.log(nmin)))).astype(np.int64)
    ns = np.clip(ns, nmin, nmax)
    th = np.asarray(thetas)[np.minimum((ub * len(thetas)).astype(np.int64), len(thetas) - 1)]
    return [(int(ns[k]), float(th[k]), int(seeds[k])) for k in range(count)]


def request_stream(count: int, rate: float, master_seed: int = 7, nmin: int = 4096, nmax: int = 4194304,
                   smin: int = 1, smax: int = 100):
    """Serving workload: Poisson arrivals at `rate`/s (exponential gaps), N log-uniform in
    [nmin, nmax], steps uniform on {smin..smax}, Plummer or cube 50/50, per-request seed.
    Returns a list of dicts sorted by arrival time."""
    idx = np.arange(count, dtype=np.uint64)
    g, un = uniforms(master_seed, idx, 0, ARRIVAL_TAG)
    us, uk = uniforms(master_seed, idx, 1, ARRIVAL_TAG)
    seeds = derived_seeds(master_seed, count, tag=ARRIVAL_TAG + 16)
    gaps = -np.log(g) / rate
    t = np.cumsum(gaps) - gaps[0]
    ns = np.clip(np.rint(np.exp(math.log(nmin) + un * (math.log(nmax) - math.log(nmin)))), nmin, nmax)
    steps = smin + np.minimum((us * (smax - smin + 1)).astype(np.int64), smax - smin)
    kind = (uk >= 0.5).astype(np.int64)
    return [dict(t=float(t[k]), n=int(ns[k]), steps=int(steps[k]), kind=int(kind[k]), seed=int(seeds[k]))
            for k in range(count)]
