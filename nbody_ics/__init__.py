"""Seeded synthetic inputs for the direct N-body force path.

This module is the only code the oracle side and the GPU side share.  It draws
random numbers and shapes them into particle sets; it contains none of the
force, predictor or integrator arithmetic.

Workloads (the paper uses Plummer spheres, Results > Block time-step
simulations, and 131072 sources for its active-particle sweep, Results >
Block-size / active-particles):

* ``plummer``    equal-mass Plummer sphere in standard N-body units
                 (G = M = 1, virial radius 1), Aarseth-Henon-Wielen sampling.
* ``salpeter``   power-law mass function dN/dm ~ m^-2.35 on [0.1, 100],
                 normalised to total mass 1.
* ``active_set`` the first n_i entries of a seeded permutation, sorted: the
                 active sinks of one block time-step.
* ``source_times`` per-source times t_j = -2^-k, k uniform in {3..10}, so the
                 predictor has a different dt for every source.
* ``derivatives`` seeded Gaussian acceleration, jerk, snap and crackle used as
                 the predictor's Taylor coefficients.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "plummer",
    "salpeter",
    "active_set",
    "source_times",
    "derivatives",
    "SourceSet",
    "make_sources",
    "few_body_sizes",
]

# Standard-unit scale factors of the Plummer model (a = 1 model units):
# lengths by 3 pi / 16, velocities by sqrt(16 / (3 pi)).
_LEN = 3.0 * math.pi / 16.0
_VEL = math.sqrt(16.0 / (3.0 * math.pi))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Vectors of length r with uniformly random directions."""
    cos_t = rng.uniform(-1.0, 1.0, size=r.shape)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=r.shape)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    return np.stack([r * sin_t * np.cos(phi), r * sin_t * np.sin(phi), r * cos_t], axis=1)


def plummer(n: int, seed: int, rmax: float = 10.0):
    """Equal-mass Plummer sphere (Aarseth, Henon & Wielen 1974 recipe).

    Radius from the inverse cumulative mass X: r = (X^(-2/3) - 1)^(-1/2),
    redrawn while r > rmax (model units, a = 1).  Speed q (fraction of the
    local escape speed) by rejection sampling of g(q) = q^2 (1 - q^2)^(7/2)
    under the bound 0.1; v = q sqrt(2) (1 + r^2)^(-1/4).  Directions are
    isotropic.  Scaled to standard units and moved to the centre-of-mass
    frame.  Returns (m[n], x[n,3], v[n,3]) as float64.
    """
    if n <= 0:
        return np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3))
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        X = rng.uniform(0.0, 1.0, size=todo.size)
        with np.errstate(divide="ignore", invalid="ignore"):
            rr = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        ok = np.isfinite(rr) & (rr <= rmax)
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        q0 = rng.uniform(0.0, 1.0, size=todo.size)
        y = rng.uniform(0.0, 0.1, size=todo.size)
        ok = y < q0 * q0 * (1.0 - q0 * q0) ** 3.5
        q[todo[ok]] = q0[ok]
        todo = todo[~ok]
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    x = _isotropic(rng, r) * _LEN
    v = _isotropic(rng, speed) * _VEL
    m = np.full(n, 1.0 / n)
    x -= np.sum(m[:, None] * x, axis=0) / np.sum(m)
    v -= np.sum(m[:, None] * v, axis=0) / np.sum(m)
    return m, np.ascontiguousarray(x), np.ascontiguousarray(v)


def salpeter(n: int, seed: int, slope: float = 2.35, mlo: float = 0.1, mhi: float = 100.0) -> np.ndarray:
    """Masses with dN/dm ~ m^-slope on [mlo, mhi] by inverse-CDF sampling, normalised to sum 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, 1.0, size=n)
    p = 1.0 - slope
    m = (mlo**p + u * (mhi**p - mlo**p)) ** (1.0 / p)
    return m / np.sum(m)


def active_set(n: int, ni: int, seed: int) -> np.ndarray:
    """Sorted int32 addresses of ni active sinks out of n (first ni of a seeded permutation)."""
    if not 0 <= ni <= n:
        raise ValueError("need 0 <= ni <= n")
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.permutation(n)[:ni]).astype(np.int32)


def source_times(n: int, seed: int, kmin: int = 3, kmax: int = 10) -> np.ndarray:
    """Per-source times t_j = -2^-k with k uniform in {kmin..kmax}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(kmin, kmax + 1, size=n)
    return -np.ldexp(1.0, -k)


def derivatives(n: int, seed: int, scales=(0.5, 2.0, 10.0, 50.0)):
    """Seeded Gaussian (acc, jerk, snap, crackle), each [n,3] float64, with the given rms scales."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return tuple(np.ascontiguousarray(rng.normal(0.0, s, size=(n, 3))) for s in scales)


class SourceSet:
    """One synthetic source set: ids, masses, times and Taylor coefficients."""

    def __init__(self, m, x, v, t, a, jerk, snap=None, crackle=None, ids=None):
        n = len(m)
        self.n = n
        self.m = np.ascontiguousarray(m, dtype=np.float64)
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.v = np.ascontiguousarray(v, dtype=np.float64)
        self.t = np.ascontiguousarray(t, dtype=np.float64)
        self.a = np.ascontiguousarray(a, dtype=np.float64)
        self.jerk = np.ascontiguousarray(jerk, dtype=np.float64)
        self.snap = None if snap is None else np.ascontiguousarray(snap, dtype=np.float64)
        self.crackle = None if crackle is None else np.ascontiguousarray(crackle, dtype=np.float64)
        self.ids = np.arange(n, dtype=np.int64) if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
        self.addr = np.arange(n, dtype=np.int32)


def make_sources(n: int, seed: int, order: int = 4, masses: str = "equal", time_offsets: bool = True,
                 id_offset: int = 0) -> SourceSet:
    """Plummer sources with seeded times and Taylor coefficients.

    Seeds: positions/velocities ``seed``; Salpeter masses ``seed + 500``;
    times ``seed + 2000``; Taylor coefficients ``seed + 3000``.  With
    time_offsets False every t_j is 0 (shared time-step start).
    """
    m, x, v = plummer(n, seed)
    if masses == "salpeter":
        m = salpeter(n, seed + 500)
    elif masses != "equal":
        raise ValueError("masses must be 'equal' or 'salpeter'")
    t = source_times(n, seed + 2000) if time_offsets else np.zeros(n)
    a, jerk, snap, crackle = derivatives(n, seed + 3000)
    if order == 4:
        snap = crackle = None
    ids = np.arange(n, dtype=np.int64) + id_offset
    return SourceSet(m, x, v, t, a, jerk, snap, crackle, ids)


def few_body_sizes(n_systems: int, seed: int, lo: int = 3, hi: int = 96) -> np.ndarray:
    """Sizes of independent few-body systems, uniform integers in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n_systems).astype(np.int32)
