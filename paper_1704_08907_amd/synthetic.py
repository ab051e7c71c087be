"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random-number generation and workload recipes only: it does
none of the method's arithmetic (no cell assignment, no distances, no sums), so
both the CPU oracle and the GPU path can be fed from it without sharing code.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), the k-th output being the 64-bit finaliser
applied to ``seed + k * 0x9E3779B97F4A7C15``.  Uniform doubles take the top 53
bits, ``(z >> 11) * 2**-53``, so they lie in [0, 1).  Normal variates use the
Box-Muller transform on pairs of uniforms.

Workloads follow the particle-method setting of the paper (Section 1: N particles
in a d-dimensional hypercube, each dimension periodic or not; Section 3: uniform
random positions in the periodic unit square).  Each workload's stream is seeded
with ``17040890700 + workload number``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
SEED_BASE = 17040890700


class SplitMix64:
    """Counter-based SplitMix64 stream; draws are consumed in call order."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed % (1 << 64))
        self.count = 0  # number of 64-bit outputs consumed so far

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            z = self.seed + k * GOLDEN
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int) -> np.ndarray:
        """n doubles in [0, 1)."""
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n: int) -> np.ndarray:
        """n standard normal doubles (Box-Muller on consecutive uniform pairs)."""
        m = (n + 1) // 2
        u = self.uniform(2 * m)
        u1 = 1.0 - u[0::2]  # in (0, 1]
        u2 = u[1::2]
        rad = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * m)
        z[0::2] = rad * np.cos(2.0 * math.pi * u2)
        z[1::2] = rad * np.sin(2.0 * math.pi * u2)
        return z[:n]


def np_dtype(precision: str):
    return {"f32": np.float32, "f64": np.float64}[precision]


def uniform_positions(rng: SplitMix64, n: int, lo, hi, precision: str) -> np.ndarray:
    """n points uniform in the box [lo, hi), row-major [n][d] in the given precision.

    A point is lo + u*(hi-lo) in float64, then rounded to the precision; a
    coordinate that rounds onto hi is replaced by lo so that every point lies in
    the half-open box.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.shape[0]
    dt = np_dtype(precision)
    u = rng.uniform(n * d).reshape(n, d)
    x = (lo + u * (hi - lo)).astype(dt)
    lo_p = lo.astype(dt)
    hi_p = hi.astype(dt)
    for k in range(d):
        col = x[:, k]
        col[col >= hi_p[k]] = lo_p[k]
    return np.ascontiguousarray(x)


def side_for_density(n: int, d: int, mean_neighbours: float, r: float = 1.0) -> float:
    """Box side giving on average ``mean_neighbours`` other points within r."""
    if d == 3:
        ball = 4.0 * math.pi / 3.0 * r ** 3
    elif d == 2:
        ball = math.pi * r ** 2
    else:
        ball = 2.0 * r
    return (n * ball / mean_neighbours) ** (1.0 / d)


@dataclass
class System:
    """One particle system: box, cutoff and positions (numpy, row-major)."""

    d: int
    lo: list
    hi: list
    periodic: list
    cutoff: float
    x: np.ndarray
    precision: str

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    precision: str
    systems: list = field(default_factory=list)
    op: str = "spring"
    params: tuple = ()
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return sum(s.n for s in self.systems)


def md_square(n: int = 1000, seed_offset: int = 1, scale: float = 1.0) -> Workload:
    """N=1000, d=2, periodic unit square, r=0.1, linear spring k=1, float64."""
    n = max(1, int(round(n * scale)))
    rng = SplitMix64(SEED_BASE + seed_offset)
    x = uniform_positions(rng, n, [0.0, 0.0], [1.0, 1.0], "f64")
    sys = System(2, [0.0, 0.0], [1.0, 1.0], [1, 1], 0.1, x, "f64")
    return Workload("md_square_n%d_d2_f64" % n, "f64", [sys], "spring", (1.0,))


def periodic_cube(n: int, mean_neighbours: float, seed_offset: int, op: str,
                  params: tuple, name: str, precision: str = "f32") -> Workload:
    L = side_for_density(n, 3, mean_neighbours)
    rng = SplitMix64(SEED_BASE + seed_offset)
    x = uniform_positions(rng, n, [0.0] * 3, [L] * 3, precision)
    sys = System(3, [0.0] * 3, [L] * 3, [1, 1, 1], 1.0, x, precision)
    w = Workload(name, precision, [sys], op, params)
    w.extra["gy"] = None
    return w


def spring_cube(n: int = 1 << 20, seed_offset: int = 2) -> Workload:
    """N=2^20, d=3 periodic cube with ~30 neighbours within r=1, spring k=1, float32."""
    w = periodic_cube(n, 30.0, seed_offset, "spring", (1.0,),
                      "spring_cube_n%d_d3_f32" % n)
    rng = SplitMix64(SEED_BASE + seed_offset + 1000)
    w.extra["gy"] = rng.normal(n * 3).astype(np.float32).reshape(n, 3)
    return w


def soft_sphere_cube(n: int = 1 << 18, seed_offset: int = 4) -> Workload:
    """N=2^18, d=3 periodic cube with ~40 neighbours within r=1, soft sphere, float32."""
    w = periodic_cube(n, 40.0, seed_offset, "soft_sphere", (),
                      "soft_sphere_cube_n%d_d3_f32" % n)
    w.extra["gy"] = np.ones((n, 1), dtype=np.float32)
    return w


def gaussian_square(n: int = 65536, seed_offset: int = 3):
    """Dense Gaussian sum inputs: n points uniform in [0,1]^2, w ~ N(0,1), float32."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    x = uniform_positions(rng, n, [0.0, 0.0], [1.0, 1.0], "f32")
    w = rng.normal(n).astype(np.float32)
    return x, w, 0.1


def batch_sizes(nsys: int = 512, seed_offset: int = 5, nmin: int = 256, nmax: int = 65536):
    """Per-system sizes, log-uniform in [nmin, nmax]."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    u = rng.uniform(nsys)
    ratio = nmax / nmin
    return [int(round(nmin * ratio ** ui)) for ui in u], rng


def batch_cubes(nsys: int = 512, seed_offset: int = 5, nmin: int = 256,
                nmax: int = 65536, mean_neighbours: float = 30.0) -> Workload:
    """Many independent d=3 periodic systems of uneven size, ~30 neighbours within r=1."""
    sizes, rng = batch_sizes(nsys, seed_offset, nmin, nmax)
    w = Workload("batch_%dsys_d3_f32" % nsys, "f32", [], "spring", (1.0,))
    for nb in sizes:
        L = side_for_density(nb, 3, mean_neighbours)
        x = uniform_positions(rng, nb, [0.0] * 3, [L] * 3, "f32")
        w.systems.append(System(3, [0.0] * 3, [L] * 3, [1, 1, 1], 1.0, x, "f32"))
    ntot = w.n
    w.extra["gy"] = np.ones((ntot, 1), dtype=np.float32)
    return w


def md_paper(n: int = 1 << 20, seed_offset: int = 6, precision: str = "f64") -> Workload:
    """The Section 3 example: n points uniform in the periodic unit square,
    cutoff sqrt(3/n) (about 3 pi ~ 9.4 neighbours for any n), exp force with
    c = 1e-3, step dt = 1, velocities starting at zero, float64."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    x = uniform_positions(rng, n, [0.0, 0.0], [1.0, 1.0], precision)
    sys = System(2, [0.0, 0.0], [1.0, 1.0], [1, 1], math.sqrt(3.0 / n), x, precision)
    w = Workload("md_paper_n%d_d2_%s" % (n, precision), precision, [sys], "exp_force", (1e-3,))
    w.extra["v"] = np.zeros((n, 2), dtype=np_dtype(precision))
    w.extra["dt"] = 1.0
    return w
