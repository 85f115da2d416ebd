"""Seeded synthetic ion clouds for the HSMA reaction-potential workloads.

This module only draws inputs: positions, charges and the physical/discretisation
parameters of each workload.  It holds none of the method's arithmetic, so both the
CPU oracle and the GPU path can be fed from it.

The paper times "N random charges inside the dielectric sphere" (Sec. 4.2) and
uses a single unit charge for its accuracy study (Sec. 4.1); there is no dataset.
Every workload below is synthetic:

* uniform in the ball: r = a U^(1/3), direction = g/|g| with g ~ N(0, I3);
* an optional shell population r^3 uniform in [(a - w)^3, a^3) to stress the
  near-interface images;
* charges +-1 (or a +-1/+-2 mix) with exactly balanced signs within each
  magnitude class, randomly permuted.

Generator: numpy PCG64, seed = 1907017240 + workload index, per-system seeds
seed * 1000003 + b.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1907017240


@dataclass
class Physics:
    """Physical parameters of one cavity: radius a, dielectrics, inverse Debye length."""
    a: float
    eps1: float
    eps2: float
    kappa: float


@dataclass
class Discretisation:
    """HSMA discretisation: surface nodes P, check points M, SH order p, tau, check radius."""
    P: int
    M: int
    p: int
    tau: float = 0.1
    rc_over_a: float = 1.1


@dataclass
class System:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    phys: Physics

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    disc: Discretisation
    systems: list = field(default_factory=list)
    note: str = ""


def default_order(P: int) -> int:
    """SH truncation order used when only the surface grid size P is given: P = (2p)^2."""
    return int(math.isqrt(P) // 2)


def _directions(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(g, axis=1)
    # a zero vector has probability 0; guard anyway
    bad = nrm == 0.0
    while np.any(bad):
        g[bad] = rng.standard_normal((int(bad.sum()), 3))
        nrm = np.linalg.norm(g, axis=1)
        bad = nrm == 0.0
    return g / nrm[:, None]


def uniform_ball(rng: np.random.Generator, n: int, a: float, rmax: float | None = None) -> np.ndarray:
    rmax = a if rmax is None else rmax
    r = rmax * rng.random(n) ** (1.0 / 3.0)
    return _directions(rng, n) * r[:, None]


def shell(rng: np.random.Generator, n: int, a: float, width: float) -> np.ndarray:
    lo3 = (a - width) ** 3
    r = (lo3 + rng.random(n) * (a ** 3 - lo3)) ** (1.0 / 3.0)
    return _directions(rng, n) * r[:, None]


def _clip_inside(pos: np.ndarray, a: float) -> np.ndarray:
    """Pull back the (measure-zero) points that rounding put on or outside r = a."""
    r = np.linalg.norm(pos, axis=1)
    lim = a * (1.0 - 1e-12)
    over = r >= lim
    if np.any(over):
        pos[over] *= (lim / r[over])[:, None]
    return pos


def balanced_charges(rng: np.random.Generator, n: int, mix: tuple = ((1.0, 1.0),)) -> np.ndarray:
    """Charges with exactly balanced signs inside each magnitude class.

    ``mix`` is a tuple of (magnitude, weight); class sizes are rounded to even counts.
    """
    weights = np.array([w for _, w in mix], dtype=np.float64)
    weights = weights / weights.sum()
    counts = [2 * int(round(n * w / 2.0)) for w in weights]
    counts[-1] = n - sum(counts[:-1])
    q = []
    for (mag, _), c in zip(mix, counts):
        h = c // 2
        q.append(np.full(h, mag))
        q.append(np.full(c - h, -mag))
    q = np.concatenate(q)
    return q[rng.permutation(n)]


def _system(pos: np.ndarray, q: np.ndarray, phys: Physics) -> System:
    pos = _clip_inside(np.ascontiguousarray(pos, dtype=np.float64), phys.a)
    return System(np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                  np.ascontiguousarray(pos[:, 2]), np.ascontiguousarray(q, dtype=np.float64), phys)


def small_uniform(N: int = 200, a: float = 10.0, seed: int = SEED_BASE + 0,
                  phys: Physics | None = None) -> System:
    """N ions uniform in the ball, charges +-1 balanced (the small one-system case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phys = phys or Physics(a, 1.0, 80.0, 0.1)
    pos = uniform_ball(rng, N, phys.a)
    q = balanced_charges(rng, N)
    return _system(pos, q, phys)


def workload_c1() -> Workload:
    """N=200 uniform in a=10, +-1 balanced, eps1=1, eps2=80, kappa=0.1; P=400, M=600."""
    disc = Discretisation(P=400, M=600, p=default_order(400))
    s = small_uniform(200, 10.0, SEED_BASE + 0)
    return Workload("c1_n200_a10", disc, [s], "single small system")


C2_PARAMS = [(80.0, 80.0, 0.05), (80.0, 80.0, 0.5), (1.0, 80.0, 0.05), (1.0, 80.0, 0.5)]


def c2_positions(N: int = 20000, a: float = 30.0, shell_frac: float = 0.3, width: float = 0.5,
                 seed: int = SEED_BASE + 1):
    rng = np.random.Generator(np.random.PCG64(seed))
    n_shell = int(round(shell_frac * N))
    pos = np.concatenate([shell(rng, n_shell, a, width), uniform_ball(rng, N - n_shell, a, a - width)])
    pos = pos[rng.permutation(N)]
    q = balanced_charges(rng, N)
    return pos, q


def workload_c2(N: int = 20000) -> Workload:
    """N=20000 (30% in the shell [a-1/2, a)), a=30, four (eps1, eps2, kappa) sets; P=1600, M=2400."""
    a = 30.0
    disc = Discretisation(P=1600, M=2400, p=default_order(1600))
    pos, q = c2_positions(N, a)
    systems = [_system(pos.copy(), q.copy(), Physics(a, e1, e2, k)) for (e1, e2, k) in C2_PARAMS]
    return Workload(f"c2_n{N}_a30_shell30", disc, systems, "same ions, four parameter sets")


def workload_c3(N: int = 1_000_000) -> Workload:
    """N=1e6 uniform in a=200, charges +-1 and +-2 (2:1), eps1=1, eps2=80, kappa=0.1; P=6400, M=9600."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2))
    a = 200.0
    disc = Discretisation(P=6400, M=9600, p=default_order(6400))
    pos = uniform_ball(rng, N, a)
    q = balanced_charges(rng, N, ((1.0, 2.0), (2.0, 1.0)))
    return Workload(f"c3_n{N}_a200", disc, [_system(pos, q, Physics(a, 1.0, 80.0, 0.1))])


def c4_sizes(nsys: int = 4096, lo: int = 100, hi: int = 20000, seed: int = SEED_BASE + 3) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(lo), math.log(hi), nsys)
    return (2 * np.round(0.5 * np.exp(u))).astype(np.int64)


def workload_c4(nsys: int = 4096) -> Workload:
    """nsys systems sharing geometry (a=25, eps1=1, eps2=78.5, kappa=0.3; P=1024, M=1536)."""
    a = 25.0
    disc = Discretisation(P=1024, M=1536, p=default_order(1024))
    sizes = c4_sizes(nsys)
    base = SEED_BASE + 3
    systems = []
    for b, n in enumerate(sizes):
        rng = np.random.Generator(np.random.PCG64(base * 1000003 + b))
        pos = uniform_ball(rng, int(n), a)
        q = balanced_charges(rng, int(n))
        systems.append(_system(pos, q, Physics(a, 1.0, 78.5, 0.3)))
    return Workload(f"c4_batched_{nsys}", disc, systems)


def workload_c5(nsys: int = 512) -> Workload:
    """nsys resident systems, N log-uniform in [500, 50000], a ~ U[15,40], kappa ~ U[0.05,1]."""
    base = SEED_BASE + 4
    rng = np.random.Generator(np.random.PCG64(base))
    u = rng.uniform(math.log(500), math.log(50000), nsys)
    sizes = (2 * np.round(0.5 * np.exp(u))).astype(np.int64)
    radii = rng.uniform(15.0, 40.0, nsys)
    kappas = rng.uniform(0.05, 1.0, nsys)
    disc = Discretisation(P=1024, M=1536, p=default_order(1024))
    systems = []
    for b in range(nsys):
        r2 = np.random.Generator(np.random.PCG64(base * 1000003 + b))
        pos = uniform_ball(r2, int(sizes[b]), float(radii[b]))
        q = balanced_charges(r2, int(sizes[b]))
        systems.append(_system(pos, q, Physics(float(radii[b]), 1.0, 78.5, float(kappas[b]))))
    return Workload(f"c5_serving_{nsys}", disc, systems)


def single_charge(r_s: float, a: float = 1.0, theta: float = 0.7, phi: float = 1.3, q: float = 1.0) -> tuple:
    """One charge at radius r_s (the accuracy study of Sec. 4.1)."""
    x = np.array([r_s * math.sin(theta) * math.cos(phi)])
    y = np.array([r_s * math.sin(theta) * math.sin(phi)])
    z = np.array([r_s * math.cos(theta)])
    return x, y, z, np.array([q])


def random_move(rng: np.random.Generator, pos: np.ndarray, a: float, half: float = 0.5) -> np.ndarray:
    """Displace one position by U([-half, half]^3), resampled until it stays inside r < a."""
    while True:
        cand = pos + rng.uniform(-half, half, 3)
        if np.linalg.norm(cand) < a * (1.0 - 1e-9):
            return cand
