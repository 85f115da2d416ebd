"""Pins of the oracle's field E = -grad Phi_RF at the targets (Algorithm 1, step 5), every
image held fixed.

* It is minus the gradient of the oracle's own potential, taken by fourth-order central
  differences of the potential at displaced targets (a different code path: the potential
  routines), for the exact surface dipole and the paper's +-dy/2 pair, well inside and within
  1e-3 a of the interface (the step scaled to the distance to the nearest image).
* Where the truncation error vanishes (sources and targets inside 0.55 a, p = 24) it is
  minus the gradient of the converged Kirkwood series (O2), to the differences' accuracy;
  at r < 0.9 a (C1-like geometry, p = 20) the two agree to the method's error (<1e-4).
* The surface images alone give minus the gradient of the harmonic polynomial they
  represent inside (Green's second identity discretised by the Fibonacci rule).
* No dielectric jump and no screening (eps1 = eps2, kappa = 0): no image, no field.
* A centred charge has a constant reaction potential, hence no field (to the Fibonacci
  rule's accuracy well inside).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _fd(f, T, h):
    """-grad f at the rows of T by fourth-order central differences with steps h (per row)."""
    h = np.broadcast_to(np.asarray(h, dtype=float), (len(T),))[:, None]
    out = np.zeros_like(T)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        out[:, k] = -(8 * (f(T + h * e) - f(T - h * e)) - (f(T + 2 * h * e) - f(T - 2 * h * e))) / (12 * h[:, 0])
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dipole", [0, 1])
def test_field_is_minus_gradient_of_potential(dipole):
    s = W.workload_c1().systems[0]
    prm = oracle.Params(a=10.0, eps1=1.0, eps2=80.0, kappa=0.1, p=10, P=400, M=600, dipole=dipole)
    r = np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2)
    T = np.stack([s.x, s.y, s.z], axis=1)[r < 9.0]
    _, E = oracle.hsma_field(prm, s.x, s.y, s.z, s.q, targets=T)
    fd = _fd(lambda t: oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, targets=t), T, 1e-3 * prm.a)
    assert _rel(E, fd) <= 1e-8


def test_field_near_the_interface_is_minus_gradient():
    """Ions within 1e-3 a of the interface: their own images are ~2e-3 a away, so the step is
    1e-3 of the distance to the nearest image."""
    a = 10.0
    rng = np.random.default_rng(11)
    pos = W.uniform_ball(rng, 60, a)
    for k in range(6):
        d = rng.standard_normal(3)
        pos[k] = d / np.linalg.norm(d) * a * (1.0 - 1e-4 * (k + 1) ** 2)
    q = W.balanced_charges(rng, 60)
    prm = oracle.Params(a=a, eps1=1.0, eps2=80.0, kappa=0.5, p=10, P=400, M=600)
    x, y, z = pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()
    T = pos[:6]
    rt = np.linalg.norm(T, axis=1)
    h = 1e-3 * (a * a / rt - rt)
    _, E = oracle.hsma_field(prm, x, y, z, q, targets=T)
    fd = _fd(lambda t: oracle.hsma_eval(prm, x, y, z, q, targets=t), T, h)
    assert _rel(E, fd) <= 1e-7


@pytest.mark.parametrize("eps1,eps2,kappa", [(1.0, 80.0, 0.1), (80.0, 80.0, 0.5), (2.0, 80.0, 5.0)])
def test_field_matches_kirkwood_well_inside(eps1, eps2, kappa):
    a = 4.0
    rng = np.random.default_rng(5)
    n = 10
    pos = rng.standard_normal((n, 3))
    pos *= (0.55 * a * rng.random(n) ** (1 / 3) / np.linalg.norm(pos, axis=1))[:, None]
    q = rng.choice([-1.0, 1.0, 2.0], n)
    prm = oracle.Params(a=a, eps1=eps1, eps2=eps2, kappa=kappa, p=24, P=2 * 1598, M=1000, F1=987)
    _, E = oracle.hsma_field(prm, pos[:, 0], pos[:, 1], pos[:, 2], q)
    fd = _fd(lambda t: oracle.kirkwood_eval(a, eps1, eps2, kappa, pos[:, 0], pos[:, 1], pos[:, 2], q, targets=t),
             pos, 1e-3 * a)
    assert np.max(np.abs(E - fd)) <= 1e-8 * np.max(np.abs(fd))


def test_field_matches_kirkwood_to_method_error():
    s = W.small_uniform(N=100, a=10.0, seed=W.SEED_BASE + 5)
    r = np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2)
    T = np.stack([s.x, s.y, s.z], axis=1)[r < 9.0]
    prm = oracle.Params(a=10.0, eps1=1.0, eps2=80.0, kappa=0.1, p=20, P=1600, M=2400)
    _, E = oracle.hsma_field(prm, s.x, s.y, s.z, s.q, targets=T)
    fd = _fd(lambda t: oracle.kirkwood_eval(10.0, 1.0, 80.0, 0.1, s.x, s.y, s.z, s.q, targets=t), T, 1e-3 * 10.0)
    assert _rel(E, fd) <= 1e-4


@pytest.mark.parametrize("dipole,tol", [(0, 1e-9), (1, 1e-7)])
def test_surface_field_is_minus_gradient_of_the_harmonic(dipole, tol):
    a = 2.0
    rng = np.random.default_rng(9)
    prm = oracle.Params(a=a, eps1=1.0, eps2=80.0, kappa=0.3, p=8, P=2 * 1598, M=200, F1=987, dipole=dipole)
    Ah = rng.standard_normal(prm.K)
    nodes, w = oracle.fibonacci_nodes(987, 1597, (1 + prm.tau) * a)
    Q, D = oracle.surface_strengths(prm, Ah, nodes, w)
    tg = rng.standard_normal((30, 3))
    tg *= (0.6 * a * rng.random(30) / np.linalg.norm(tg, axis=1))[:, None]
    nn = np.repeat(np.arange(prm.p + 1), 2 * np.arange(prm.p + 1) + 1)

    def harmonic(t):
        return np.array([np.sum(Ah * (np.linalg.norm(v) / a) ** nn * oracle.real_sh(prm.p, v)) for v in t])

    E = oracle.surface_field(prm, nodes, Q, D, tg)
    fd = _fd(harmonic, tg, 1e-3 * a)
    assert np.max(np.abs(E - fd)) <= tol * np.max(np.abs(fd))


def test_no_jump_no_field():
    s = W.small_uniform(N=50, a=5.0, seed=W.SEED_BASE + 6)
    prm = oracle.Params(a=5.0, eps1=2.0, eps2=2.0, kappa=0.0, p=6, P=144, M=100)
    phi, E = oracle.hsma_field(prm, s.x, s.y, s.z, s.q)
    assert np.all(phi == 0.0) and np.all(E == 0.0)


def test_centred_charge_has_no_field():
    a = 10.0
    prm = oracle.Params(a=a, eps1=1.0, eps2=80.0, kappa=0.1, p=20, P=1600, M=2400)
    rng = np.random.default_rng(3)
    T = rng.standard_normal((40, 3))
    T *= (0.5 * a * rng.random(40) ** (1 / 3) / np.linalg.norm(T, axis=1))[:, None]
    _, E = oracle.hsma_field(prm, [0.0], [0.0], [0.0], [1.0], targets=T)
    scale = 1.0 / (4 * math.pi * prm.eps1 * a * a)
    assert np.max(np.abs(E)) <= 1e-9 * scale
