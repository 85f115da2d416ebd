"""Pins of the oracle's spherical harmonics, node sets and least-squares fit.

* real SH: orthonormal under an exact product quadrature, and the addition theorem
  sum_m Y_nm(u) Y_nm(v) = (2n+1)/(4 pi) P_n(u.v) with numpy's Legendre polynomials;
* Fibonacci rule of Sec. 2.4: weights sum to the sphere's area, the single-layer
  potential of a uniform unit density is R everywhere inside, and low-degree
  harmonics integrate to zero;
* least squares: numpy.linalg.lstsq on a random system, and exact recovery of the
  multipole moments of band-limited sources from check-point potentials.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre

import oracle


def _sphere_quadrature(p):
    x, w = legendre.leggauss(p + 2)
    nphi = 2 * p + 4
    phis = 2 * np.pi * np.arange(nphi) / nphi
    pts, wts = [], []
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for ph in phis:
            pts.append((st * math.cos(ph), st * math.sin(ph), ct))
            wts.append(wt * 2 * np.pi / nphi)
    return np.array(pts), np.array(wts)


def test_real_sh_orthonormal():
    p = 12
    pts, wts = _sphere_quadrature(p)
    Y = np.array([oracle.real_sh(p, v) for v in pts])
    G = Y.T @ (Y * wts[:, None])
    assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-13


def test_real_sh_addition_theorem():
    rng = np.random.default_rng(5)
    p = 25
    for _ in range(5):
        u = rng.standard_normal(3)
        v = rng.standard_normal(3)
        cu = u / np.linalg.norm(u)
        cv = v / np.linalg.norm(v)
        Yu = oracle.real_sh(p, u)
        Yv = oracle.real_sh(p, v)
        for n in range(p + 1):
            s = Yu[n * n: (n + 1) ** 2] @ Yv[n * n: (n + 1) ** 2]
            c = np.zeros(n + 1)
            c[n] = 1
            ref = (2 * n + 1) / (4 * np.pi) * legendre.legval(cu @ cv, c)
            assert abs(s - ref) < 1e-12 * (2 * n + 1)


def test_real_sh_pole_and_zero_vector():
    # at the north pole only m = 0 survives: Y_n0 = sqrt((2n+1)/(4 pi))
    p = 8
    Y = oracle.real_sh(p, (0.0, 0.0, 3.0))
    for n in range(p + 1):
        for m in range(-n, n + 1):
            ref = math.sqrt((2 * n + 1) / (4 * math.pi)) if m == 0 else 0.0
            assert abs(Y[n * n + n + m] - ref) < 1e-14


@pytest.mark.parametrize("F1,F2", [(987, 1597), (123, 199), (494, 799)])
def test_fibonacci_weights_area(F1, F2):
    R = 1.7
    xyz, w = oracle.fibonacci_nodes(F1, F2, R)
    assert xyz.shape == (2 * (F2 + 1), 3)
    assert abs(w.sum() - 4 * np.pi * R * R) < 1e-12 * 4 * np.pi * R * R
    assert np.allclose(np.linalg.norm(xyz, axis=1), R, rtol=1e-15, atol=1e-15)
    # the two pole rows carry zero weight
    assert w[0] == 0.0 and w[1] == 0.0 and abs(w[-1]) < 1e-30 and abs(w[-2]) < 1e-30


@pytest.mark.parametrize("F1,F2,rmax,tol", [(987, 1597, 0.6, 1e-13), (123, 199, 0.3, 1e-11),
                                             (987, 1597, 0.9, 1e-4)])
def test_fibonacci_shell_potential(F1, F2, rmax, tol):
    # int dS / (4 pi |x - y|) over the sphere of radius R equals R for |x| < R; the rule
    # converges fast away from the sphere and slowly as |x| -> R (near-singular integrand)
    R = 1.1
    xyz, w = oracle.fibonacci_nodes(F1, F2, R)
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.standard_normal(3)
        x *= rng.uniform(0, rmax * R) / np.linalg.norm(x)
        val = np.sum(w / (4 * np.pi * np.linalg.norm(xyz - x, axis=1)))
        assert abs(val - R) < tol * R


def test_fibonacci_integrates_harmonics():
    xyz, w = oracle.fibonacci_nodes(987, 1597, 1.0)
    p = 12
    Y = np.array([oracle.real_sh(p, v) for v in xyz])
    integ = w @ Y
    ref = np.zeros_like(integ)
    ref[0] = math.sqrt(4 * math.pi)
    assert np.max(np.abs(integ - ref)) < 1e-10


def test_check_lattice():
    M, rc = 600, 11.0
    c = oracle.check_lattice(M, rc)
    assert np.allclose(np.linalg.norm(c, axis=1), rc, rtol=1e-14)
    assert np.all(np.diff(c[:, 2]) < 0)
    # equal-area in z: the mean of z over the lattice is 0, of z^2 is about 1/3
    assert abs(c[:, 2].mean()) < 1e-12 * rc
    assert abs((c[:, 2] ** 2).mean() / rc ** 2 - 1 / 3) < 1e-5


def test_lstsq_against_numpy():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((300, 47))
    B = rng.standard_normal((300, 3))
    X = oracle.lstsq(A, B)
    ref = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.max(np.abs(X - ref)) < 1e-12


def test_fit_recovers_band_limited_moments():
    """Sources deep inside (r <= 0.15 a) are band-limited to rounding at p = 20 for
    check points on rc = 1.1 a; the fit must return alpha_nm = sum q (r/a)^n Y_nm and
    beta_nm = sum q (r/a)^{n+1} Y_nm, the exterior moments of eq. "phicoul_final"."""
    a = 3.0
    prm = oracle.Params(a=a, eps1=2.5, eps2=80.0, kappa=0.4, p=20, P=400, M=700)
    rng = np.random.default_rng(2)
    n_src = 9
    pos = rng.standard_normal((n_src, 3))
    pos *= (0.15 * a * rng.random(n_src) ** (1 / 3) / np.linalg.norm(pos, axis=1))[:, None]
    q = rng.choice([-1.0, 1.0, 2.0], n_src)
    chk = oracle.check_lattice(prm.M, prm.rc_over_a * a)
    u, v = oracle.check_fields(prm, pos[:, 0], pos[:, 1], pos[:, 2], q, chk)
    al, be = oracle.fit_moments(prm, chk, u, v)
    ref_a = np.zeros(prm.K)
    ref_b = np.zeros(prm.K)
    for i in range(n_src):
        r = np.linalg.norm(pos[i])
        Y = oracle.real_sh(prm.p, pos[i])
        nn = np.repeat(np.arange(prm.p + 1), 2 * np.arange(prm.p + 1) + 1)
        ref_a += q[i] * (r / a) ** nn * Y
        ref_b += q[i] * (r / a) ** (nn + 1) * Y
    assert np.max(np.abs(al - ref_a)) < 1e-11
    assert np.max(np.abs(be - ref_b)) < 1e-11
