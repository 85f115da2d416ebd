"""Pins of the oracle's Kirkwood factors (Sec. 2.2-2.3) against things other than itself.

* S_n = k_n/(mu k_n') against scipy's modified spherical Bessel functions (library);
* the same ratio from the finite sum for k_n printed in Sec. 2.2, evaluated here with
  exact rational arithmetic (a different formula from the oracle's recurrence);
* the decomposition M_n = gamma + dbar/(n + sigma) + Mhat_n (eq. "Anuapp"): exact when
  mu = 0, Mhat_n = O(1/mu^2) for large mu and O(mu) for small mu (eqs. "Snuinfty",
  "Snuzero");
* no dielectric or ionic jump (eps1 = eps2, kappa = 0) gives M_n = 0 for every n.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import spherical_kn

import oracle


def _S_scipy(n, mu):
    return spherical_kn(n, mu) / (mu * spherical_kn(n, mu, derivative=True))


@pytest.mark.parametrize("mu", [0.05, 0.75, 1.0, 5.0, 15.0, 40.0])
def test_S_n_against_scipy(mu):
    nmax = 60
    S, _ = oracle.kirkwood_factor(nmax, 0.5, mu)
    ref = np.array([_S_scipy(n, mu) for n in range(nmax + 1)])
    ok = np.isfinite(ref)
    assert ok.sum() > 10
    rel = np.abs(S[ok] - ref[ok]) / np.abs(ref[ok])
    assert rel.max() < 1e-13


def _S_paper_sum(n, mu):
    """k_n(mu) = pi e^{-mu}/(2 mu) sum_{l<=n} (n+l)!/(l!(n-l)!) (2 mu)^{-l} (Sec. 2.2), with
    its derivative taken term by term; the prefactor cancels in the ratio."""
    m = Fraction(mu).limit_denominator(10 ** 12)
    num = Fraction(0)
    den = Fraction(0)
    for l in range(n + 1):
        t = Fraction(math.factorial(n + l), math.factorial(l) * math.factorial(n - l)) / (2 * m) ** l
        num += t
        # d/dmu [e^{-mu} mu^{-l-1}] = -e^{-mu} mu^{-l-1} (1 + (l+1)/mu)
        den += t * (-(m + l + 1))
    return float(num / den)


@pytest.mark.parametrize("mu", [0.25, 1.0, 7.5, 30.0])
def test_S_n_against_paper_finite_sum(mu):
    nmax = 40
    S, _ = oracle.kirkwood_factor(nmax, 0.5, mu)
    for n in range(nmax + 1):
        ref = _S_paper_sum(n, mu)
        assert abs(S[n] - ref) <= 1e-14 * abs(ref), n


def test_S_0_closed_form():
    # k_0 = pi e^{-mu}/(2 mu) gives S_0 = -1/(1 + mu), the leading form being exact at n = 0
    for mu in (0.0, 0.3, 2.0, 50.0):
        S, _ = oracle.kirkwood_factor(3, 1.0, mu)
        assert abs(S[0] + 1.0 / (1.0 + mu)) < 1e-16


@pytest.mark.parametrize("eps", [1.0 / 80.0, 0.5, 1.0, 2.0 / 80.0])
def test_decomposition_exact_at_mu_zero(eps):
    nmax = 200
    _, M = oracle.kirkwood_factor(nmax, eps, 0.0)
    g, s, d = oracle.image_constants(eps, 0.0)
    n = np.arange(nmax + 1)
    assert np.max(np.abs(M - (g + d / (n + s)))) < 1e-15


def test_decomposition_remainder_orders():
    eps = 1.0 / 40.0
    n = np.arange(0, 12)

    def mhat(mu):
        _, M = oracle.kirkwood_factor(20, eps, mu)
        g, s, d = oracle.image_constants(eps, mu)
        return (M - (g + d / (n_all + s)))[: len(n)]

    n_all = np.arange(21)
    # large mu: Mhat_n ~ C_n / mu^2
    r1 = mhat(1e3) * 1e3 ** 2
    r2 = mhat(1e4) * 1e4 ** 2
    assert np.all(np.abs(r1[1:] - r2[1:]) <= 2e-2 * np.abs(r2[1:]))
    assert np.all(np.abs(r2) < 50.0)
    # small mu: Mhat_n ~ C_n mu
    s1 = mhat(1e-4) / 1e-4
    s2 = mhat(1e-5) / 1e-5
    assert np.all(np.abs(s1[1:] - s2[1:]) <= 1e-2 * np.abs(s2[1:]) + 1e-12)
    # n = 0 is exact for every mu (S_0 is exactly the leading form)
    for mu in (1e-3, 0.5, 5.0, 300.0):
        _, M = oracle.kirkwood_factor(2, eps, mu)
        g, s, d = oracle.image_constants(eps, mu)
        assert abs(M[0] - (g + d / s)) < 1e-14


def test_no_jump_no_reaction():
    _, M = oracle.kirkwood_factor(100, 1.0, 0.0)
    assert np.max(np.abs(M)) < 1e-15


def test_constants_values():
    # gamma, sigma, dbar for the parameters of Sec. 4 (eps = 2/80, mu = 5), from their definitions
    eps = 2.0 / 80.0
    g, s, d = oracle.image_constants(eps, 5.0)
    assert abs(g - (eps - 1) / (eps + 1)) < 1e-16
    assert abs(s - 6.0 / (1 + eps)) < 1e-15
    assert abs(d - (g * (1 - s) - 5.0 / (1 + eps))) < 1e-15
