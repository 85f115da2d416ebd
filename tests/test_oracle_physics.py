"""Pins of the two oracles' physics.

O2 (Kirkwood series, Sec. 2.2) against:
* the interface problem itself (eqs. "phiinsideeq"-"boundarycondition"): per Legendre
  degree, eps1 dPhi_1/dr / Phi_1 on r = a must equal eps2 kappa k_n'(kappa a)/k_n(kappa a)
  with scipy's Bessel functions (or -(n+1) eps2 / a when kappa = 0);
* the centred-charge closed form q/(4 pi a) [1/(eps2 (1 + kappa a)) - 1/eps1];
* the symmetry G(x, x') = G(x', x); no reaction field when eps1 = eps2, kappa = 0;
* a 30-digit mpmath evaluation (its own Bessel functions) of the single-charge energy.

O1 (HSMA, Sec. 2.3-2.4) against O2:
* the accuracy statements printed in Sec. 4 (tests/golden/paper_accuracy_claims.json);
* near-exact agreement where the truncation error is negligible (sources and targets
  well inside), for one and several charges, dielectric jump or not;
* the surface images reproduce any harmonic polynomial inside (Green's second identity
  discretised by the Fibonacci rule), for the exact dipole and the paper's +-dy/2 pair.
"""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre
from scipy.special import spherical_kn

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_accuracy_claims.json")


def _centred(a, eps1, eps2, kappa, q=1.0):
    return q / (4 * math.pi * a) * (1.0 / (eps2 * (1.0 + kappa * a)) - 1.0 / eps1)


@pytest.mark.parametrize("a,eps1,eps2,kappa", [(10.0, 1.0, 80.0, 0.1), (30.0, 80.0, 80.0, 0.5),
                                               (1.0, 2.0, 80.0, 5.0), (25.0, 1.0, 78.5, 0.0)])
def test_centred_charge_closed_form(a, eps1, eps2, kappa):
    ref = _centred(a, eps1, eps2, kappa)
    z = np.zeros(1)
    k = oracle.kirkwood_eval(a, eps1, eps2, kappa, z, z, z, np.ones(1))
    assert abs(k[0] - ref) <= 1e-15 * abs(ref) + 1e-300
    prm = oracle.Params(a=a, eps1=eps1, eps2=eps2, kappa=kappa, p=10, P=400, M=600)
    h = oracle.hsma_eval(prm, z, z, z, np.ones(1))
    assert abs(h[0] - ref) <= 1e-13 * abs(ref)
    # and at any other target inside: the reaction field of a centred charge is uniform
    tg = np.array([[0.3 * a, -0.2 * a, 0.5 * a]])
    k2 = oracle.kirkwood_eval(a, eps1, eps2, kappa, z, z, z, np.ones(1), targets=tg)
    assert abs(k2[0] - ref) <= 1e-14 * abs(ref)
    # off the centre the double layer's Fibonacci rule carries the error: use F2 = 1597
    prm_fine = oracle.Params(a=a, eps1=eps1, eps2=eps2, kappa=kappa, p=10, P=2 * 1598, M=600, F1=987)
    h2 = oracle.hsma_eval(prm_fine, z, z, z, np.ones(1), targets=tg)
    assert abs(h2[0] - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("eps1,eps2,kappa", [(2.0, 80.0, 5.0), (1.0, 80.0, 0.1), (80.0, 80.0, 0.5),
                                             (4.0, 20.0, 0.0)])
def test_kirkwood_satisfies_interface_conditions(eps1, eps2, kappa):
    a, r_s, q = 1.3, 0.7, 1.0
    nq = 80
    ct, wt = legendre.leggauss(nq)
    targets = np.stack([a * np.sqrt(1 - ct ** 2), np.zeros(nq), a * ct], axis=1)
    one = np.ones(1)
    phi = oracle.kirkwood_eval(a, eps1, eps2, kappa, 0 * one, 0 * one, r_s * one, q * one, targets=targets)
    for n in range(0, 16):
        c = np.zeros(n + 1)
        c[n] = 1
        An_an = (2 * n + 1) / 2 * np.sum(wt * phi * legendre.legval(ct, c))  # A_n a^n
        coul = q * r_s ** n / (4 * math.pi * eps1 * a ** (n + 1))
        phi1 = An_an + coul
        dphi1 = n * An_an / a - (n + 1) * coul / a
        if kappa > 0:
            mu = kappa * a
            dn = eps2 * kappa * spherical_kn(n, mu, derivative=True) / spherical_kn(n, mu)
        else:
            dn = -(n + 1) * eps2 / a
        lhs = eps1 * dphi1
        rhs = dn * phi1
        # scale: the Coulomb terms nearly cancel the reaction when M_n -> -1, and the
        # projection extracts a small component of a potential of size max|phi|
        scale = (abs(eps1 * (n + 1) / a) + abs(dn)) * (abs(coul) + np.max(np.abs(phi)))
        assert abs(lhs - rhs) <= 1e-12 * scale, n


def test_kirkwood_symmetry_and_no_jump():
    rng = np.random.default_rng(7)
    a = 2.0
    for _ in range(5):
        x1 = rng.uniform(-1, 1, 3) * 0.5 * a
        x2 = rng.uniform(-1, 1, 3) * 0.5 * a
        g12 = oracle.kirkwood_eval(a, 1.0, 80.0, 0.7, *x1.reshape(3, 1), np.ones(1), targets=x2[None])
        g21 = oracle.kirkwood_eval(a, 1.0, 80.0, 0.7, *x2.reshape(3, 1), np.ones(1), targets=x1[None])
        assert abs(g12[0] - g21[0]) <= 1e-14 * abs(g12[0])
        z = oracle.kirkwood_eval(a, 3.0, 3.0, 0.0, *x1.reshape(3, 1), np.ones(1), targets=x2[None])
        assert abs(z[0]) < 1e-15 / (4 * math.pi * 3.0 * a)


def test_hsma_no_jump_no_reaction():
    s = W.small_uniform(40, 5.0, phys=W.Physics(5.0, 3.0, 3.0, 0.0))
    prm = oracle.Params(a=5.0, eps1=3.0, eps2=3.0, kappa=0.0, p=8, P=400, M=200)
    phi = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
    scale = 1.0 / (4 * math.pi * 3.0 * 5.0)  # one unit charge at distance a
    assert np.max(np.abs(phi)) < 1e-13 * scale


def test_kirkwood_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    a, eps1, eps2, kappa = 1.0, 2.0, 80.0, 5.0
    mu = mp.mpf(kappa) * a
    eps = mp.mpf(eps1) / eps2

    def kn(n, z):
        return mp.sqrt(mp.pi / (2 * z)) * mp.besselk(n + mp.mpf(1) / 2, z)

    def dkn(n, z):
        return mp.diff(lambda t: kn(n, t), z)

    nterm = 400
    Mn = []
    for n in range(nterm):
        S = kn(n, mu) / (mu * dkn(n, mu))
        Mn.append((eps * (n + 1) * S + 1) / (eps * n * S - 1))
    for r_s in (0.5, 0.9):
        t = mp.mpf(r_s) ** 2
        e_ref = sum(Mn[n] * t ** n for n in range(nterm)) / (4 * mp.pi * eps1 * a) / 2
        x, y, z, q = W.single_charge(r_s, a)
        e = 0.5 * oracle.kirkwood_eval(a, eps1, eps2, kappa, x, y, z, q)[0]
        assert abs(e - float(e_ref)) <= 1e-14 * abs(float(e_ref))


def _claims():
    with open(GOLDEN) as f:
        return json.load(f)


def _self_energy_errors(p, tau, F1, F2, rs_list, setup, kirk_orders=()):
    out = []
    for r_s in rs_list:
        x, y, z, q = W.single_charge(r_s, setup["a"])
        ref = oracle.kirkwood_eval(setup["a"], setup["eps1"], setup["eps2"], setup["kappa"], x, y, z, q)[0]
        prm = oracle.Params(a=setup["a"], eps1=setup["eps1"], eps2=setup["eps2"], kappa=setup["kappa"], p=p,
                            P=2 * (F2 + 1), M=int(math.ceil(1.5 * (p + 1) ** 2)), tau=tau, rc_over_a=1.0 + tau,
                            F1=F1, dipole=0)
        h = oracle.hsma_eval(prm, x, y, z, q)[0]
        row = {"r_s": r_s, "ref": 0.5 * ref, "hsma": abs(0.5 * (h - ref))}
        for o in kirk_orders:
            k = oracle.kirkwood_eval(setup["a"], setup["eps1"], setup["eps2"], setup["kappa"], x, y, z, q,
                                     order=o)[0]
            row[f"kirk{o}"] = abs(0.5 * (k - ref))
        out.append(row)
    return out


def test_paper_claim_error_below_1e5_inside_093():
    g = _claims()
    c = next(c for c in g["claims"] if c["id"] == "cpu_run_parameters_below_1e-5")
    rows = _self_energy_errors(c["p"], c["tau"], c["F1"], c["F2"], c["r_s"], g["setup"])
    for r in rows:
        assert r["hsma"] < c["abs_err_below"], r


def test_paper_claim_tau_insensitive_at_095():
    g = _claims()
    c = next(c for c in g["claims"] if c["id"] == "fig2a_tau_insensitive_1e-4_at_0.95")
    errs = []
    for tau in c["taus"]:
        (r,) = _self_energy_errors(c["p"], tau, c["F1"], c["F2"], [c["r_s"]], g["setup"])
        errs.append(r["hsma"])
        assert r["hsma"] < c["abs_err_below"]
    # little change with tau: within one order of magnitude of each other
    assert max(errs) / min(errs) < 10.0


@pytest.mark.slow
def test_paper_claim_five_digits_needs_p55():
    g = _claims()
    c = next(c for c in g["claims"] if c["id"] == "fig3_five_digits_needs_p55")
    (fine,) = _self_energy_errors(c["p"], c["tau"], c["F1"], c["F2"], [c["r_s"]], g["setup"])
    (coarse,) = _self_energy_errors(c["coarser_p"], c["tau"], c["F1"], c["F2"], [c["r_s"]], g["setup"])
    assert fine["hsma"] / abs(fine["ref"]) < c["rel_err_below"]
    assert coarse["hsma"] > 2 * fine["hsma"]


def test_paper_claim_hsma_beats_kirkwood():
    g = _claims()
    c = next(c for c in g["claims"] if c["id"] == "fig4_hsma_vs_kirkwood")
    rows = _self_energy_errors(c["p_hsma"], c["tau"], c["F1"], c["F2"], c["r_s"], g["setup"],
                               kirk_orders=(c["p_kirkwood_worse"], c["p_kirkwood_fails"]))
    for r in rows:
        assert r["hsma"] < r[f"kirk{c['p_kirkwood_worse']}"], r
        assert r["hsma"] < c["hsma_abs_err_below"], r
    assert max(r[f"kirk{c['p_kirkwood_fails']}"] for r in rows) > c["kirkwood_fails_above"]


@pytest.mark.parametrize("dipole", [0, 2])
@pytest.mark.parametrize("eps1,eps2,kappa", [(1.0, 80.0, 0.1), (80.0, 80.0, 0.5), (2.0, 80.0, 5.0),
                                             (1.0, 78.5, 40.0)])
def test_hsma_matches_kirkwood_well_inside(eps1, eps2, kappa, dipole):
    """Sources and targets inside r < 0.55 a: the truncation error at p = 24 is ~0.3^25,
    so the HSMA and the series must agree to near rounding (a dropped term, wrong sign
    or wrong factor anywhere in the image construction would show as O(1) here).  The
    single-layer variant (dipole = 2) represents the same harmonic by another density and
    must agree just as closely."""
    a = 4.0
    rng = np.random.default_rng(3)
    n = 10
    pos = rng.standard_normal((n, 3))
    pos *= (0.55 * a * rng.random(n) ** (1 / 3) / np.linalg.norm(pos, axis=1))[:, None]
    q = rng.choice([-1.0, 1.0, 2.0], n)
    prm = oracle.Params(a=a, eps1=eps1, eps2=eps2, kappa=kappa, p=24, P=2 * 1598, M=1000, F1=987, dipole=dipole)
    h = oracle.hsma_eval(prm, pos[:, 0], pos[:, 1], pos[:, 2], q)
    k = oracle.kirkwood_eval(a, eps1, eps2, kappa, pos[:, 0], pos[:, 1], pos[:, 2], q)
    assert np.max(np.abs(h - k)) <= 1e-10 * np.max(np.abs(k))


def test_surface_images_reproduce_harmonics():
    """Green's second identity on the auxiliary sphere (eq. "GreenSecond"): for
    Phi = sum Ahat (r/a)^n Y_nm, the Fibonacci-discretised monopole + dipole layer
    reproduces Phi inside; the +-dy/2 pair of eq. "approxG" agrees to O(dy^2); the single
    layer alone (dipole = 2, the monopole integral of eq. "threeintegrals" with the density
    of the same interior harmonic) reproduces it too."""
    a = 2.0
    rng = np.random.default_rng(9)
    for dip, tol in ((0, 1e-11), (1, 1e-8), (2, 1e-11)):
        prm = oracle.Params(a=a, eps1=1.0, eps2=80.0, kappa=0.3, p=8, P=2 * 1598, M=200, F1=987, dipole=dip)
        Ah = rng.standard_normal(prm.K)
        nodes, w = oracle.fibonacci_nodes(987, 1597, (1 + prm.tau) * a)
        Q, D = oracle.surface_strengths(prm, Ah, nodes, w)
        if dip == 2:
            assert not np.any(D)
        tg = rng.standard_normal((30, 3))
        # well inside R_tau the Fibonacci rule is at rounding; near it, at its O(1e-5) level
        tg *= (0.6 * a * rng.random(30) / np.linalg.norm(tg, axis=1))[:, None]
        phi = oracle.surface_potential(prm, nodes, Q, D, tg)
        nn = np.repeat(np.arange(prm.p + 1), 2 * np.arange(prm.p + 1) + 1)
        ref = np.array([np.sum(Ah * (np.linalg.norm(t) / a) ** nn * oracle.real_sh(prm.p, t)) for t in tg])
        assert np.max(np.abs(phi - ref)) <= tol * np.max(np.abs(ref))


def test_kirkwood_truncated_converges():
    x, y, z, q = W.single_charge(0.8, 1.0)
    ref = oracle.kirkwood_eval(1.0, 2.0, 80.0, 5.0, x, y, z, q)[0]
    errs = [abs(oracle.kirkwood_eval(1.0, 2.0, 80.0, 5.0, x, y, z, q, order=o)[0] - ref) for o in (10, 20, 40, 80)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-14


def test_kirkwood_truncation_order_is_exact():
    """The truncated series (order n) holds exactly the terms 0..n of eq. "phirf" summed over m: the
    difference of orders n and n - 1 is the single term q/(4 pi eps1 a) M_n t^n P_n(c), with M_n from
    the factor function (pinned to scipy's Bessel functions elsewhere) and P_n from scipy's Legendre
    polynomials, not the oracle's recurrence; an off-by-one in the truncation gives the neighbouring
    term instead."""
    from scipy.special import eval_legendre
    a, eps1, eps2, kappa = 1.5, 2.0, 80.0, 0.7
    src = np.array([[0.3, -0.5, 0.6]])
    tgt = np.array([[-0.2, 0.7, 0.4], [0.9, 0.1, -0.3]])
    q = 1.7
    rs, rt = np.linalg.norm(src[0]), np.linalg.norm(tgt, axis=1)
    t = rt * rs / a ** 2
    c = tgt @ src[0] / (rt * rs)
    _, M = oracle.kirkwood_factor(12, eps1 / eps2, kappa * a)
    pref = q / (4 * math.pi * eps1 * a)

    def o2(order):
        return oracle.kirkwood_eval(a, eps1, eps2, kappa, src[:, 0], src[:, 1], src[:, 2], [q], targets=tgt,
                                    order=order)

    one = pref * (M[0] + M[1] * t * c)
    assert np.allclose(o2(1), one, rtol=1e-14, atol=0)
    for n in range(2, 12):
        term = pref * M[n] * t ** n * eval_legendre(n, c)
        assert np.allclose(o2(n) - o2(n - 1), term, rtol=1e-9, atol=1e-15 * abs(one).max()), n


def test_coulomb_energy_closed_forms():
    """Two charges: q1 q2 / (4 pi eps1 r); a unit square of alternating charges: four nearest
    pairs at distance 1 and two diagonal pairs at sqrt 2."""
    e = oracle.coulomb_energy(2.0, [0.0, 3.0], [0.0, 0.0], [0.0, 4.0], [1.5, -2.0])
    assert abs(e - 1.5 * -2.0 / (4 * math.pi * 2.0 * 5.0)) <= 1e-16
    xs, ys = [0.0, 1.0, 1.0, 0.0], [0.0, 0.0, 1.0, 1.0]
    e = oracle.coulomb_energy(1.0, xs, ys, [0.0] * 4, [1.0, -1.0, 1.0, -1.0])
    assert abs(e - (-4.0 + 2.0 / math.sqrt(2.0)) / (4 * math.pi)) <= 1e-15
