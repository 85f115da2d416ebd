"""The expanded squared distances of the FP64 energy launch, on the CPU in exact arithmetic.

The energy launch replaces exact coordinate differences by expanded forms where they cannot
cancel badly (the kernels' comments state the bounds):
- Kelvin pairs of which one ion lies at r <= 0.995 a: D = (r_i/a)^2 (r_j/a)^2 + 1 - 2 (x_i/a).(x_j/a),
  which is |x_i - r_K,j|^2 (r_j/a)^2 / a^2 for the Kelvin point r_K,j = (a/r_j)^2 x_j (Sec. 2.4),
  is symmetric in i and j, and is at least (1 - r_i r_j / a^2)^2;
- check sums over sources at r <= 0.995 a: with w = (r/a)^2 + (rc/a)^2 and |c| = rc,
  |c - x|^2 / (a^2 w) = 1 + (c/a).(-2x/(a w));
- surface pairs with every node on one sphere R_tau >= 1.05 a: |x - y|^2 = |x|^2 + R_tau^2 - 2 x.y,
  and the dipole's (x - y).y = (|x|^2 - R_tau^2 - |x - y|^2)/2.
Here each identity is checked exactly with rationals, and each form is evaluated in FP64 in the
kernels' order of operations (every FMA rounded once, emulated exactly) against the exact value
from the same FP64 inputs, at configurations that approach each form's smallest value.
"""
import math
from fractions import Fraction as Fr

import numpy as np

NEAR = 0.995


def fma(a, b, c):
    """a b + c rounded once to FP64 (the conversion of an exact rational rounds to nearest)."""
    return float(Fr(a) * Fr(b) + Fr(c))


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _near(rng, u, spread):
    """A unit vector within about `spread` radians of u (the worst cases are nearly aligned)."""
    v = u + spread * rng.random() * _unit(rng)
    return v / np.linalg.norm(v)


def _dot(p, q):
    return sum(Fr(s) * Fr(t) for s, t in zip(p, q))


def test_kelvin_identity_is_symmetric_and_exact():
    rng = np.random.default_rng(11)
    a = Fr(37, 2)
    for _ in range(50):
        xi = [Fr(float(v)) for v in float(a) * rng.random() ** (1 / 3) * _unit(rng)]
        xj = [Fr(float(v)) for v in float(a) * rng.random() ** (1 / 3) * _unit(rng)]
        ri2, rj2 = _dot(xi, xi), _dot(xj, xj)
        D = ri2 * rj2 / a**4 + 1 - 2 * _dot(xi, xj) / a**2
        kj = [a * a / rj2 * v for v in xj]  # Kelvin point of j
        ki = [a * a / ri2 * v for v in xi]
        assert D == sum((p - q) ** 2 for p, q in zip(xi, kj)) * rj2 / a**4
        assert D == sum((p - q) ** 2 for p, q in zip(xj, ki)) * ri2 / a**4


def test_kelvin_expanded_form_rounding():
    rng = np.random.default_rng(12)
    a = 23.7
    ia = 1.0 / a
    worst = 0.0
    for t in range(900):
        # one ion within NEAR a (often just inside it), the other anywhere up to the interface
        r_far = a * NEAR * (1 - 1e-3 * rng.random()) if t % 3 else a * NEAR * rng.random() ** (1 / 3)
        r_any = a * (1 - 1e-9 * rng.random()) if t % 4 == 0 else a * (0.9 + 0.1 * rng.random()) if t % 2 \
            else a * rng.random() ** (1 / 3)
        ri, rj = (r_far, r_any) if t % 5 < 3 else (r_any, r_far)
        ui = _unit(rng)
        uj = _near(rng, ui, 0.02) if t % 5 else _unit(rng)
        xi = [float(v) for v in ri * ui]
        xj = [float(v) for v in rj * uj]
        # per-target features (in units of a) and per-source features, as the packing kernel
        tx, ty, tz = (v * ia for v in xi)
        uu = fma(tx, tx, fma(ty, ty, tz * tz))
        reff = math.sqrt(xj[0] * xj[0] + xj[1] * xj[1] + xj[2] * xj[2])
        u = (reff / a) * (reff / a)
        m = (-2.0 * xj[0] / a, -2.0 * xj[1] / a, -2.0 * xj[2] / a, u)
        d = fma(tx, m[0], fma(ty, m[1], fma(tz, m[2], fma(uu, m[3], 1.0))))
        A = Fr(a)
        D = _dot(xi, xi) * _dot(xj, xj) / A**4 + 1 - 2 * _dot(xi, xj) / A**2
        assert D >= (1 - Fr(NEAR)) ** 2 * Fr(99, 100)  # (1 - r_i r_j/a^2)^2, one of them <= NEAR a
        worst = max(worst, float(abs(Fr(d) - D) / D))
    assert worst <= 4e-11, worst


def test_check_normalised_form():
    rng = np.random.default_rng(13)
    a = 23.7
    ia = 1.0 / a
    for rc_over_a, bound in ((1.0, 6e-11), (1.1, 2e-13)):
        rc = rc_over_a * a
        worst = 0.0
        for t in range(600):
            r = a * NEAR * (1 - 1e-3 * rng.random()) if t % 2 else a * NEAR * rng.random() ** (1 / 3)
            uc = _unit(rng)
            ux = _near(rng, uc, 0.02) if t % 3 else _unit(rng)
            c = [float(v) for v in rc * uc]
            x = [float(v) for v in r * ux]
            # the exact identity, with w and the check radius exact
            C, X, A = [Fr(v) for v in c], [Fr(v) for v in x], Fr(a)
            rc2 = _dot(c, c)
            w_exact = (_dot(x, x) + rc2) / A**2
            S = sum((p - q) ** 2 for p, q in zip(C, X)) / A**2
            assert S / w_exact == 1 + _dot([v / A for v in C], [-2 * v / (A * w_exact) for v in X])
            # the packed features and the kernel's three FMAs
            r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2]
            w = r2 / (a * a) + (rc / a) * (rc / a)
            sc = -2.0 / (a * w)
            cx, cy, cz = (v * ia for v in c)
            d = fma(cx, x[0] * sc, fma(cy, x[1] * sc, fma(cz, x[2] * sc, 1.0)))
            # 1/sqrt(w) rides in the weights, so the kernel's reciprocal distance is that of d w
            assert S >= (Fr(rc_over_a) - Fr(NEAR)) ** 2 * Fr(99, 100)  # |c - x| >= rc - |x|
            worst = max(worst, float(abs(Fr(d) * Fr(w) - S) / S))
        assert worst <= bound, (rc_over_a, worst)


def test_surface_expanded_form():
    rng = np.random.default_rng(14)
    a = 23.7
    worst_d = worst_dot = 0.0
    for Rt_over_a in (1.05, 1.1, 1.5):
        Rt = Rt_over_a * a
        R2 = Rt * Rt
        for t in range(300):
            r = a * (1 - 1e-9 * rng.random()) if t % 2 else a * rng.random() ** (1 / 3)
            ux = _unit(rng)
            uy = _near(rng, ux, 0.02) if t % 3 else _unit(rng)
            x = [float(v) for v in r * ux]
            y = [float(v) for v in Rt * uy]  # a node: R_tau times a unit vector, rounded
            xx = fma(x[0], x[0], fma(x[1], x[1], x[2] * x[2]))
            f = (-2.0 * x[0], -2.0 * x[1], -2.0 * x[2], xx + R2, 0.125 * (xx - R2))
            d = fma(f[0], y[0], fma(f[1], y[1], fma(f[2], y[2], f[3])))
            dq = fma(-0.125, d, f[4])
            S = sum((Fr(p) - Fr(q)) ** 2 for p, q in zip(x, y))
            dot = _dot([Fr(p) - Fr(q) for p, q in zip(x, y)], y)
            worst_d = max(worst_d, float(abs(Fr(d) - S) / S))
            worst_dot = max(worst_dot, float(abs(Fr(dq) - dot / 4) / abs(dot / 4)))
    assert worst_d <= 1e-12, worst_d
    assert worst_dot <= 1e-12, worst_dot
