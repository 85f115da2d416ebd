"""CPU checks of the mathematics the treecode kernels rest on, written out in numpy (no GPU, no
library call): the Taylor coefficients of 1/|x - y| by their recurrence, the harmonic folding of
Cartesian moments onto the multi-indices with k_z <= 1, and the moments of a radial dipole.

* The recurrence |R|^2 a_k = ((2n-1)/n) sum_i R_i a_{k-e_i} - ((n-1)/n) sum_i a_{k-2e_i},
  a_0 = 1/|R|, gives the Taylor coefficients: sum_k a_k(R) y^k converges to 1/|R - y| for
  |y| < |R|, with the truncation error falling like (|y|/|R|)^(p+1).
* Folding: the a_k are harmonic, k! a_k = -(m+2e_x)! a_{m+2e_x} - (m+2e_y)! a_{m+2e_y} for
  k = m + 2e_z, so moving each M_k with k_z >= 2 onto those two multi-indices leaves
  sum_k a_k M_k unchanged; the reduced sum over k_z <= 1 then equals the full one for any M.
* A dipole p at y has moments sum_i p_i k_i d^(k - e_i) (d = y - c): its multipole sum equals
  p . (x - y) / |x - y|^3 to the truncation error.
"""
import math

import numpy as np
import pytest


def graded(P):
    """Multi-indices |k| <= P: degree n, then k_x descending, then k_y descending."""
    return [(x, y, n - x - y) for n in range(P + 1) for x in range(n, -1, -1) for y in range(n - x, -1, -1)]


def kidx(x, y, z):
    n = x + y + z
    return n * (n + 1) * (n + 2) // 6 + (n - x) * (n - x + 1) // 2 + (n - x - y)


def ridx(x, y, z):
    """Reduced order: degree n from n^2, k_z = 0 (k_x = n..0), then k_z = 1 (k_x = n-1..0)."""
    n = x + y + z
    return n * n + ((n - x) if z == 0 else n + 1 + (n - 1 - x))


def taylor(R, P):
    ks = graded(P)
    a = np.zeros(len(ks))
    r2 = float(R @ R)
    a[0] = 1.0 / math.sqrt(r2)
    for i, (x, y, z) in enumerate(ks[1:], 1):
        n = x + y + z
        s1 = (R[0] * a[kidx(x - 1, y, z)] if x else 0) + (R[1] * a[kidx(x, y - 1, z)] if y else 0) + \
             (R[2] * a[kidx(x, y, z - 1)] if z else 0)
        s2 = (a[kidx(x - 2, y, z)] if x >= 2 else 0) + (a[kidx(x, y - 2, z)] if y >= 2 else 0) + \
             (a[kidx(x, y, z - 2)] if z >= 2 else 0)
        a[i] = ((2 * n - 1) / n * s1 - (n - 1) / n * s2) / r2
    return ks, a


def fold(M, P):
    ks = graded(P)
    f = np.array(M, dtype=float)
    for K in range(len(ks) - 1, -1, -1):
        x, y, z = ks[K]
        if z >= 2:
            d = z * (z - 1)
            f[kidx(x + 2, y, z - 2)] -= (x + 2) * (x + 1) / d * f[K]
            f[kidx(x, y + 2, z - 2)] -= (y + 2) * (y + 1) / d * f[K]
    return f


@pytest.mark.parametrize("P", [2, 4, 6, 8])
def test_index_maps(P):
    ks = graded(P)
    assert len(ks) == (P + 1) * (P + 2) * (P + 3) // 6
    assert all(kidx(*k) == i for i, k in enumerate(ks))
    red = sorted((k for k in ks if k[2] <= 1), key=lambda k: ridx(*k))
    assert [ridx(*k) for k in red] == list(range((P + 1) ** 2))


@pytest.mark.parametrize("P", [2, 4, 6, 8])
def test_taylor_recurrence_converges(P):
    rng = np.random.default_rng(11 + P)
    R = rng.standard_normal(3)
    R *= 3.0 / np.linalg.norm(R)
    errs = []
    for scale in (0.6, 0.3):
        y = rng.standard_normal(3)
        y *= scale / np.linalg.norm(y)
        ks, a = taylor(R, P)
        approx = sum(a[i] * y[0] ** k[0] * y[1] ** k[1] * y[2] ** k[2] for i, k in enumerate(ks))
        exact = 1.0 / np.linalg.norm(R - y)
        errs.append(abs(approx - exact) / exact)
    # truncation about (|y|/|R|)^(P+1): 0.2^(P+1) and 0.1^(P+1), times a modest constant
    assert errs[0] < 4 * 0.2 ** (P + 1)
    assert errs[1] < 4 * 0.1 ** (P + 1)


@pytest.mark.parametrize("P", [2, 4, 6, 8])
def test_fold_preserves_the_multipole_sum(P):
    rng = np.random.default_rng(23 + P)
    ks = graded(P)
    for _ in range(5):
        R = rng.standard_normal(3) * 4
        _, a = taylor(R, P)
        M = rng.standard_normal(len(ks))
        f = fold(M, P)
        full = float(a @ M)
        reduced = sum(a[kidx(*k)] * f[kidx(*k)] for k in ks if k[2] <= 1)
        assert abs(reduced - full) <= 1e-12 * max(1.0, float(np.abs(a * M).sum()))
    # a moment with k_z >= 2 alone does not vanish from the sum: the fold is not a truncation
    M = np.zeros(len(ks))
    M[kidx(0, 0, 2)] = 1.0
    _, a = taylor(np.array([0.3, -0.4, 2.0]), P)
    assert abs(float(a @ M)) > 1e-3


@pytest.mark.parametrize("P", [4, 8])
def test_dipole_moments(P):
    rng = np.random.default_rng(5)
    c = np.zeros(3)
    y = rng.standard_normal(3) * 0.2
    p = rng.standard_normal(3)
    x = np.array([2.5, -1.0, 1.5])
    ks = graded(P)
    d = y - c
    M = np.zeros(len(ks))
    for i, (kx, ky, kz) in enumerate(ks):
        k = (kx, ky, kz)
        for ax in range(3):
            if k[ax]:
                e = list(k)
                e[ax] -= 1
                M[i] += p[ax] * k[ax] * d[0] ** e[0] * d[1] ** e[1] * d[2] ** e[2]
    _, a = taylor(x - c, P)
    exact = float(p @ (x - y)) / np.linalg.norm(x - y) ** 3
    ratio = np.linalg.norm(d) / np.linalg.norm(x - c)
    assert abs(float(a @ M) - exact) < 20 * ratio ** P * abs(exact) + 1e-15
