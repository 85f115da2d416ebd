"""HSMA reaction-potential oracle (test infrastructure only).

Python view of ``hsma_oracle.c``: a plain FP64 CPU implementation of the harmonic
surface mapping algorithm (O1) and of the converged Kirkwood series (O2) of
Fu & Gan, arXiv:1907.01724.  Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark may import this module; the GPU library never
does, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsma_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhsma_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


NATIVE_FLAGS = ["-O3", "-march=native", "-std=c11", "-fopenmp", "-fPIC", "-shared"]


def build_native(path: str) -> list:
    """Compile the same source for the host it runs on (-O3 -march=native, no fast-math) into
    ``path`` (for timing the oracle as a CPU baseline); returns the flags used."""
    subprocess.check_call(["gcc", *NATIVE_FLAGS, "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", path, "-lm"])
    return list(NATIVE_FLAGS)


def use_library(path: str) -> None:
    """Load the oracle from ``path`` from now on (a build of the same source)."""
    global _lib, _LIB_PATH
    _LIB_PATH = path
    _lib = None


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("eps1", C.c_double), ("eps2", C.c_double), ("kappa", C.c_double),
                ("tau", C.c_double), ("rc_over_a", C.c_double), ("p", C.c_int), ("P", C.c_int),
                ("M", C.c_int), ("F1", C.c_int), ("dipole", C.c_int), ("dy_over_Rtau", C.c_double),
                ("check_set", C.c_int)]


class _Diag(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in
                ("u", "v", "alpha", "beta", "Ahat", "Q", "D", "nodes", "w", "checks", "kelvin")]


_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.orc_num_threads.restype = C.c_int
        L.orc_lambda.argtypes = [C.c_int, C.c_double, _DP]
        L.orc_kirkwood_factor.argtypes = [C.c_int, C.c_double, C.c_double, _DP, _DP]
        L.orc_image_constants.argtypes = [C.c_double, C.c_double, _DP]
        L.orc_real_sh.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _DP]
        L.orc_fibonacci_nodes.argtypes = [C.c_int, C.c_int, C.c_double, _DP, _DP]
        L.orc_check_lattice.argtypes = [C.c_int, C.c_double, _DP]
        L.orc_gl_nodes.argtypes = [C.c_int, _DP, _DP]
        L.orc_check_gl.argtypes = [C.c_int, C.c_double, _DP, _DP]
        L.orc_lstsq.argtypes = [C.c_int, C.c_int, _DP, C.c_int, _DP, _DP]
        L.orc_lstsq.restype = C.c_int
        P = C.POINTER(_Params)
        L.orc_check_fields.argtypes = [P, C.c_long, _DP, _DP, _DP, _DP, _DP, _DP, _DP]
        L.orc_fit_moments.argtypes = [P, _DP, _DP, _DP, _DP, _DP]
        L.orc_fit_moments.restype = C.c_int
        L.orc_correction_coeffs.argtypes = [P, _DP, _DP, _DP]
        L.orc_surface_strengths.argtypes = [P, _DP, _DP, _DP, _DP, _DP]
        L.orc_surface_potential.argtypes = [P, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP]
        L.orc_kelvin_potential.argtypes = [P, C.c_long, _DP, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP]
        L.orc_hsma_eval.argtypes = [P, C.c_long, _DP, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP,
                                    C.POINTER(_Diag)]
        L.orc_hsma_eval.restype = C.c_int
        L.orc_hsma_field.argtypes = [P, C.c_long, _DP, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP, _DP, _DP, _DP]
        L.orc_hsma_field.restype = C.c_int
        L.orc_surface_field.argtypes = [P, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP, _DP, _DP]
        L.orc_kelvin_field.argtypes = [P, C.c_long, _DP, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, _DP, _DP, _DP]
        L.orc_kirkwood_eval.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_long,
                                        _DP, _DP, _DP, _DP, C.c_long, _DP, _DP, _DP, C.c_int, C.c_int,
                                        C.c_double, _DP, _DP]
        L.orc_kirkwood_eval.restype = C.c_int
        L.orc_coulomb_energy.argtypes = [C.c_double, C.c_long, _DP, _DP, _DP, _DP]
        L.orc_coulomb_energy.restype = C.c_double
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


@dataclass
class Params:
    """Physics + discretisation of one HSMA evaluation."""
    a: float
    eps1: float
    eps2: float
    kappa: float
    p: int
    P: int
    M: int
    tau: float = 0.1
    rc_over_a: float = 1.1
    F1: int | None = None
    dipole: int = 0  # 0 exact normal dipoles, 1 the +-dy/2 point pairs, 2 a single layer (monopoles only)
    dy_over_Rtau: float = 1e-5
    check_set: int = 0  # 0 golden-angle lattice, 1 the Gauss-Legendre grid, 2p x (2p + 1) (M = 2p (2p + 1))

    @property
    def K(self) -> int:
        return (self.p + 1) ** 2

    @property
    def F2(self) -> int:
        return self.P // 2 - 1

    def f1(self) -> int:
        return fibonacci_f1(self.F2) if self.F1 is None else int(self.F1)

    def c(self) -> _Params:
        return _Params(self.a, self.eps1, self.eps2, self.kappa, self.tau, self.rc_over_a, self.p, self.P,
                       self.M, self.f1(), self.dipole, self.dy_over_Rtau, self.check_set)


def fibonacci_f1(F2: int) -> int:
    """F1 for the Fibonacci rule: round(F2 / golden ratio), moved to the nearest value
    coprime to F2 (for consecutive Fibonacci numbers this is the predecessor)."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    base = int(round(F2 / g))
    for d in range(0, F2):
        for cand in (base - d, base + d):
            if 0 < cand < F2 and math.gcd(cand, F2) == 1:
                return cand
    return 1


def lam(nmax: int, mu: float) -> np.ndarray:
    out = np.zeros(nmax + 1)
    lib().orc_lambda(nmax, mu, _p(out))
    return out


def kirkwood_factor(nmax: int, eps: float, mu: float):
    S = np.zeros(nmax + 1)
    M = np.zeros(nmax + 1)
    lib().orc_kirkwood_factor(nmax, eps, mu, _p(S), _p(M))
    return S, M


def image_constants(eps: float, mu: float):
    out = np.zeros(3)
    lib().orc_image_constants(eps, mu, _p(out))
    return tuple(out)


def real_sh(p: int, v) -> np.ndarray:
    out = np.zeros((p + 1) ** 2)
    lib().orc_real_sh(p, float(v[0]), float(v[1]), float(v[2]), _p(out))
    return out


def fibonacci_nodes(F1: int, F2: int, R: float):
    P = 2 * (F2 + 1)
    xyz = np.zeros((P, 3))
    w = np.zeros(P)
    lib().orc_fibonacci_nodes(F1, F2, R, _p(xyz), _p(w))
    return xyz, w


def check_lattice(M: int, rc: float) -> np.ndarray:
    xyz = np.zeros((M, 3))
    lib().orc_check_lattice(M, rc, _p(xyz))
    return xyz


def gl_nodes(n: int):
    """Gauss-Legendre nodes (decreasing) and weights on [-1, 1]."""
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gl_nodes(n, _p(x), _p(w))
    return x, w


def check_gl(p: int, rc: float):
    """The check grid of Algorithm 1 step 1 (2p Gauss-Legendre nodes x 2p + 1 azimuths) on
    radius rc, and its quadrature weights on the unit sphere."""
    xyz = np.zeros((2 * p * (2 * p + 1), 3))
    wq = np.zeros(2 * p * (2 * p + 1))
    lib().orc_check_gl(p, rc, _p(xyz), _p(wq))
    return xyz, wq


def lstsq(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = _f64(A)
    B = _f64(B)
    if B.ndim == 1:
        B = B[:, None]
    m, n = A.shape
    X = np.zeros((n, B.shape[1]))
    st = lib().orc_lstsq(m, n, _p(A), B.shape[1], _p(_f64(B)), _p(X))
    if st != 0:
        raise ValueError("oracle least squares failed")
    return X


def check_fields(prm: Params, x, y, z, q, checks):
    x, y, z, q, checks = map(_f64, (x, y, z, q, checks))
    u = np.zeros(prm.M)
    v = np.zeros(prm.M)
    cp = prm.c()
    lib().orc_check_fields(C.byref(cp), len(x), _p(x), _p(y), _p(z), _p(q), _p(checks), _p(u), _p(v))
    return u, v


def fit_moments(prm: Params, checks, u, v):
    al = np.zeros(prm.K)
    be = np.zeros(prm.K)
    cp = prm.c()
    st = lib().orc_fit_moments(C.byref(cp), _p(_f64(checks)), _p(_f64(u)), _p(_f64(v)), _p(al), _p(be))
    if st != 0:
        raise ValueError("oracle fit failed")
    return al, be


def correction_coeffs(prm: Params, alpha, beta):
    Ah = np.zeros(prm.K)
    cp = prm.c()
    lib().orc_correction_coeffs(C.byref(cp), _p(_f64(alpha)), _p(_f64(beta)), _p(Ah))
    return Ah


def surface_strengths(prm: Params, Ahat, nodes, w):
    Q = np.zeros(prm.P)
    D = np.zeros(prm.P)
    cp = prm.c()
    lib().orc_surface_strengths(C.byref(cp), _p(_f64(Ahat)), _p(_f64(nodes)), _p(_f64(w)), _p(Q), _p(D))
    return Q, D


def surface_potential(prm: Params, nodes, Q, D, targets):
    t = _f64(targets)
    tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    out = np.zeros(len(tx))
    cp = prm.c()
    lib().orc_surface_potential(C.byref(cp), _p(_f64(nodes)), _p(_f64(Q)), _p(_f64(D)), len(tx),
                                _p(tx), _p(ty), _p(tz), _p(out))
    return out


def surface_field(prm: Params, nodes, Q, D, targets):
    """Field -grad of the surface images' potential at ``targets`` (nt, 3)."""
    t = _f64(targets)
    tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    ex, ey, ez = np.zeros(len(tx)), np.zeros(len(tx)), np.zeros(len(tx))
    cp = prm.c()
    lib().orc_surface_field(C.byref(cp), _p(_f64(nodes)), _p(_f64(Q)), _p(_f64(D)), len(tx), _p(tx), _p(ty), _p(tz),
                            _p(ex), _p(ey), _p(ez))
    return np.stack([ex, ey, ez], axis=1)


def kelvin_potential(prm: Params, x, y, z, q, targets):
    x, y, z, q = map(_f64, (x, y, z, q))
    t = _f64(targets)
    tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    out = np.zeros(len(tx))
    cp = prm.c()
    lib().orc_kelvin_potential(C.byref(cp), len(x), _p(x), _p(y), _p(z), _p(q), len(tx), _p(tx), _p(ty),
                               _p(tz), _p(out))
    return out


def kelvin_field(prm: Params, x, y, z, q, targets):
    """Field of the Kelvin images of the ions (x, y, z, q) at ``targets`` (nt, 3)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    t = _f64(targets)
    tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    ex, ey, ez = np.zeros(len(tx)), np.zeros(len(tx)), np.zeros(len(tx))
    cp = prm.c()
    lib().orc_kelvin_field(C.byref(cp), len(x), _p(x), _p(y), _p(z), _p(q), len(tx), _p(tx), _p(ty), _p(tz),
                           _p(ex), _p(ey), _p(ez))
    return np.stack([ex, ey, ez], axis=1)


def hsma_eval(prm: Params, x, y, z, q, targets=None, diag: bool = False):
    """O1 reaction potential at ``targets`` (default: at the ions themselves)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    if targets is None:
        tx, ty, tz = x, y, z
    else:
        t = _f64(targets)
        tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    nt = len(tx)
    phi = np.zeros(nt)
    d = None
    dg = None
    if diag:
        d = {"u": np.zeros(prm.M), "v": np.zeros(prm.M), "alpha": np.zeros(prm.K), "beta": np.zeros(prm.K),
             "Ahat": np.zeros(prm.K), "Q": np.zeros(prm.P), "D": np.zeros(prm.P),
             "nodes": np.zeros((prm.P, 3)), "w": np.zeros(prm.P), "checks": np.zeros((prm.M, 3)),
             "kelvin": np.zeros(nt)}
        dg = _Diag(*[_p(d[k]) for k in ("u", "v", "alpha", "beta", "Ahat", "Q", "D", "nodes", "w", "checks",
                                         "kelvin")])
    cp = prm.c()
    st = lib().orc_hsma_eval(C.byref(cp), len(x), _p(x), _p(y), _p(z), _p(q), nt, _p(tx), _p(ty), _p(tz),
                             _p(phi), C.byref(dg) if dg is not None else None)
    if st != 0:
        raise ValueError(f"oracle HSMA failed with status {st}")
    return (phi, d) if diag else phi


def hsma_field(prm: Params, x, y, z, q, targets=None):
    """O1 reaction potential and field E = -grad Phi_RF at ``targets`` (default: at the ions),
    every image held fixed (Algorithm 1, step 5).  Returns (phi, E) with E of shape (nt, 3)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    if targets is None:
        tx, ty, tz = x, y, z
    else:
        t = _f64(targets)
        tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    nt = len(tx)
    phi = np.zeros(nt)
    ex, ey, ez = np.zeros(nt), np.zeros(nt), np.zeros(nt)
    cp = prm.c()
    st = lib().orc_hsma_field(C.byref(cp), len(x), _p(x), _p(y), _p(z), _p(q), nt, _p(tx), _p(ty), _p(tz),
                              _p(phi), _p(ex), _p(ey), _p(ez))
    if st != 0:
        raise ValueError(f"oracle HSMA field failed with status {st}")
    return phi, np.stack([ex, ey, ez], axis=1)


def kirkwood_eval(a, eps1, eps2, kappa, x, y, z, q, targets=None, order: int = 0, nmax: int = 200000,
                  tol: float = 1e-17, return_tail: bool = False):
    """O2 reaction potential (Kirkwood series) at ``targets`` (default: at the ions)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    if targets is None:
        tx, ty, tz = x, y, z
    else:
        t = _f64(targets)
        tx, ty, tz = (_f64(t[:, k]) for k in range(3))
    phi = np.zeros(len(tx))
    tail = C.c_double(0.0)
    st = lib().orc_kirkwood_eval(a, eps1, eps2, kappa, len(x), _p(x), _p(y), _p(z), _p(q), len(tx), _p(tx),
                                 _p(ty), _p(tz), int(order), int(nmax), float(tol), _p(phi), C.byref(tail))
    if st != 0:
        raise ValueError("oracle Kirkwood failed")
    return (phi, tail.value) if return_tail else phi


def coulomb_energy(eps1: float, x, y, z, q) -> float:
    """Direct Coulomb energy (1/2) sum_{i != j} q_i q_j / (4 pi eps1 |x_i - x_j|)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    return float(lib().orc_coulomb_energy(float(eps1), len(x), _p(x), _p(y), _p(z), _p(q)))


def energy(q, phi) -> float:
    """E = (1/2) sum_i q_i Phi_i: the self-energy definition of Sec. 4.1 for N ions."""
    return 0.5 * float(np.dot(_f64(q), _f64(phi)))
