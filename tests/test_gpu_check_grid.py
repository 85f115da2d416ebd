"""GPU parity with the paper's Gauss-Legendre check grid (Algorithm 1, step 1): 2p nodes in
cos(theta) times 2p + 1 azimuths (M = 2p (2p + 1)), on r_c = 1.1 a and on the interface
r_c = a as in the paper, against the oracle built with the same grid.  Potentials within
1e-6 (compensated FP32) and 1e-10 (FP64) relative L2; the check fields within 1e-6 / 1e-11.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL = {"fp32c": 1e-6, "fp64": 1e-10}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hs.load_library()
    return torch.device("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("rc_over_a", [1.0, 1.1])
@pytest.mark.parametrize("case", ["c1", "shell_n2000"])
def test_grid_parity(dev, prec, rc_over_a, case):
    if case == "c1":
        s = W.workload_c1().systems[0]
        P = 400
    else:
        pos, q = W.c2_positions(N=2000)
        s = W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, W.Physics(30.0, 1.0, 80.0, 0.5))
        P = 1600
    ph = s.phys
    p = math.isqrt(P) // 2
    M = 2 * p * (2 * p + 1)
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, P, M, pair_prec=prec, rc_over_a=rc_over_a, check_set=1)
    info = plan.info
    assert info["check_set"] == 1 and info["p"] == p and info["M"] == M
    x, y, z, q = (torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    phi = torch.empty(s.n, dtype=torch.float64, device=dev)
    plan.energy(x, y, z, q, phi=phi)
    assert plan.stream_check() == 0
    prm = oracle.Params(a=ph.a, eps1=ph.eps1, eps2=ph.eps2, kappa=ph.kappa, p=p, P=P, M=M, rc_over_a=rc_over_a,
                        F1=info["F1"], check_set=1)
    ref, dg = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, diag=True)
    got = phi.cpu().numpy()
    print(f"[{case} rc={rc_over_a} {prec}] relL2 {_rel(got, ref):.3e}", flush=True)
    assert _rel(got, ref) <= TOL[prec]
    u, v, _, _ = plan.intermediates(s.n, dev)
    tol_uv = 1e-6 if prec != "fp64" else 1e-11
    assert _rel(u, dg["u"]) <= tol_uv and _rel(v, dg["v"]) <= tol_uv
    plan.close()


def test_grid_needs_its_point_count(dev):
    with pytest.raises(RuntimeError):
        hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 400, check_set=1)
    with pytest.raises(RuntimeError):
        hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 420, check_set=2)
    with pytest.raises(RuntimeError):
        hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 600, rc_over_a=0.99)
