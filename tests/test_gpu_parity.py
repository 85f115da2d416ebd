"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: potentials within 1e-6 relative L2 of the oracle for the FP32 pair modes and
1e-10 for the FP64 mode.  Energies, in every pair precision of the plan: |E - E*| <= 1e-9 |E*|
(the energy target).  An energy is always summed from FP64 pairs (the energy-only launch),
so the plan's pair precision only sets the potentials; measured errors are 1e-16 to 1e-15.
Inputs are the seeded synthetic workloads of workloads.py.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL_PHI = {"fp32": 1e-6, "fp32c": 1e-6, "fp64": 1e-10}
TOL_E = 1e-9  # relative to |E*|, every pair precision


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hs.load_library()  # must be built: never skipped, never emulated
    return torch.device("cuda:0")


def _dev(arrs, dev):
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev) for a in arrs]


def _oracle_params(plan, dipole=0):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=dipole)


def _run(plan, s, dev):
    x, y, z, q = _dev((s.x, s.y, s.z, s.q), dev)
    E_only = plan.energy(x, y, z, q)  # the energy alone runs the same FP64 launch as with phi
    assert plan.stream_check() == 0
    phi = torch.empty(s.n, dtype=torch.float64, device=dev)
    E = plan.energy(x, y, z, q, phi=phi)  # the potential launch runs last: intermediates are its own
    assert plan.stream_check() == 0
    assert float(E_only.cpu()[0]) == float(E.cpu()[0])
    return phi.cpu().numpy(), float(E.cpu().numpy()[0])


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_plan_constants_match_oracle(dev):
    for (e1, e2, k) in [(1.0, 80.0, 0.1), (80.0, 80.0, 0.5), (2.0, 80.0, 5.0), (1.0, 78.5, 0.0)]:
        plan = hs.Plan(10.0, e1, e2, k, 400, 600)
        g, s, d = oracle.image_constants(e1 / e2, k * 10.0)
        inf = plan.info
        assert abs(inf["gamma"] - g) <= 1e-15 and abs(inf["sigma"] - s) <= 1e-14 * abs(s)
        assert abs(inf["dbar"] - d) <= 1e-14 * max(1.0, abs(d))
        assert inf["p"] == 10 and inf["K"] == 121 and inf["F2"] == 199
        assert inf["F1"] == oracle.fibonacci_f1(199)
        plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp32c", "fp64"])
def test_small_system_parity(dev, prec):
    wl = W.workload_c1()
    s, d, ph = wl.systems[0], wl.disc, wl.systems[0].phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, d.P, d.M, pair_prec=prec)
    phi, E = _run(plan, s, dev)
    ref, dg = oracle.hsma_eval(_oracle_params(plan), s.x, s.y, s.z, s.q, diag=True)
    e_ref = oracle.energy(s.q, ref)
    print(f"[{prec}] N={s.n} relL2={_rel_l2(phi, ref):.3e} relE={abs(E - e_ref) / abs(e_ref):.3e}")
    assert _rel_l2(phi, ref) <= TOL_PHI[prec]
    assert abs(E - e_ref) <= TOL_E * abs(e_ref)
    # intermediates: check fields and surface strengths
    u, v, Q, D = plan.intermediates(s.n, dev)
    tol = 1e-6 if prec != "fp64" else 1e-11
    assert _rel_l2(u, dg["u"]) <= tol and _rel_l2(v, dg["v"]) <= tol
    Rt = plan.info["R_tau"]
    assert _rel_l2(Q, dg["Q"] / (4 * math.pi)) <= 10 * tol
    assert _rel_l2(D, dg["D"] / (4 * math.pi * Rt)) <= 10 * tol
    plan.close()


@pytest.mark.parametrize("params", W.C2_PARAMS)
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_shell_system_parity(dev, params, prec):
    """N = 20000 with 30% of the ions within 1/2 of the interface (a = 30), P = 1600, M = 2400."""
    wl = W.workload_c2()
    idx = W.C2_PARAMS.index(params)
    s, d, ph = wl.systems[idx], wl.disc, wl.systems[idx].phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, d.P, d.M, pair_prec=prec)
    phi, E = _run(plan, s, dev)
    ref = oracle.hsma_eval(_oracle_params(plan), s.x, s.y, s.z, s.q)
    e_ref = oracle.energy(s.q, ref)
    print(f"[{prec} {params}] relL2={_rel_l2(phi, ref):.3e} relE={abs(E - e_ref) / abs(e_ref):.3e}")
    assert _rel_l2(phi, ref) <= TOL_PHI[prec]
    assert abs(E - e_ref) <= TOL_E * abs(e_ref)
    plan.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_edge_cases(dev, prec):
    a = 7.0
    plan = hs.Plan(a, 1.0, 80.0, 0.3, 400, 600, pair_prec=prec)
    prm = _oracle_params(plan)
    tol = TOL_PHI[prec]
    # empty system: zero energy
    e0 = torch.full((1,), 123.0, dtype=torch.float64, device=dev)
    empty = torch.empty(0, dtype=torch.float64, device=dev)
    plan.energy(empty, empty, empty, empty, E=e0)
    assert plan.stream_check() == 0 and float(e0.cpu()[0]) == 0.0
    # one ion at the centre: closed form q/(4 pi a)[1/(eps2 (1 + kappa a)) - 1/eps1]
    z1 = np.zeros(1)
    phi, _ = _run(plan, W.System(z1, z1, z1, np.ones(1), None), dev)
    closed = 1.0 / (4 * math.pi * a) * (1.0 / (80.0 * (1 + 0.3 * a)) - 1.0)
    assert abs(phi[0] - closed) <= 1e-6 * abs(closed)
    # one ion very close to the interface, and ragged sizes spanning several tiles
    for N in (1, 2, 33, 257, 1000, 3001):
        s = W.small_uniform(N, a, seed=N)
        if N == 1:
            s.x[:] = a * (1 - 1e-7)
            s.y[:] = 0.0
            s.z[:] = 0.0
        if N == 1000:
            s.x[7] = s.y[7] = s.z[7] = 0.0          # an ion exactly at the centre
            s.q[100:200] = 0.0                      # neutral ions
        phi, E = _run(plan, s, dev)
        ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
        # the oracle forms |x - r_K| by subtracting coordinates: for an ion at distance
        # delta from the interface that difference carries ~1e-16 a / delta relative error
        delta = a - np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2).max()
        tol_n = max(tol, 1e-15 * a / delta)
        assert _rel_l2(phi, ref) <= tol_n, (N, _rel_l2(phi, ref))
        e_ref = oracle.energy(s.q, ref)
        assert abs(E - e_ref) <= max(TOL_E, 1e-15 * a / delta) * abs(e_ref), (N, E, e_ref)
    plan.close()


def test_domain_flag(dev):
    plan = hs.Plan(5.0, 1.0, 80.0, 0.3, 400, 600)
    s = W.small_uniform(64, 5.0, seed=3)
    s.x[10] = 5.5  # outside the cavity
    x, y, z, q = _dev((s.x, s.y, s.z, s.q), dev)
    plan.potential(x, y, z, q)
    assert plan.stream_check() == 2
    s.x[10] = 1.0
    x, y, z, q = _dev((s.x, s.y, s.z, s.q), dev)
    plan.potential(x, y, z, q)
    assert plan.stream_check() == 0
    plan.close()


def test_deterministic_and_stream(dev):
    wl = W.workload_c1()
    s, d, ph = wl.systems[0], wl.disc, wl.systems[0].phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, d.P, d.M)
    x, y, z, q = _dev((s.x, s.y, s.z, s.q), dev)
    a1 = plan.potential(x, y, z, q).cpu().numpy()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a2 = plan.potential(x, y, z, q, stream=st)
    st.synchronize()
    assert np.array_equal(a1, a2.cpu().numpy())
    plan.close()


def test_invalid_arguments(dev):
    for args in [(0.0, 1, 80, 0.1, 400, 600), (10.0, -1, 80, 0.1, 400, 600), (10.0, 1, 80, -0.1, 400, 600),
                 (10.0, 1, 80, 0.1, 401, 600), (10.0, 1, 80, 0.1, 400, 100), (float("nan"), 1, 80, 0.1, 400, 600)]:
        with pytest.raises(hs.HsmaError) as ei:
            hs.Plan(*args)
        assert ei.value.code == 1
