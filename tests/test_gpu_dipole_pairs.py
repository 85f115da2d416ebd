"""GPU parity with the paper's point-pair surface dipoles (eq. "approxG": charges -+D/dy at
R_tau -+ dy/2 along each node's normal, option dipole = 1) against the oracle built the same
way.  The pair's two potentials cancel about log10(R_tau/dy) digits, so the FP32 pair modes
are compared at dy = 1e-2 R_tau (1e-6 relative L2) and the FP64 mode at the paper's
dy = 1e-5 R_tau (1e-10).  Cases: C1 potentials and strengths, a batch of two cavities, the
field, a ragged batch through both symmetric Kelvin kernels, and single-ion moves on a resident
system.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hs.load_library()
    return torch.device("cuda:0")


def _params(plan):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=i["dipole"],
                         dy_over_Rtau=i["dy_over_Rtau"])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _t(v, dev):
    return torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("prec,dy,tol", [("fp32c", 1e-2, 1e-6), ("fp64", 1e-5, 1e-10), ("fp64", 1e-2, 1e-10)])
def test_c1_point_pairs(dev, prec, dy, tol):
    s = W.workload_c1().systems[0]
    ph = s.phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, 400, 600, pair_prec=prec, dipole=1, dy_over_Rtau=dy)
    assert plan.info["dipole"] == 1 and abs(plan.info["dy_over_Rtau"] - dy) <= 1e-18
    phi = torch.empty(s.n, dtype=torch.float64, device=dev)
    plan.energy(_t(s.x, dev), _t(s.y, dev), _t(s.z, dev), _t(s.q, dev), phi=phi)
    assert plan.stream_check() == 0
    prm = _params(plan)
    ref, dg = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, diag=True)
    got = phi.cpu().numpy()
    print(f"[{prec} dy={dy}] relL2 {_rel(got, ref):.3e}", flush=True)
    assert _rel(got, ref) <= tol
    # the strengths read back from the point-pair layout
    _, _, Q, D = plan.intermediates(s.n, dev)
    Rt = plan.info["R_tau"]
    tq = 1e-5 if prec != "fp64" else 1e-10
    assert _rel(Q, dg["Q"] / (4 * math.pi)) <= tq and _rel(D, dg["D"] / (4 * math.pi * Rt)) <= tq
    # the pair and the exact dipole differ by O(dy^2)
    exact = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, 400, 600, pair_prec=prec)
    phi2 = torch.empty(s.n, dtype=torch.float64, device=dev)
    exact.energy(_t(s.x, dev), _t(s.y, dev), _t(s.z, dev), _t(s.q, dev), phi=phi2)
    assert _rel(got, phi2.cpu().numpy()) <= max(tol, 10 * dy * dy)
    plan.close()
    exact.close()


@pytest.mark.parametrize("prec,dy,tol", [("fp32c", 1e-2, 1e-6), ("fp64", 1e-5, 1e-10)])
def test_batch_of_two_cavities_and_field(dev, prec, dy, tol):
    cav = [(15.0, 0.05), (27.0, 0.4)]
    plans = [hs.Plan(a, 1.0, 78.5, k, 1024, 1536, pair_prec=prec, dipole=1, dy_over_Rtau=dy) for a, k in cav]
    group = hs.Group(plans)
    which = [0, 1, 1, 0]
    systems = [W.small_uniform(300 + 211 * b, cav[w][0], seed=W.SEED_BASE + 400 + b) for b, w in enumerate(which)]
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    off_h = np.concatenate([[0], np.cumsum([s.n for s in systems])]).astype(np.int64)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    plan_of = torch.tensor(which, dtype=torch.int32, device=dev)
    t = [_t(v, dev) for v in cat]
    total, max_n = int(off_h[-1]), max(s.n for s in systems)
    phi, f, E = group.field(off, *t, total_n=total, max_n=max_n, plan_of=plan_of)
    assert group.stream_check() == 0
    phi, f = phi.cpu().numpy(), f.cpu().numpy()
    for b, s in enumerate(systems):
        prm = _params(plans[which[b]])
        rp, rf = oracle.hsma_field(prm, s.x, s.y, s.z, s.q)
        lo, hi = off_h[b], off_h[b + 1]
        assert _rel(phi[lo:hi], rp) <= tol, (b, _rel(phi[lo:hi], rp))
        assert _rel(f[lo:hi], rf) <= tol, (b, _rel(f[lo:hi], rf))


@pytest.mark.parametrize("prec,dy,tol", [("fp32c", 1e-2, 1e-6), ("fp64", 1e-5, 1e-10)])
@pytest.mark.parametrize("sym", [2, 3])
def test_symmetric_kernels_with_point_pairs(dev, prec, dy, tol, sym):
    """The symmetric Kelvin kernels (forced on, blocks of 256 or 512) take the 3P point charges
    of each node as their surface sources: a ragged batch over two cavities against the oracle,
    and against the one-directional kernel of the library."""
    cav = [(15.0, 0.05), (27.0, 0.4)]
    plans = [hs.Plan(a, 1.0, 78.5, k, 1024, 1536, pair_prec=prec, dipole=1, dy_over_Rtau=dy) for a, k in cav]
    group = hs.Group(plans)
    which = [0, 1, 1, 0, 1]
    sizes = [700, 1, 1300, 513, 64]
    systems = [W.small_uniform(n, cav[w][0], seed=W.SEED_BASE + 405 + b) for b, (w, n) in enumerate(zip(which, sizes))]
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    plan_of = torch.tensor(which, dtype=torch.int32, device=dev)
    t = [_t(v, dev) for v in cat]
    total, max_n = int(off_h[-1]), max(sizes)
    out = {}
    for mode in (sym, 0):
        group.set_symmetric(mode)
        assert group.eval_kernel(len(sizes), total, max_n) == {0: 0, 2: 256, 3: 512}[mode]
        phi = torch.empty(total, dtype=torch.float64, device=dev)
        group.energy(off, *t, total_n=total, max_n=max_n, plan_of=plan_of, phi=phi)
        assert group.stream_check() == 0
        out[mode] = phi.cpu().numpy()
    for b, s in enumerate(systems):
        ref = oracle.hsma_eval(_params(plans[which[b]]), s.x, s.y, s.z, s.q)
        lo, hi = off_h[b], off_h[b + 1]
        assert _rel(out[sym][lo:hi], ref) <= tol, (b, _rel(out[sym][lo:hi], ref))
        assert _rel(out[sym][lo:hi], out[0][lo:hi]) <= (1e-6 if prec == "fp32c" else 1e-12)


def test_groups_do_not_mix_dipole_forms(dev):
    p0 = hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 600)
    p1 = hs.Plan(12.0, 1.0, 80.0, 0.1, 400, 600, dipole=1)
    with pytest.raises(RuntimeError):
        hs.Group([p0, p1])
    with pytest.raises(RuntimeError):
        hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 600, dipole=1, dy_over_Rtau=0.5)


def test_moves_with_point_pairs(dev):
    a = 15.0
    plan = hs.Plan(a, 1.0, 78.5, 0.5, 1024, 1536, pair_prec="fp64", dipole=1)
    prm = _params(plan)
    s = W.small_uniform(500, a, seed=W.SEED_BASE + 410)
    pos = np.stack([s.x, s.y, s.z], axis=1)
    sysm = hs.System(plan, _t(s.x, dev), _t(s.y, dev), _t(s.z, dev), _t(s.q, dev))

    def energy(p):
        return oracle.energy(s.q, oracle.hsma_eval(prm, p[:, 0], p[:, 1], p[:, 2], s.q))

    e0 = energy(pos)
    assert abs(float(sysm.energy().cpu()[0]) - e0) <= 1e-11 * abs(e0)
    rng = np.random.default_rng(31)
    for step in range(8):
        k = int(rng.integers(500))
        new = W.random_move(rng, pos[k], a)
        dE = float(sysm.delta_energy(k, new).cpu()[0])
        moved = pos.copy()
        moved[k] = new
        ref = energy(moved) - energy(pos)
        assert abs(dE - ref) <= 1e-12 * abs(e0) + 1e-9 * abs(ref), (k, dE, ref)
        if step % 2 == 0:
            sysm.commit(k, new)
            pos = moved
    torch.cuda.synchronize()
    assert abs(float(sysm.energy().cpu()[0]) - energy(pos)) <= 1e-11 * abs(e0)
    sysm.close()
