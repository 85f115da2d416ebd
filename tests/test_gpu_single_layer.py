"""GPU parity of the single-layer surface variant (option dipole = 2) against the oracle built
the same way.

The variant keeps only the monopole integral of eq. "threeintegrals": the surface charges
Q'_s = w_s sigma(y_s) of the single-layer density sigma_nm = (2n+1)/R_tau (R_tau/a)^n Ahat_nm,
whose potential inside the auxiliary sphere is the same harmonic as the Green's-identity form,
and no dipoles (the oracle's pins: it reproduces harmonic polynomials and agrees with the
Kirkwood series to near rounding well inside).  Tolerances as for the default form: 1e-6
relative L2 for the compensated FP32 pairs, 1e-10 for FP64.  Cases: C1 with the fit routes of
FP32 accuracy (GEMV, FP32 MFMA, split-BF16x6), the shell system, a ragged batch through the
symmetric and the one-directional kernels in both pair precisions, the field, single-ion moves
on a resident system, and the library's dipole strengths being zero.
"""
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


def _params(plan):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=i["dipole"])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _t(v, dev):
    return torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("prec,route", [("fp32c", 1), ("fp32c", 2), ("fp32c", 4), ("fp64", 1)])
def test_c1(dev, prec, route):
    s = W.workload_c1().systems[0]
    ph = s.phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, 400, 600, pair_prec=prec, dipole=2)
    assert plan.info["dipole"] == 2
    plan.set_fit(route)
    args = [_t(v, dev) for v in (s.x, s.y, s.z, s.q)]
    phi = torch.empty(s.n, dtype=torch.float64, device=dev)
    E = plan.energy(*args, phi=phi)
    assert plan.stream_check() == 0
    _, _, Q, D = plan.intermediates(s.n, dev)
    ref, dg = oracle.hsma_eval(_params(plan), s.x, s.y, s.z, s.q, diag=True)
    got = phi.cpu().numpy()
    print(f"[{prec} route {route}] phi relL2 {_rel(got, ref):.3e}", flush=True)
    assert _rel(got, ref) <= TOL[prec]
    assert not np.any(D) and not np.any(dg["D"])
    assert _rel(Q, dg["Q"] / (4 * np.pi)) <= 1e-3
    e_ref = oracle.energy(s.q, ref)
    assert abs(float(E.cpu().numpy()[0]) - e_ref) <= 1e-9 * abs(e_ref)
    plan.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_shell_system(dev, prec):
    pos, q = W.c2_positions(N=3000)
    plan = hs.Plan(30.0, 1.0, 80.0, 0.05, 1600, 2400, pair_prec=prec, dipole=2)
    x, y, z, qq = (_t(v, dev) for v in (pos[:, 0], pos[:, 1], pos[:, 2], q))
    phi = torch.empty(3000, dtype=torch.float64, device=dev)
    plan.energy(x, y, z, qq, phi=phi)
    assert plan.stream_check() == 0
    ref = oracle.hsma_eval(_params(plan), pos[:, 0], pos[:, 1], pos[:, 2], q)
    assert _rel(phi.cpu().numpy(), ref) <= TOL[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("sym", [0, 2, 3])
def test_ragged_batch(dev, sym, prec):
    a = 25.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536, pair_prec=prec, dipole=2)
    group = hs.Group([plan])
    group.set_symmetric(sym)
    sizes = [700, 0, 1, 1537, 64, 513]
    systems = [W.small_uniform(N=n, a=a, seed=W.SEED_BASE + 420 + b) if n > 0 else None for b, n in enumerate(sizes)]
    parts = [s for s in systems if s is not None]
    cat = [np.concatenate([getattr(s, k) for s in parts]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    total = int(off_h[-1])
    assert group.eval_kernel(len(sizes), total, max(sizes)) == {0: 0, 2: 256, 3: 512}[sym]
    phi = torch.empty(total, dtype=torch.float64, device=dev)
    E = group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max(sizes), phi=phi)
    assert group.stream_check() == 0
    phi, E = phi.cpu().numpy(), E.cpu().numpy()
    prm = _params(plan)
    for b, s in enumerate(systems):
        if s is None:
            assert E[b] == 0.0
            continue
        ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
        assert _rel(phi[off_h[b]:off_h[b + 1]], ref) <= TOL[prec], (b, _rel(phi[off_h[b]:off_h[b + 1]], ref))


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_field(dev, prec):
    s = W.small_uniform(N=900, a=20.0, seed=W.SEED_BASE + 430)
    plan = hs.Plan(20.0, 1.0, 80.0, 0.5, 1024, 1536, pair_prec=prec, dipole=2)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    phi, f = plan.field(*[_t(v, dev) for v in (s.x, s.y, s.z, s.q)], E=E)
    assert plan.stream_check() == 0
    ref_phi, ref_f = oracle.hsma_field(_params(plan), s.x, s.y, s.z, s.q)
    assert _rel(f.cpu().numpy(), ref_f) <= TOL[prec]
    assert _rel(phi.cpu().numpy(), ref_phi) <= TOL[prec]
    plan.close()


def test_moves(dev):
    a = 15.0
    plan = hs.Plan(a, 1.0, 78.5, 0.5, 1024, 1536, pair_prec="fp64", dipole=2)
    prm = _params(plan)
    s = W.small_uniform(500, a, seed=W.SEED_BASE + 440)
    pos = np.stack([s.x, s.y, s.z], axis=1)
    sysm = hs.System(plan, _t(s.x, dev), _t(s.y, dev), _t(s.z, dev), _t(s.q, dev))

    def energy(p):
        return oracle.energy(s.q, oracle.hsma_eval(prm, p[:, 0], p[:, 1], p[:, 2], s.q))

    e0 = energy(pos)
    assert abs(float(sysm.energy().cpu()[0]) - e0) <= 1e-11 * abs(e0)
    rng = np.random.default_rng(37)
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


def test_groups_do_not_mix_layer_forms(dev):
    p0 = hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 600)
    p2 = hs.Plan(12.0, 1.0, 80.0, 0.1, 400, 600, dipole=2)
    with pytest.raises(RuntimeError):
        hs.Group([p0, p2])
    with pytest.raises(RuntimeError):
        hs.Plan(10.0, 1.0, 80.0, 0.1, 400, 600, dipole=3)
