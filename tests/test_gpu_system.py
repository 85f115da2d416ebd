"""GPU parity of resident systems: single-ion-move energy changes and commits.

The reference change is E(x') - E(x) from two full FP64 oracle evaluations.  The GPU
evaluates the change from ion k's row and column of the bilinear HSMA energy in FP64, so
the two agree to FP64 rounding of the energy (tested at 1e-12 |E| + 1e-9 |dE|).
"""
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


def _oparams(plan):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"])


def _energy(prm, pos, q):
    return oracle.energy(q, oracle.hsma_eval(prm, pos[:, 0], pos[:, 1], pos[:, 2], q))


def _system(plan, s, dev):
    t = [torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq"]
    return hs.System(plan, *t)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_delta_energy_matches_oracle(dev, prec):
    a = 20.0
    plan = hs.Plan(a, 1.0, 78.5, 0.5, 1024, 1536, pair_prec=prec)
    prm = _oparams(plan)
    s = W.small_uniform(800, a, seed=77)
    s.x[5] = s.y[5] = s.z[5] = 0.0  # an ion at the centre
    pos = np.stack([s.x, s.y, s.z], axis=1)
    sysm = _system(plan, s, dev)
    e0 = _energy(prm, pos, s.q)
    got0 = float(sysm.energy().cpu()[0])
    assert abs(got0 - e0) <= 1e-11 * abs(e0)
    rng = np.random.default_rng(5)
    moves = [(int(rng.integers(800)), None) for _ in range(8)]
    moves += [(11, np.array([0.0, 0.0, 0.0])),                    # to the centre
              (5, np.array([3.0, -2.0, 1.0])),                    # from the centre
              (17, np.array([a * (1 - 1e-4), 0.0, 0.0])),         # next to the interface
              (23, pos[23] * (a * 0.999 / np.linalg.norm(pos[23])))]
    for k, new in moves:
        if new is None:
            new = W.random_move(rng, pos[k], a)
        dE = float(sysm.delta_energy(k, new).cpu()[0])
        moved = pos.copy()
        moved[k] = new
        ref = _energy(prm, moved, s.q) - e0
        assert abs(dE - ref) <= 1e-12 * abs(e0) + 1e-9 * abs(ref), (k, dE, ref)
    # the query left the state alone
    assert float(sysm.energy().cpu()[0]) == got0
    sysm.close()


def test_commits_track_the_energy(dev):
    a = 15.0
    plan = hs.Plan(a, 1.0, 78.5, 1.0, 1024, 1536)
    prm = _oparams(plan)
    s = W.small_uniform(600, a, seed=99)
    pos = np.stack([s.x, s.y, s.z], axis=1)
    sysm = _system(plan, s, dev)
    e = _energy(prm, pos, s.q)
    rng = np.random.default_rng(17)
    acc = e
    for step in range(40):
        k = int(rng.integers(600))
        new = W.random_move(rng, pos[k], a)
        dE = float(sysm.delta_energy(k, new).cpu()[0])
        if rng.random() < 0.5:
            sysm.commit(k, new)
            pos[k] = new
            acc += dE
    torch.cuda.synchronize()
    stored = float(sysm.energy().cpu()[0])
    fresh = _energy(prm, pos, s.q)
    assert abs(stored - fresh) <= 1e-11 * abs(fresh)
    assert abs(stored - acc) <= 1e-12 * abs(fresh)
    xyz = [t.cpu().numpy() for t in sysm.positions()]
    assert np.array_equal(np.stack(xyz, axis=1), pos)
    # a new system built on the moved configuration agrees with the committed one
    s2 = W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), s.q, None)
    sys2 = _system(plan, s2, dev)
    assert abs(float(sys2.energy().cpu()[0]) - stored) <= 1e-11 * abs(fresh)
    k, new = 3, W.random_move(rng, pos[3], a)
    d1 = float(sysm.delta_energy(k, new).cpu()[0])
    d2 = float(sys2.delta_energy(k, new).cpu()[0])
    assert abs(d1 - d2) <= 1e-11 * abs(fresh)
    sysm.close()
    sys2.close()


def test_invalid_moves(dev):
    a = 10.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 400, 600)
    sysm = _system(plan, W.small_uniform(50, a, seed=1), dev)
    for k, new in [(50, (0.0, 0.0, 0.0)), (-1, (0.0, 0.0, 0.0)), (3, (a, 0.0, 0.0)), (3, (float("nan"), 0, 0))]:
        with pytest.raises(hs.HsmaError) as ei:
            sysm.delta_energy(k, new)
        assert ei.value.code == 1
    sysm.close()


def test_total_energy_with_coulomb(dev):
    """HSMA_SYSTEM_COULOMB: the energy and every move's change hold the direct Coulomb energy of
    the ions too; the reference is (E_RF + E_C)(x') - (E_RF + E_C)(x) from the oracle, with
    E_C the FP64 pair sum of its definition."""
    a = 15.0
    plan = hs.Plan(a, 1.0, 78.5, 0.5, 1024, 1536, pair_prec="fp64")
    prm = _oparams(plan)
    s = W.small_uniform(700, a, seed=123)
    pos = np.stack([s.x, s.y, s.z], axis=1)
    t = [torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq"]
    sysm = hs.System(plan, *t, coulomb=True)
    plain = hs.System(plan, *t)

    def total(p):
        return _energy(prm, p, s.q) + oracle.coulomb_energy(1.0, p[:, 0], p[:, 1], p[:, 2], s.q)

    e0 = total(pos)
    assert abs(float(sysm.energy().cpu()[0]) - e0) <= 1e-11 * abs(e0)
    rng = np.random.default_rng(29)
    for step in range(12):
        k = int(rng.integers(700))
        new = W.random_move(rng, pos[k], a)
        dE = float(sysm.delta_energy(k, new).cpu()[0])
        moved = pos.copy()
        moved[k] = new
        ref = total(moved) - total(pos)
        assert abs(dE - ref) <= 1e-12 * abs(e0) + 1e-9 * abs(ref), (k, dE, ref)
        # the reaction-only system's change differs by exactly the Coulomb change
        d_rf = float(plain.delta_energy(k, new).cpu()[0])
        dc = (oracle.coulomb_energy(1.0, moved[:, 0], moved[:, 1], moved[:, 2], s.q) -
              oracle.coulomb_energy(1.0, pos[:, 0], pos[:, 1], pos[:, 2], s.q))
        assert abs((dE - d_rf) - dc) <= 1e-12 * abs(e0) + 1e-9 * abs(dc)
        if step % 2 == 0:
            sysm.commit(k, new)
            plain.commit(k, new)
            pos = moved
    torch.cuda.synchronize()
    fresh = total(pos)
    assert abs(float(sysm.energy().cpu()[0]) - fresh) <= 1e-11 * abs(fresh)
    assert abs(float(sysm.full_energy().cpu()[0]) - fresh) <= 1e-11 * abs(fresh)
    sysm.close()
    plain.close()
