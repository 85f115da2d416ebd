"""GPU parity of the batched path (hsma_energy_batched) against the FP64 CPU oracle.

Each system of a batch is compared with the oracle run on that system alone, and with
the library's own single-system call (the same result alone and in the mix, within the
tolerance), including empty and one-ion systems, systems of ragged sizes, several plans
(different cavities) in one group, a batch of 200 systems (the automatic fit route applies
the FP32 MFMA GEMMs to the potentials from 192 systems on) and HIP graph replay.  Energies
are held to 1e-9 of |E*| in every pair precision: they always come from FP64 pair sums.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL_PHI = {"fp32c": 1e-6, "fp64": 1e-10}
TOL_E = 1e-9  # relative to |E*|, every pair precision


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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def _batch(systems, dev):
    sizes = [s.n for s in systems]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = [np.concatenate([getattr(s, k) for s in systems]) if off[-1] > 0 else np.zeros(0) for k in "xyzq"]
    t = [torch.tensor(v, dtype=torch.float64, device=dev) for v in cat]
    return off, torch.tensor(off, dtype=torch.int64, device=dev), t


def _check_systems(group, plans_of_sys, systems, off, phi, E, prec, dev):
    for b, (pl, s) in enumerate(zip(plans_of_sys, systems)):
        got = phi[off[b]:off[b + 1]]
        if s.n == 0:
            assert E[b] == 0.0
            continue
        ref = oracle.hsma_eval(_oparams(pl), s.x, s.y, s.z, s.q)
        e_ref = oracle.energy(s.q, ref)
        print(f"  sys {b} N={s.n} relL2={_rel(got, ref):.2e} relE={abs(E[b] - e_ref) / abs(e_ref):.2e}")
        assert _rel(got, ref) <= TOL_PHI[prec], (b, s.n, _rel(got, ref))
        scale = abs(e_ref)
        assert abs(E[b] - e_ref) <= TOL_E * scale, (b, s.n, abs(E[b] - e_ref) / scale)
        # alone: the single-system entry point on the same ions
        x, y, z, q = (torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq")
        alone = torch.empty(s.n, dtype=torch.float64, device=dev)
        ea = pl.energy(x, y, z, q, phi=alone)
        assert pl.stream_check() == 0
        assert _rel(got, alone.cpu().numpy()) <= TOL_PHI[prec]
        assert abs(E[b] - float(ea.cpu()[0])) <= 2 * TOL_E * scale


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_four_parameter_sets_one_call(dev, prec):
    """The N = 20000 shell configuration under the four (eps1, eps2, kappa) sets as one batch."""
    wl = W.workload_c2()
    d = wl.disc
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=prec) for s in wl.systems]
    group = hs.Group(plans)
    off, off_d, t = _batch(wl.systems, dev)
    plan_of = torch.arange(4, dtype=torch.int32, device=dev)
    phi = torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
    E = group.energy(off_d, *t, total_n=int(off[-1]), max_n=20000, plan_of=plan_of, phi=phi)
    assert group.stream_check() == 0
    _check_systems(group, plans, wl.systems, off, phi.cpu().numpy(), E.cpu().numpy(), prec, dev)


def _uneven_systems(a, sizes, seed0):
    out = []
    for k, n in enumerate(sizes):
        s = W.small_uniform(int(n), a, seed=seed0 + k)
        out.append(s)
    return out


@pytest.mark.parametrize("prec,persistent,items", [("fp32c", False, 8192), ("fp64", False, 8192),
                                                   ("fp32c", True, 8192), ("fp32c", True, 300)])
def test_uneven_batch_shared_plan(dev, prec, persistent, items):
    """24 systems sharing a = 25, P = 1024, M = 1536 (the GEMV fit below 192 systems), ragged
    sizes; both launch shapes of the pair kernels, with few and many items per block."""
    a = 25.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536, pair_prec=prec)
    group = hs.Group([plan])
    group.tune(persistent=persistent, target_items=items)
    sizes = [0, 1, 2, 63, 64, 65, 129, 257, 300, 511, 1000, 1234, 2000, 3001, 4097, 17, 5, 700, 999, 1500, 0, 88,
             640, 2500]
    systems = _uneven_systems(a, sizes, 100)
    systems[3].x[0] = systems[3].y[0] = systems[3].z[0] = 0.0  # an ion at the centre
    off, off_d, t = _batch(systems, dev)
    phi = torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
    E = group.energy(off_d, *t, total_n=int(off[-1]), max_n=max(sizes), phi=phi)
    assert group.stream_check() == 0
    _check_systems(group, [plan] * len(systems), systems, off, phi.cpu().numpy(), E.cpu().numpy(), prec, dev)


@pytest.mark.parametrize("symmetric", [1, 2])
def test_plans_with_different_cavities(dev, symmetric):
    """One group, three cavities of different radius and screening; systems mapped by plan_of.
    Symmetric mode 1 leaves this small batch to the one-directional kernel; mode 2 forces the
    symmetric kernel, whose surface items take each system's own sphere radius R_tau."""
    cav = [(15.0, 0.05), (27.0, 0.4), (40.0, 1.0)]
    plans = [hs.Plan(a, 1.0, 78.5, k, 1024, 1536) for a, k in cav]
    group = hs.Group(plans)
    group.set_symmetric(symmetric)
    which = [0, 2, 1, 1, 0, 2, 2, 0, 1, 0]
    systems = [W.small_uniform(300 + 97 * b, cav[w][0], seed=500 + b) for b, w in enumerate(which)]
    off, off_d, t = _batch(systems, dev)
    plan_of = torch.tensor(which, dtype=torch.int32, device=dev)
    phi = torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
    E = group.energy(off_d, *t, total_n=int(off[-1]), max_n=max(s.n for s in systems), plan_of=plan_of, phi=phi)
    assert group.stream_check() == 0
    _check_systems(group, [plans[w] for w in which], systems, off, phi.cpu().numpy(), E.cpu().numpy(), "fp32c", dev)


@pytest.mark.parametrize("mode", [0, 2])
def test_graph_replay_matches_eager(dev, mode):
    """Mode 0 captures the one-directional evaluation kernel and mode 2 the symmetric Kelvin
    kernel; every replay must reproduce the eager call."""
    a = 25.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536)
    group = hs.Group([plan])
    group.set_symmetric(mode)
    systems = _uneven_systems(a, [100, 2000, 0, 513, 1500, 64, 1, 900, 3000], 900)
    off, off_d, t = _batch(systems, dev)
    n = int(off[-1])
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    E = torch.empty(len(systems), dtype=torch.float64, device=dev)
    ws = hs.workspace(group.workspace_bytes(len(systems), n, 3000), dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        group.energy(off_d, *t, total_n=n, max_n=3000, phi=phi, E=E, stream=s, ws=ws)
    s.synchronize()
    ref_phi, ref_E = phi.clone(), E.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        group.energy(off_d, *t, total_n=n, max_n=3000, phi=phi, E=E, stream=s, ws=ws)
    assert group.eval_kernel(len(systems), n, 3000) == (256 if mode == 2 else 0)
    for rep in range(4):
        phi.zero_()
        E.zero_()
        _ = (t[0] * 2.0).sum().item()  # eager work and a synchronisation between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(phi, ref_phi) and torch.equal(E, ref_E), rep


def test_inconsistent_sizes_are_refused(dev):
    """A workspace sized for other launch parameters is refused on the host; device offsets or
    plan indices that disagree with the host sizes make the call do nothing and report EINVAL."""
    a = 25.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536)
    group = hs.Group([plan])
    systems = _uneven_systems(a, [500, 700, 300], 40)
    off, off_d, t = _batch(systems, dev)
    n = int(off[-1])
    small = hs.workspace(group.workspace_bytes(3, n, 700) - 1024, dev)
    with pytest.raises(hs.HsmaError) as ei:
        group.energy(off_d, *t, total_n=n, max_n=700, ws=small)
    assert ei.value.code == 1
    # a system larger than the declared max_n
    group.energy(off_d, *t, total_n=n, max_n=600)
    assert group.stream_check() == 1
    # offsets ending short of total_n
    bad = off_d.clone()
    bad[-1] = n - 10
    group.energy(bad, *t, total_n=n, max_n=700)
    assert group.stream_check() == 1
    # a plan index outside the group
    group.energy(off_d, *t, total_n=n, max_n=700, plan_of=torch.tensor([0, 1, 0], dtype=torch.int32, device=dev))
    assert group.stream_check() == 1
    # and a consistent call afterwards is fine
    E = group.energy(off_d, *t, total_n=n, max_n=700)
    assert group.stream_check() == 0
    for b, s in enumerate(systems):
        ref = oracle.hsma_eval(_oparams(plan), s.x, s.y, s.z, s.q)
        e_ref = oracle.energy(s.q, ref)
        assert abs(float(E[b].cpu()) - e_ref) <= TOL_E * abs(e_ref)


def test_batch_of_200_systems_automatic_route(dev):
    """200 systems of the batched geometry (a = 25, eps1 = 1, eps2 = 78.5, kappa = 0.3, P = 1024,
    M = 1536; sizes log-uniform in [100, 2000], even, as the 4096-system workload draws them on
    [100, 20000]) in one call with the default settings: the potentials take the FP32 MFMA fit
    (192 systems or more), the energies the FP64 energy launch.  Every system against the oracle."""
    a = 25.0
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536)
    group = hs.Group([plan])
    assert group.fit_route(200) == 2
    sizes = W.c4_sizes(200, 100, 2000, seed=W.SEED_BASE + 30)
    systems = []
    for b, n in enumerate(sizes):
        rng = np.random.Generator(np.random.PCG64((W.SEED_BASE + 30) * 1000003 + b))
        pos = W.uniform_ball(rng, int(n), a)
        systems.append(W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), W.balanced_charges(rng, int(n)),
                                W.Physics(a, 1.0, 78.5, 0.3)))
    off, off_d, t = _batch(systems, dev)
    phi = torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
    E = group.energy(off_d, *t, total_n=int(off[-1]), max_n=int(max(sizes)), phi=phi)
    assert group.stream_check() == 0
    phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()
    worst_phi = worst_e = 0.0
    for b, s in enumerate(systems):
        ref = oracle.hsma_eval(_oparams(plan), s.x, s.y, s.z, s.q)
        e_ref = oracle.energy(s.q, ref)
        worst_phi = max(worst_phi, _rel(phi_h[off[b]:off[b + 1]], ref))
        worst_e = max(worst_e, abs(E_h[b] - e_ref) / abs(e_ref))
    print(f"200 systems: worst rel L2 {worst_phi:.2e}, worst rel E {worst_e:.2e}")
    assert worst_phi <= TOL_PHI["fp32c"]
    assert worst_e <= TOL_E
