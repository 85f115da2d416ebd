"""Launch settings and the timing-based tuner (hsma_group_autotune) through the C ABI.

A batch of 160 systems of the batched geometry (a = 25, eps1 = 1, eps2 = 78.5, kappa = 0.3,
P = 1024, M = 1536; sizes log-uniform in [100, 4000]) is evaluated under every value of each
launch setting (the persistent per-die item loops of the check, evaluation and symmetric
kernels included) and after tuning.  The settings only move the same sums over the device,
so results may differ from the default ones in the summation order alone:

* energies (FP64 pairs): within 1e-13 of |E|, bitwise for the energy grid (which only decides
  which wave takes an item);
* potentials (compensated FP32 pairs): within 5e-7 relative L2 (their rounding; each stays
  within the 1e-6 potential target of the oracle, checked on sampled systems).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL_E_ROUND = 1e-13
TOL_PHI_ROUND = 5e-7


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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def batch(dev):
    a = 25.0
    sizes = W.c4_sizes(160, 100, 4000, seed=W.SEED_BASE + 40)
    systems = []
    for b, n in enumerate(sizes):
        s = W.small_uniform(int(n), a, seed=W.SEED_BASE + 4000 + b)
        systems.append(s)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    t = [torch.tensor(np.concatenate([getattr(s, k) for s in systems]), dtype=torch.float64, device=dev)
         for k in "xyzq"]
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536)
    group = hs.Group([plan])
    total, max_n = int(off[-1]), int(sizes.max())
    ws = hs.workspace(group.autotune_workspace_bytes(len(sizes), total, max_n), dev)
    offd = torch.tensor(off, dtype=torch.int64, device=dev)

    def run(energy=True):
        phi = torch.empty(total, dtype=torch.float64, device=dev)
        group.potential(offd, *t, total_n=total, max_n=max_n, phi=phi, ws=ws)
        assert group.stream_check() == 0
        E = None
        if energy:
            E = group.energy(offd, *t, total_n=total, max_n=max_n, ws=ws).cpu().numpy()
            assert group.stream_check() == 0
        return phi.cpu().numpy(), E

    default = group.settings()
    ref_phi, ref_E = run()
    yield {"plan": plan, "group": group, "systems": systems, "off": off, "offd": offd, "t": t, "total": total,
           "max_n": max_n, "ws": ws, "run": run, "default": default, "ref_phi": ref_phi, "ref_E": ref_E, "dev": dev}
    group.close()
    plan.close()


CASES = [("persistent", 1), ("symmetric", 0), ("symmetric", 2), ("symmetric", 3), ("sym_order", 1),
         ("sym_order", 2), ("target_items", 4096), ("target_items", 16384), ("fit", 1), ("fit", 2), ("fit", 4),
         ("energy_block", 128), ("energy_block", 256), ("energy_block", 512), ("energy_workgroups", 8),
         ("energy_workgroups", 256)]


@pytest.mark.parametrize("field,value", CASES)
def test_setting_changes_results_only_in_rounding(batch, field, value):
    g = batch["group"]
    s = dict(batch["default"])
    s[field] = value
    g.apply_settings(s)
    try:
        phi, E = batch["run"]()
    finally:
        g.apply_settings(batch["default"])
    de = np.max(np.abs(E - batch["ref_E"]) / np.abs(batch["ref_E"]))
    dp = _rel(phi, batch["ref_phi"])
    print(f"{field}={value}: energies max rel {de:.1e}, potentials rel L2 {dp:.1e}", flush=True)
    assert dp <= TOL_PHI_ROUND
    if field == "energy_workgroups":
        assert np.array_equal(E, batch["ref_E"])
    else:
        assert de <= TOL_E_ROUND


def test_persistent_symmetric_with_every_block_size(batch):
    """The persistent form of the check, evaluation and symmetric kernels with both ion-block
    sizes and the one-directional kernel."""
    g = batch["group"]
    for sym in (0, 2, 3):
        s = dict(batch["default"], persistent=1, symmetric=sym)
        g.apply_settings(s)
        try:
            phi, _ = batch["run"](energy=False)
        finally:
            g.apply_settings(batch["default"])
        dp = _rel(phi, batch["ref_phi"])
        print(f"persistent, symmetric {sym}: potentials rel L2 {dp:.1e}", flush=True)
        assert dp <= TOL_PHI_ROUND


def test_autotune_then_cache(batch):
    g, t, dev = batch["group"], batch["t"], batch["dev"]
    total, max_n, offd, ws = batch["total"], batch["max_n"], batch["offd"], batch["ws"]
    phi = torch.empty(total, dtype=torch.float64, device=dev)
    E = torch.empty(len(batch["off"]) - 1, dtype=torch.float64, device=dev)
    r_pot = g.autotune(offd, *t, total_n=total, max_n=max_n, phi=phi, ws=ws, force=True)
    r_e = g.autotune(offd, *t, total_n=total, max_n=max_n, E=E, ws=ws, force=True)
    print(f"potentials: {r_pot}\nenergies: {r_e}", flush=True)
    assert r_pot["timed"] > 1 and not r_pot["cached"] and r_pot["ms_tuned"] <= r_pot["ms_start"]
    assert r_e["timed"] > 1 and not r_e["cached"] and r_e["ms_tuned"] <= r_e["ms_start"]
    assert r_pot["chosen"]["fit"] != 3  # never the route that can miss the potential target
    tuned = g.settings()
    phi_t, E_t = batch["run"]()
    assert _rel(phi_t, batch["ref_phi"]) <= TOL_PHI_ROUND
    assert np.max(np.abs(E_t - batch["ref_E"]) / np.abs(batch["ref_E"])) <= TOL_E_ROUND
    # the same shape again: the cached choice, nothing timed
    g.apply_settings(batch["default"])
    r2 = g.autotune(offd, *t, total_n=total, max_n=max_n, E=E, ws=ws)
    assert r2["cached"] and r2["timed"] == 0 and r2["chosen"] == r_e["chosen"]
    assert g.settings() == r_e["chosen"]
    g.apply_settings(tuned)
    # the tuned results against the oracle on sampled systems
    plan, systems, off = batch["plan"], batch["systems"], batch["off"]
    for b in (0, 57, 131):
        s = systems[b]
        ref = oracle.hsma_eval(_oparams(plan), s.x, s.y, s.z, s.q)
        e_ref = oracle.energy(s.q, ref)
        assert _rel(phi_t[off[b]:off[b + 1]], ref) <= 1e-6
        assert abs(E_t[b] - e_ref) <= 1e-9 * abs(e_ref)
    g.apply_settings(batch["default"])


def test_graph_replay_of_tuned_persistent_call(batch):
    """The persistent call captured into a HIP graph: every replay reproduces the eager result."""
    g, t, dev = batch["group"], batch["t"], batch["dev"]
    total, max_n, offd, ws = batch["total"], batch["max_n"], batch["offd"], batch["ws"]
    g.apply_settings(dict(batch["default"], persistent=1, energy_workgroups=256))
    try:
        phi = torch.empty(total, dtype=torch.float64, device=dev)
        E = torch.empty(len(batch["off"]) - 1, dtype=torch.float64, device=dev)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            g.energy(offd, *t, total_n=total, max_n=max_n, phi=phi, E=E, stream=s, ws=ws)
        s.synchronize()
        ref_phi, ref_E = phi.clone(), E.clone()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            g.energy(offd, *t, total_n=total, max_n=max_n, phi=phi, E=E, stream=s, ws=ws)
        for rep in range(3):
            phi.zero_()
            E.zero_()
            _ = (t[0] * 2.0).sum().item()  # eager work and a synchronisation between replays
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(phi, ref_phi) and torch.equal(E, ref_E), rep
    finally:
        g.apply_settings(batch["default"])


def test_invalid_settings(batch):
    g = batch["group"]
    for field, bad in (("persistent", 2), ("target_items", 10), ("symmetric", 4), ("sym_order", 3), ("fit", 5),
                       ("energy_block", 64), ("energy_workgroups", -1)):
        with pytest.raises(hs.HsmaError) as ei:
            g.apply_settings(dict(batch["default"], **{field: bad}))
        assert ei.value.code == 1
    assert g.settings() == batch["default"]
