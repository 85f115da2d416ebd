"""The allocation-free entry point hsma_energy_noalloc against hsma_energy (the same launches on a
caller workspace) and the oracle: two calls in a row on the library's device scratch, the second
with a smaller input, with and without potentials; a size beyond the scratch is refused."""
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


def _t(v, dev):
    return torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev)


def _oparams(plan):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"])


def test_noalloc_matches_the_workspace_entry_point(dev):
    wl = W.workload_c2()
    d = wl.disc
    big = wl.systems[1]  # N = 20000, 30% near the interface
    ph = big.phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, d.P, d.M)
    pos, q = W.c2_positions(N=3000)
    small = W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, ph)
    L = hs.load_library()
    print("workspace bytes N=20000:", plan.workspace_bytes(20000), "scratch:", 64 << 20, flush=True)
    for s in (big, small):  # the second call is smaller: the scratch keeps the first call's contents
        t = [_t(v, dev) for v in (s.x, s.y, s.z, s.q)]
        phi_a = torch.empty(s.n, dtype=torch.float64, device=dev)
        E_a = torch.empty(1, dtype=torch.float64, device=dev)
        plan.energy_noalloc(*t, phi=phi_a, E=E_a)
        assert plan.stream_check() == 0
        E_o = torch.empty(1, dtype=torch.float64, device=dev)
        plan.energy_noalloc(*t, E=E_o)  # the energy alone
        assert plan.stream_check() == 0
        phi_b = torch.empty(s.n, dtype=torch.float64, device=dev)
        E_b = plan.energy(*t, phi=phi_b)
        assert plan.stream_check() == 0
        assert torch.equal(phi_a, phi_b) and torch.equal(E_a, E_b) and torch.equal(E_o, E_b)
        ref = oracle.hsma_eval(_oparams(plan), s.x, s.y, s.z, s.q)
        e_ref = oracle.energy(s.q, ref)
        got = phi_a.cpu().numpy()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        rel_e = abs(float(E_a.cpu()[0]) - e_ref) / abs(e_ref)
        print(f"noalloc N={s.n}: phi rel L2 {rel:.2e}, E rel {rel_e:.2e}", flush=True)
        assert rel <= 1e-6 and rel_e <= 1e-9
    # the largest N the scratch holds with potentials, and a refusal beyond it
    lo, hi = 1, 1 << 22
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if plan.workspace_bytes(mid) <= (64 << 20):
            lo = mid
        else:
            hi = mid
    print("largest N for the scratch (P = 1600, M = 2400):", lo, flush=True)
    n = hi
    t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(4)]
    with pytest.raises(hs.HsmaError) as ei:
        plan.energy_noalloc(*t, E=torch.empty(1, dtype=torch.float64, device=dev))
    assert ei.value.code == 1
    plan.close()
