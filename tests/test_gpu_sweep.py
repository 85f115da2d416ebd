"""GPU parity at full size: N = 1e6 ions uniform in a = 200 (charges +-1 and +-2, 2:1), eps1 = 1,
eps2 = 80, kappa = 0.1, P = 6400, M = 9600 (p = 40), through the C ABI.

The oracle cannot evaluate all 1e6 potentials (1e12 FP64 pairs), so it evaluates 128 seeded
sampled ions against all sources, which it can do one by one: each sample's potential
includes its own image, as the library's does.  Potentials are compared within 1e-6 relative
L2 (compensated FP32 pairs) and 1e-9 (FP64 pairs).  The energies of the two precisions, which
no oracle can give at this size, must agree within 1e-6 relative (a property of both paths).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

import paper_1907_01724_amd as hs  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hs.load_library()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def sweep(dev):
    wl = W.workload_c3()
    s, d = wl.systems[0], wl.disc
    x, y, z, q = (torch.tensor(v, dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    idx = np.sort(np.random.Generator(np.random.PCG64(W.SEED_BASE + 21)).choice(s.n, 128, replace=False))
    out = {}
    for prec in ("fp32c", "fp64"):
        plan = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=prec)
        phi = torch.empty(s.n, dtype=torch.float64, device=dev)
        E = plan.energy(x, y, z, q, phi=phi)
        assert plan.stream_check() == 0
        out[prec] = (phi.cpu().numpy()[idx], float(E.cpu().numpy()[0]))
        info = plan.info
        del phi
    prm = oracle.Params(a=info["a"], eps1=info["eps1"], eps2=info["eps2"], kappa=info["kappa"], p=info["p"],
                        P=info["P"], M=info["M"], tau=info["tau"], rc_over_a=info["rc"] / info["a"], F1=info["F1"])
    ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, targets=np.stack([s.x[idx], s.y[idx], s.z[idx]], axis=1))
    return out, ref


@pytest.mark.parametrize("prec,tol", [("fp32c", 1e-6), ("fp64", 1e-9)])
def test_sampled_potentials_match_oracle(sweep, prec, tol):
    out, ref = sweep
    got = out[prec][0]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"N=1e6 {prec}: sampled relative L2 error {rel:.3e}", flush=True)
    assert rel <= tol


def test_energies_of_the_two_precisions_agree(sweep):
    out, _ = sweep
    e32, e64 = out["fp32c"][1], out["fp64"][1]
    assert np.isfinite(e32) and np.isfinite(e64) and e64 != 0.0
    assert abs(e32 - e64) <= 1e-6 * abs(e64)
