"""GPU parity at full size: N = 1e6 ions uniform in a = 200 (charges +-1 and +-2, 2:1), eps1 = 1,
eps2 = 80, kappa = 0.1, P = 6400, M = 9600 (p = 40), through the C ABI.

The oracle cannot evaluate all 1e6 potentials (1e12 FP64 pairs), so it evaluates 128 seeded
sampled ions against all sources, which it can do one by one: each sample's potential
includes its own image, as the library's does.  Potentials are compared within 1e-6 relative
L2 for compensated FP32 pairs with the fit applied by FP32 GEMVs, FP32 MFMA GEMMs or
split-BF16x6 MFMA GEMMs, and 1e-9 for FP64 pairs.  Split-BF16x3 (two-term BF16 splits, up to
3 * 2^-16 per product) misses 1e-6 here (3.6e-6 measured) and is held to its budget
max(1e-6, 3 * 2^-16 * A * s), with A = (r_c/a)^(p+1) (R_tau/a)^p and s the surface share of the
sampled potentials in the oracle.  The energies of the two pair precisions, which no oracle
can give at this size, must agree within 1e-6 relative (a property of both paths).
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
    for label, prec, fit in (("fp32c", "fp32c", 1), ("fp32c_mfma_fp32", "fp32c", 2),
                             ("fp32c_mfma_bf16x3", "fp32c", 3), ("fp32c_mfma_bf16x6", "fp32c", 4),
                             ("fp64", "fp64", 0)):
        plan = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=prec)
        plan.set_fit(fit)
        print(f"N=1e6 {label}: fit route {plan.fit_route()}", flush=True)
        phi = torch.empty(s.n, dtype=torch.float64, device=dev)
        E = plan.energy(x, y, z, q, phi=phi)
        assert plan.stream_check() == 0
        out[label] = (phi.cpu().numpy()[idx], float(E.cpu().numpy()[0]))
        info = plan.info
        del phi
        plan.close()
    prm = oracle.Params(a=info["a"], eps1=info["eps1"], eps2=info["eps2"], kappa=info["kappa"], p=info["p"],
                        P=info["P"], M=info["M"], tau=info["tau"], rc_over_a=info["rc"] / info["a"], F1=info["F1"])
    ref, dg = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, targets=np.stack([s.x[idx], s.y[idx], s.z[idx]], axis=1),
                               diag=True)
    share = float(np.linalg.norm(ref - dg["kelvin"]) / np.linalg.norm(ref))
    A = (info["rc"] / info["a"]) ** (info["p"] + 1) * (info["R_tau"] / info["a"]) ** info["p"]
    return out, ref, max(1e-6, 3 * 2.0 ** -16 * A * share)


@pytest.mark.parametrize("prec,tol", [("fp32c", 1e-6), ("fp32c_mfma_fp32", 1e-6), ("fp32c_mfma_bf16x3", None),
                                      ("fp32c_mfma_bf16x6", 1e-6), ("fp64", 1e-9)])
def test_sampled_potentials_match_oracle(sweep, prec, tol):
    out, ref, budget_bf16x3 = sweep
    if tol is None:
        tol = budget_bf16x3
    got = out[prec][0]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"N=1e6 {prec}: sampled relative L2 error {rel:.3e}", flush=True)
    assert rel <= tol


def test_energies_of_the_two_precisions_agree(sweep):
    out, _, _ = sweep
    e32, e64 = out["fp32c"][1], out["fp64"][1]
    assert np.isfinite(e32) and np.isfinite(e64) and e64 != 0.0
    assert abs(e32 - e64) <= 1e-6 * abs(e64)
