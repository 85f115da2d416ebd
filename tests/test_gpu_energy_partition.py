"""The energy launch's near-interface partition (FP64 energies, hsma_energy_batched with E only)
through the C ABI, against the oracle.

The energy launch places each system's ions with r > 0.995 a after its other ions, keeping their
order within each part; the Kelvin pairs whose target block holds only the first kind (all but
the pairs of two ions near the interface, and those of blocks across the split), and the check
sums over such ions, take an expanded squared distance; every other pair takes the exact
differences.  Which pairs take which form moves with the block size (128, 256 or 512 ions)
and with the split point of each system, so the batch below holds systems whose ions near the
interface are none, all, about half, exactly two blocks' worth of ions far from it, ions on the
0.995 a boundary itself, ions within 2e-6 a of the interface, and ragged small systems, in shuffled
order.  Every system's energy is held to 1e-9 of |E*| against the oracle under every block size,
and the block sizes agree with each other to 1e-12 (a pair's expanded form rounds to at most about
5e-11 of the pair, at sources on the 0.995 a boundary, and its errors do not add up coherently).
(Nearer the interface the energy is dominated by the own-image terms, ~1/(a - r), and a - r itself
carries the rounding of r relative to a - r: at 1e-9 a that is ~2e-7, beyond any 1e-9 comparison.)
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL_E = 1e-9
TOL_BLOCKS = 1e-12
NEAR = 0.995


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


def _mixed(rng, a, n_far, n_near, near_lo=NEAR, near_hi=1.0 - 1e-9, far_hi=NEAR):
    """n_far ions uniform in r <= far_hi a and n_near with r uniform in (near_lo a, near_hi a),
    in shuffled order."""
    far = W.uniform_ball(rng, n_far, a, rmax=far_hi * a)
    r = a * (near_lo + (near_hi - near_lo) * rng.random(n_near))
    near = W._directions(rng, n_near) * r[:, None]
    pos = np.concatenate([far, near])[rng.permutation(n_far + n_near)]
    return pos


def _systems(a):
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 610))
    phys = W.Physics(a, 1.0, 78.5, 0.3)
    out = {}
    out["none near"] = _mixed(rng, a, 600, 0)
    out["all near"] = _mixed(rng, a, 0, 500)
    out["half near"] = _mixed(rng, a, 450, 450)
    out["512 far"] = _mixed(rng, a, 512, 189)  # the split on a block boundary of every size
    d = W._directions(rng, 300)
    out["on 0.995 a"] = np.concatenate([d[:150] * (NEAR * a), _mixed(rng, a, 100, 50)])
    out["1e-6 a from the interface"] = _mixed(rng, a, 200, 60, near_lo=1.0 - 2e-6, near_hi=1.0 - 1e-6)
    out["one ion"] = _mixed(rng, a, 1, 0)
    out["two ions, one near"] = _mixed(rng, a, 1, 1)
    out["65 ions"] = _mixed(rng, a, 40, 25)
    systems = []
    for name, pos in out.items():
        n = len(pos)
        q = W.balanced_charges(rng, n) if n > 1 else np.array([1.0])
        pos = np.ascontiguousarray(pos)
        systems.append((name, W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, phys)))
    return systems


@pytest.fixture(scope="module")
def batch(dev):
    a = 20.0
    systems = _systems(a)
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536)
    group = hs.Group([plan])
    sizes = [s.n for _, s in systems]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    t = [torch.tensor(np.concatenate([getattr(s, k) for _, s in systems]), dtype=torch.float64, device=dev)
         for k in "xyzq"]
    offd = torch.tensor(off, dtype=torch.int64, device=dev)
    refs = []
    for name, s in systems:
        phi = oracle.hsma_eval(_oparams(plan), s.x, s.y, s.z, s.q)
        refs.append(oracle.energy(s.q, phi))
    yield {"plan": plan, "group": group, "systems": systems, "off": off, "offd": offd, "t": t, "refs": refs}
    group.close()
    plan.close()


def _energies(b, block):
    g = b["group"]
    g.set_energy_launch(block, 0)
    try:
        off = b["off"]
        E = g.energy(b["offd"], *b["t"], total_n=int(off[-1]), max_n=int(np.diff(off).max()))
        assert g.stream_check() == 0
        return E.cpu().numpy()
    finally:
        g.set_energy_launch(0, 0)


@pytest.mark.parametrize("block", [128, 256, 512])
def test_partitioned_energies_against_oracle(batch, block):
    E = _energies(batch, block)
    for (name, s), e, e_ref in zip(batch["systems"], E, batch["refs"]):
        rel = abs(e - e_ref) / abs(e_ref)
        print(f"block {block}: {name} (N={s.n}): rel {rel:.2e}", flush=True)
        assert rel <= TOL_E, (name, rel)


def test_block_sizes_agree(batch):
    Es = {blk: _energies(batch, blk) for blk in (128, 256, 512)}
    for blk in (128, 512):
        rel = np.abs(Es[blk] - Es[256]) / np.abs(Es[256])
        print(f"block {blk} vs 256: max rel {rel.max():.2e}", flush=True)
        assert rel.max() <= TOL_BLOCKS


def test_potential_call_energies_unchanged(batch, dev):
    """A call that asks for potentials as well computes the energies in the same energy launch:
    the same values as the energies alone."""
    g, off = batch["group"], batch["off"]
    phi = torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
    E = g.energy(batch["offd"], *batch["t"], total_n=int(off[-1]), max_n=int(np.diff(off).max()), phi=phi)
    assert g.stream_check() == 0
    alone = _energies(batch, 0)
    assert np.array_equal(E.cpu().numpy(), alone)


# (tau, surface form, r_c / a): the surface pairs take the expanded form when every node lies on
# R_tau >= 1.05 a (exact dipoles or a single layer), the exact differences otherwise (tau = 0.04,
# and the point-pair form); check points on the interface itself (r_c = a, the paper's placement)
# leave the expanded check sums only the ions within 0.995 a.
SURFACE_CASES = [(0.04, 0, None), (0.05, 0, None), (0.2, 0, None), (0.1, 2, None), (0.04, 2, None),
                 (0.1, 1, None), (0.1, 0, 1.0)]


@pytest.mark.parametrize("tau,dipole,rc", SURFACE_CASES)
def test_surface_and_check_forms_against_oracle(dev, tau, dipole, rc):
    a = 15.0
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 620))
    pos = _mixed(rng, a, 1100, 400)
    q = W.balanced_charges(rng, len(pos))
    kw = {"tau": tau, "dipole": dipole}
    if rc is not None:
        kw["rc_over_a"] = rc
    if dipole == 1:
        kw["dy_over_Rtau"] = 1e-5
    plan = hs.Plan(a, 1.0, 78.5, 0.3, 1024, 1536, **kw)
    i = plan.info
    prm = oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                        tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=i["dipole"],
                        dy_over_Rtau=i["dy_over_Rtau"])
    e_ref = oracle.energy(q, oracle.hsma_eval(prm, pos[:, 0], pos[:, 1], pos[:, 2], q))
    t = [torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev) for v in (pos[:, 0], pos[:, 1],
                                                                                          pos[:, 2], q)]
    E = float(plan.energy(*t).cpu()[0])
    assert plan.stream_check() == 0
    rel = abs(E - e_ref) / abs(e_ref)
    print(f"tau {tau} dipole {dipole} rc/a {i['rc'] / i['a']:.2f}: E rel {rel:.2e}", flush=True)
    assert rel <= TOL_E
    plan.close()
