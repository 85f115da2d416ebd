"""GPU parity of the symmetric Kelvin kernels (compensated FP32 and FP64 pairs) through the C ABI.

The kernel computes each ion pair's reciprocal image distance once and uses it for both ions,
through the identity |x_j - r_K,i| = (r_j / r_i) |x_i - r_K,j| of the modified Kelvin images
(Sec. 2.4).  It runs on blocks of 256 or 512 ions with one-directional diagonal blocks and
surface chunks, so the cases are chosen around those edges: systems of 1, 2, 63-65, 255-257,
511-513 and 1300 ions, an ion at the exact centre (image at infinity), ions within 1e-9 a of
the interface and an uneven batch, with either block size forced on, in compensated FP32 and in
FP64 pairs (k_kelvin_sym64).  Each is compared with the FP64 oracle (1e-6 relative L2 for FP32
pairs, 1e-10 for FP64) and with the one-directional kernel of the library (1e-6 / 1e-12).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1907_01724_amd as hs  # noqa: E402

TOL = {"fp32c": 1e-6, "fp64": 1e-10}       # against the oracle
TOL_ONE = {"fp32c": 1e-6, "fp64": 1e-12}   # against the one-directional kernel


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hs.load_library()
    return torch.device("cuda:0")


def _params(plan):
    i = plan.info
    return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"], M=i["M"],
                         tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(plan, s, dev, block):
    plan.set_symmetric({0: 0, 256: 2, 512: 3}[block])
    assert plan.eval_kernel(s.n) == (block if s.n > 0 else 0)
    x, y, z, q = (torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    phi = torch.empty(s.n, dtype=torch.float64, device=dev)
    E = plan.energy(x, y, z, q, phi=phi)
    assert plan.stream_check() == 0
    return phi.cpu().numpy(), float(E.cpu().numpy()[0])


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("block", [256, 512])
@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 255, 256, 257, 511, 512, 513, 1300])
def test_block_edges(dev, N, block, prec):
    s = W.small_uniform(N=N, a=10.0, seed=W.SEED_BASE + 300 + N)
    plan = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, 400, 600, pair_prec=prec)
    phi_s, e_s = _run(plan, s, dev, block)
    phi_o, e_o = _run(plan, s, dev, 0)
    ref = oracle.hsma_eval(_params(plan), s.x, s.y, s.z, s.q)
    e_ref = oracle.energy(s.q, ref)
    assert _rel(phi_s, ref) <= TOL[prec], (N, _rel(phi_s, ref))
    assert _rel(phi_s, phi_o) <= TOL_ONE[prec]
    assert abs(e_s - e_ref) <= 1e-9 * abs(e_ref)  # every energy comes from FP64 pairs


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("block", [256, 512])
def test_centre_and_interface_ions(dev, block, prec):
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 310))
    a = 30.0
    N = 1200
    pos = W.uniform_ball(rng, N, a)
    pos[0] = (0.0, 0.0, 0.0)  # image at infinity
    for k in range(1, 9):    # ions just inside the interface
        d = rng.standard_normal(3)
        pos[k] = d / np.linalg.norm(d) * a * (1.0 - 1e-9 * k)
    q = W.balanced_charges(rng, N)
    s = W.System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, W.Physics(a, 1.0, 80.0, 0.5))
    plan = hs.Plan(a, 1.0, 80.0, 0.5, 1600, 2400, pair_prec=prec)
    phi_s, _ = _run(plan, s, dev, block)
    phi_o, _ = _run(plan, s, dev, 0)
    ref = oracle.hsma_eval(_params(plan), s.x, s.y, s.z, s.q)
    delta = a - float(np.max(np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2)))
    tol = max(TOL[prec], 1e-15 * a / delta)
    assert _rel(phi_s, ref) <= tol
    assert _rel(phi_s, phi_o) <= max(TOL_ONE[prec], 1e-15 * a / delta)
    assert math.isfinite(phi_s[0])


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("block", [256, 512])
def test_uneven_batch(dev, block, prec):
    sizes = [700, 1, 1537, 64, 0, 2049, 513]
    systems = [W.small_uniform(N=n, a=25.0, seed=W.SEED_BASE + 320 + k) if n > 0 else None
               for k, n in enumerate(sizes)]
    plan = hs.Plan(25.0, 1.0, 78.5, 0.3, 1024, 1536, pair_prec=prec)
    group = hs.Group([plan])
    parts = [s for s in systems if s is not None]
    cat = [np.concatenate([getattr(s, k) for s in parts]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    total, max_n = int(off_h[-1]), int(max(sizes))
    out = {}
    for sym in (block, 0):
        group.set_symmetric({0: 0, 256: 2, 512: 3}[sym])
        assert group.eval_kernel(len(sizes), total, max_n) == sym
        phi = torch.empty(total, dtype=torch.float64, device=dev)
        E = group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi)
        assert group.stream_check() == 0
        out[sym] = (phi.cpu().numpy(), E.cpu().numpy())
    prm = _params(plan)
    for b, s in enumerate(systems):
        if s is None:
            assert out[block][1][b] == 0.0
            continue
        lo, hi = off_h[b], off_h[b + 1]
        ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
        assert _rel(out[block][0][lo:hi], ref) <= TOL[prec], (b, _rel(out[block][0][lo:hi], ref))
        assert _rel(out[block][0][lo:hi], out[0][0][lo:hi]) <= TOL_ONE[prec]


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("block", [256, 512])
def test_item_orders_are_bit_identical(dev, block, prec):
    """The two item orders of the symmetric kernel (each system's surface items after its own
    block pairs, or all block pairs first) compute the same sums into the same slots, so the
    potentials and energies agree bit for bit; the batch has empty, single-block and ragged
    systems so that the two item -> system maps differ everywhere."""
    sizes = [1300, 0, 1, 700, 513, 0, 2049, 64]
    systems = [W.small_uniform(N=n, a=25.0, seed=W.SEED_BASE + 325 + k) if n > 0 else None
               for k, n in enumerate(sizes)]
    plan = hs.Plan(25.0, 1.0, 78.5, 0.3, 1024, 1536, pair_prec=prec)
    group = hs.Group([plan])
    group.set_symmetric({256: 2, 512: 3}[block])
    parts = [s for s in systems if s is not None]
    cat = [np.concatenate([getattr(s, k) for s in parts]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    total, max_n = int(off_h[-1]), int(max(sizes))
    assert group.eval_kernel(len(sizes), total, max_n) == block
    out = {}
    for order in (1, 2, 0):
        group.set_sym_order(order)
        phi = torch.empty(total, dtype=torch.float64, device=dev)
        E = group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi)
        assert group.stream_check() == 0
        out[order] = (phi.cpu().numpy(), E.cpu().numpy())
    assert np.array_equal(out[1][0], out[2][0]) and np.array_equal(out[1][1], out[2][1])
    assert np.array_equal(out[0][0], out[2][0])  # a launch this small takes order 2
    prm = _params(plan)
    for b, s in enumerate(systems):
        if s is not None:
            ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
            assert _rel(out[1][0][off_h[b]:off_h[b + 1]], ref) <= TOL[prec]
    with pytest.raises(RuntimeError):
        group.set_sym_order(3)
