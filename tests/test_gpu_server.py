"""The request server: continuous batching over resident systems.

Each result is compared with the same request run alone (the system API, requests of a
system replayed in their order): single-ion moves and full energies come out bitwise
equal, because a request's work and reduction order do not depend on its batch, nor on
the grid its full energy runs on.  Also:
admission by memory budget, invalid requests, an open-loop Poisson run, and the served
full energies against the oracle.
"""
import time

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


def _make(n_sys, seed, dev, nmin=300, nmax=1500):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_sys):
        a = float(rng.uniform(15, 40))
        kappa = float(rng.uniform(0.05, 1.0))
        plan = hs.Plan(a, 1.0, 78.5, kappa, 1024, 1536)
        s = W.small_uniform(int(rng.integers(nmin, nmax)) // 2 * 2, a, seed=seed * 100 + b)
        t = [torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq"]
        out.append((plan, s, t))
    return out


def _stream(items, n_req, seed, p_energy=0.1):
    rng = np.random.default_rng(seed)
    pos = [np.stack([s.x, s.y, s.z], axis=1).copy() for _, s, _ in items]
    reqs = []
    for _ in range(n_req):
        b = int(rng.integers(len(items)))
        if rng.random() < p_energy:
            reqs.append((hs.REQ_ENERGY, b, 0, 0, 0.0, 0.0, 0.0))
            continue
        a = items[b][0].info["a"]
        k = int(rng.integers(len(pos[b])))
        new = W.random_move(rng, pos[b][k], a)
        commit = int(rng.random() < 0.5)
        if commit:
            pos[b][k] = new
        reqs.append((hs.REQ_DELTA, b, commit, k, *new))
    return reqs, pos


def _collect(server, n, timeout=120.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in server.poll():
            got[r.tag] = r
        assert time.time() - t0 < timeout, f"{len(got)}/{n} results"
        time.sleep(0.001)
    return [got[i] for i in range(n)]


@pytest.mark.parametrize("ewg", [0, -1, 8])
def test_mix_equals_alone(dev, ewg):
    """Full energies on a limited persistent grid (0: half the compute units; 8: one workgroup per
    die) or on the whole device (-1) take the same items in the same reduction order."""
    items = _make(6, 11, dev)
    server = hs.Server(max_batch=64, energy_workgroups=ewg)
    ids = [server.add_system(p, *t) for p, _, t in items]
    assert ids == list(range(6))
    reqs, final_pos = _stream(items, 240, 5)
    server.submit(reqs)
    res = _collect(server, len(reqs))
    assert all(r.status == 0 for r in res)
    st = server.stats()
    assert st["batches"] < st["batched_requests"]  # requests were batched
    # alone: every system replays its own requests in order
    alone = [hs.System(p, *t) for p, _, t in items]
    for i, (typ, b, commit, k, x, y, z) in enumerate(reqs):
        if typ == hs.REQ_ENERGY:
            v = float(alone[b].full_energy().cpu()[0])
        else:
            v = float(alone[b].delta_energy(k, (x, y, z)).cpu()[0])
            if commit:
                alone[b].commit(k, (x, y, z))
        assert res[i].value == v, (i, typ, res[i].value, v)
    # the served configurations match the oracle
    for b, (p, s, _) in enumerate(items[:2]):
        i = p.info
        prm = oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"],
                            M=i["M"], tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"])
        pos = final_pos[b]
        e_ref = oracle.energy(s.q, oracle.hsma_eval(prm, pos[:, 0], pos[:, 1], pos[:, 2], s.q))
        server.submit([(hs.REQ_ENERGY, b, 0, 0, 0.0, 0.0, 0.0)])
        (r,) = _collect(server, 1)
        assert abs(r.value - e_ref) <= 1e-11 * abs(e_ref)
    for s in alone:
        s.close()
    server.close()


def test_admission_by_memory(dev):
    """Each system's resident state counts against the budget, and so do the full-energy
    workspaces, which are shared and sized by the largest system admitted."""
    items = _make(3, 21, dev, 1000, 1001)
    probe = hs.Server()
    probe.add_system(items[0][0], *items[0][2])
    one = probe.stats()["memory_used"]
    probe.add_system(items[1][0], *items[1][2])
    per = probe.stats()["memory_used"] - one      # one more system of the same size
    shared = one - per                            # the workspaces
    probe.close()
    assert per > 0 and shared > 0
    server = hs.Server(memory_budget=int(shared + 2.5 * per))
    a = server.add_system(items[0][0], *items[0][2])
    server.add_system(items[1][0], *items[1][2])
    with pytest.raises(hs.HsmaError) as ei:
        server.add_system(items[2][0], *items[2][2])
    assert ei.value.code == 4  # HSMA_EBUSY
    server.remove_system(a)
    assert server.add_system(items[2][0], *items[2][2]) == a  # the freed id is reused
    server.close()


def test_invalid_requests(dev):
    items = _make(1, 31, dev)
    server = hs.Server()
    server.add_system(items[0][0], *items[0][2])
    a = items[0][0].info["a"]
    bad = [(hs.REQ_DELTA, 0, 0, 10 ** 6, 0.0, 0.0, 0.0), (hs.REQ_DELTA, 5, 0, 0, 0.0, 0.0, 0.0),
           (hs.REQ_DELTA, 0, 0, 0, a, 0.0, 0.0), (7, 0, 0, 0, 0.0, 0.0, 0.0)]
    server.submit(bad)
    res = _collect(server, len(bad))
    assert all(r.status == 1 for r in res)
    server.close()


def test_open_loop_poisson(dev):
    items = _make(4, 41, dev)
    server = hs.Server(max_batch=128)
    for p, _, t in items:
        server.add_system(p, *t)
    reqs, _ = _stream(items, 400, 9)
    rng = np.random.default_rng(3)
    arrival = np.cumsum(rng.exponential(1.0 / 20000.0, len(reqs)))
    res = server.run_load(reqs, arrival)
    assert all(r.status == 0 for r in res)
    sub = np.array([r.t_submit for r in res])
    done = np.array([r.t_done for r in res])
    assert np.all(done >= sub)
    assert np.all(np.abs(sub - arrival) < 5e-3)
    # per system: committed moves and full energies start in their order, and moves complete
    # in theirs (a query may pass a waiting full energy, and a full energy runs on a copy of the
    # state, so it may complete after later moves)
    for b in range(4):
        st = [r.t_start for r, q in zip(res, reqs) if q[1] == b and (q[0] == hs.REQ_ENERGY or q[2])]
        assert all(x <= y for x, y in zip(st, st[1:]))
        d = [r.t_done for r, q in zip(res, reqs) if q[1] == b and q[0] == hs.REQ_DELTA]
        assert all(x <= y for x, y in zip(d, d[1:]))
    server.close()
