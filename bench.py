#!/usr/bin/env python3
"""Benchmark of the HSMA reaction-potential hot path on one MI355X.

Workload (default): one ion configuration, N = 20,000 ions with 30% in the shell
r in [a - 1/2, a) of a cavity of radius a = 30, charges +-1 balanced, P = 1,600
surface nodes, M = 2,400 check points, evaluated for four parameter sets
(eps1, eps2) in {(80, 80), (1, 80)} x kappa in {0.05, 0.5}.  One step = the whole
hot path for all four parameter sets: Kelvin images, check sums, fit apply,
evaluation pair sums, potentials and FP64 energy reduction (hsma_energy).
Inputs are resident in HBM before timing starts.

Pairs per system and step = N*M (check) + N*(N-1) (Kelvin images, own image
analytic) + N*P (surface nodes).  value = pairs / time, in GPairs/s.

Prints one JSON line.  Accuracy against the FP64 CPU oracle is measured outside the
timed regions, by the cpu_baseline leg at the end, which also times the oracle on the host
cores; the other legs hand it their GPU results as plain arrays.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Derived ALU ceiling of the evaluation kernel: 256 CUs x 4 SIMDs x 16 lanes issue
# 256 * 64 FP32 lane-instructions per cycle at 2.4 GHz (78.6 TFLOP/s of FMA; packed FP32
# is not used).  Only the non-transcendental VALU instructions are counted, one issue cycle
# each; how the transcendental v_rsq_f32 overlaps with them is left out, so the peak is an
# upper bound.  One-directional Kelvin pair: 3 sub, 1 mul + 2 fma for |d|^2, 1 fma to
# accumulate = 7; surface-node pair: 3 sub, 3 for |d|^2, 3 for d.y_s, 4 for the
# monopole+dipole = 13.
CU, LANES, CLOCK = 256, 64, 2.4e9
ISSUE_RATE = CU * LANES * CLOCK              # lane-instructions / s
SLOTS_KELVIN, SLOTS_SURFACE = 7, 13
# The symmetric Kelvin kernel computes each ion pair's reciprocal image distance once for both
# ions: 3 sub, 3 for |d|^2 and one fma per direction, 8 instructions per unordered pair, i.e. 4
# per Kelvin pair counted in one direction.
SLOTS_KELVIN_SYM = 4
# Field kernel (potential and E = -grad Phi together): Kelvin pair with hi/lo coordinates 9 (d) +
# 3 (|d|^2) + 2 (strength / r, potential) + 2 (1/r^3 factor) + 3 (E); surface node 3 + 3 + 1 (1/r^2)
# + 3 (d . y) + 2 + 1 + 1 (potential) + 4 (factors) + 6 (E).  rsq not counted, as above.
SLOTS_FIELD_KELVIN, SLOTS_FIELD_SURFACE = 19, 24
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hsma_eval_c2_n20000_hbm_traffic.txt")
ENGINE_SRC = os.path.join(ROOT, "paper_1907_01724_amd", "csrc", "hsma_engine.hip")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


class OracleChecks:
    """Accuracy checks of the legs' GPU results.  A leg hands over plain data (plan parameters,
    inputs, its GPU outputs) and a function that receives the errors; the cpu_baseline leg, the
    only code in this file that runs the oracle, computes the references and calls it."""

    def __init__(self):
        self.jobs = []

    def add(self, kind: str, report, **data):
        self.jobs.append((kind, data, report))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32c", choices=["fp32", "fp32c", "fp64"])
    ap.add_argument("--no-oracle", action="store_true", help="skip the accuracy check and the CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-stage HIP events")
    ap.add_argument("--legs", default="batched,serving,sweep,field,kirkwood,accuracy,single_layer,tree",
                    help="extra workloads after the headline one: batched, serving, sweep, field, kirkwood, "
                         "accuracy, single_layer, tree (comma list, or none)")
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up steps, so that the device has left its idle "
                         "clock state when timing starts (the first steps after idle run about 8%% slower)")
    ap.add_argument("--serving-requests", type=int, default=6000)
    ap.add_argument("--serving-slots", default="1,2",
                    help="request server: concurrent single-ion-move batches and full energies")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run two device copies of 256 MiB (a known-traffic kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        return 2

    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration: 2 x (256 MiB read + 256 MiB written)")
        del src, dst
    wl = W.workload_c2()
    d = wl.disc
    systems = wl.systems
    s0 = systems[0]
    N = s0.n
    nsys = len(systems)
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec)
             for s in systems]
    group = hs.Group(plans)
    # the four parameter sets share the ion configuration: one batch of four systems
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off = torch.tensor(np.arange(nsys + 1) * N, dtype=torch.int64, device=dev)
    plan_of = torch.arange(nsys, dtype=torch.int32, device=dev)
    phi = torch.empty(nsys * N, dtype=torch.float64, device=dev)
    E = torch.empty(nsys, dtype=torch.float64, device=dev)
    ws = hs.workspace(group.workspace_bytes(nsys, nsys * N, N), dev)
    stream = torch.cuda.current_stream()
    inf = plans[0].info
    M, P = inf["M"], inf["P"]
    pairs_check = N * M
    pairs_kelvin = N * (N - 1)
    pairs_surface = N * P
    pairs_sys = pairs_check + pairs_kelvin + pairs_surface
    pairs_step = pairs_sys * nsys

    def step():
        group.energy(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of, phi=phi, E=E,
                     stream=stream, ws=ws)

    log(f"bench: workload {wl.name}, N={N}, P={P}, M={M}, p={inf['p']}, prec={args.prec}, {nsys} systems/step")
    t_settle, settle_steps = time.perf_counter(), 0
    while time.perf_counter() - t_settle < args.settle_s:
        step()
        torch.cuda.synchronize()
        settle_steps += 1
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert group.stream_check() == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    log(f"bench: {ms:.4f} ms/step over {args.steps} steps")
    stages = {}
    if not args.no_profile:
        # per-stage HIP events in a separate pass of the same steps (events cost time of their own)
        group.profile(True)
        group.profile_read()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stages = {k: list(v) for k, v in group.profile_read().items()}
        group.profile(False)

    # the plain per-system path on the same work, for comparison (not the reported value)
    x, y, z, q = xb[:N], yb[:N], zb[:N], qb[:N]
    single_ws = [hs.workspace(p.workspace_bytes(N), dev) for p in plans]
    single_phi = [torch.empty(N, dtype=torch.float64, device=dev) for _ in plans]
    single_E = [torch.empty(1, dtype=torch.float64, device=dev) for _ in plans]

    def step_single():
        for p, w, ph, e in zip(plans, single_ws, single_phi, single_E):
            p.energy(x, y, z, q, phi=ph, E=e, stream=stream, ws=w)

    for _ in range(args.warmup):
        step_single()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step_single()
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t2) * 1e3 / args.steps

    out = {
        "metric": "GPairs/s (HSMA reaction potential + energy, pairs = check + Kelvin + surface)",
        "value": pairs_step / (ms * 1e-3) / 1e9,
        "unit": "GPairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32c": "f32 pairs, f64 tile accumulation", "fp64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "single cavity a=30, N=20000 (30% in the shell [a-1/2,a)), +-1 charges, "
                               "P=1600, M=2400, p=20, 4 (eps1,eps2,kappa) sets",
                   "N": N, "P": P, "M": M, "p": inf["p"], "systems_per_step": len(plans),
                   "pair_precision": args.prec},
        "systems_per_s": nsys / (ms * 1e-3),
        "settle": {"seconds": args.settle_s, "steps": settle_steps},
        "per_system_path_ms_per_step": ms_single,
    }
    if stages:
        ev_ms, ev_n = stages["eval"]
        avg = ev_ms / max(ev_n, 1) * 1e-3               # one launch covers the whole batch
        eval_pairs = (pairs_kelvin + pairs_surface) * nsys
        sym = group.eval_kernel(nsys, nsys * N, N)
        sk = SLOTS_KELVIN_SYM if sym > 0 else SLOTS_KELVIN
        t_min = (pairs_kelvin * sk + pairs_surface * SLOTS_SURFACE) * nsys / ISSUE_RATE
        peak = eval_pairs / t_min
        achieved = eval_pairs / avg
        traffic = _measured_traffic(args.prec, "k_kelvin_sym<%d>" % (sym // 64) if sym > 0 else "k_eval<%d>" % {
            "fp32": 0, "fp32c": 1, "fp64": 2}[args.prec])
        out["roofline"] = {
            "bound": "alu",
            "kernel": ("k_kelvin_sym (symmetric Kelvin pairs in blocks of %d ions + surface chunks)" % sym if sym > 0
                       else "k_eval (evaluation pair sums)") + ", all systems of the step in one launch",
            "achieved": achieved / 1e9,
            "peak": peak / 1e9,
            "unit": "Gpair/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 256 MiB copy)",
            "algorithmic_bytes": 40 * N * nsys + 24 * P * nsys,
            "avg_launch_ms": avg * 1e3,
            "pairs_per_launch": eval_pairs,
            "peak_model": "256 CU x 64 lanes x 2.4 GHz VALU issue, one instruction per cycle; %s non-transcendental "
                          "VALU instructions per Kelvin pair, 13 per surface pair" % sk,
        }
        out["stage_ms_per_step"] = {k: v[0] / args.steps for k, v in stages.items()}

    checks = None if args.no_oracle else OracleChecks()
    if checks is not None:
        phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()

        def report_headline(r):
            out["rel_err_phi_l2_max"] = max(r["rel_phi"])
            out["rel_err_energy_max"] = max(r["rel_e"])
            out["cpu_baseline"] = {
                "value": pairs_sys * r["calls"] / r["seconds"] / 1e9,
                "unit": "GPairs/s",
                "cores": r["cores"],
                "kind": "oracle",
                "sample": f"{r['calls']} oracle evaluations (cycling over the four parameter sets) of the full "
                          f"N={N} configuration: FP64 direct check sums, Householder least squares, Kelvin and "
                          f"surface sums",
                "seconds": r["seconds"],
            }
            log(f"bench: oracle: phi rel L2 {out['rel_err_phi_l2_max']:.2e}, energy {out['rel_err_energy_max']:.2e}; "
                f"cpu_baseline {out['cpu_baseline']['value']:.2f} GPairs/s on {r['cores']} threads")

        checks.add("baseline", report_headline, infos=[p.info for p in plans],
                   systems=[(s.x, s.y, s.z, s.q) for s in systems],
                   phis=[phi_h[b * N:(b + 1) * N] for b in range(nsys)], Es=[float(e) for e in E_h],
                   min_seconds=10.0)
    legs = [l for l in args.legs.split(",") if l and l != "none"]
    if "batched" in legs:
        out["batched"] = leg_batched(args, checks)
    if "serving" in legs:
        out["serving"] = leg_serving(args)
    if "sweep" in legs:
        out["precision_sweep"] = leg_sweep(args, checks)
    if "field" in legs:
        out["field"] = leg_field(args, checks)
    if "kirkwood" in legs:
        out["kirkwood"] = leg_kirkwood(args, checks)
    if "accuracy" in legs:
        out["accuracy"] = leg_accuracy(args, checks)
    if "single_layer" in legs:
        out["single_layer"] = leg_single_layer(args, checks)
    if "tree" in legs:
        out["tree"] = leg_tree(args, checks)
    if checks is not None:
        leg_cpu_baseline(checks)
    print(json.dumps(out), flush=True)
    return 0


def _measured_traffic(prec: str, kernel: str):
    """HBM bytes per launch of the batched evaluation kernel from the committed PMC summary, or
    None when the kernel, its source (hash) or the pair precision differ from the counted run."""
    import hashlib
    try:
        kv = dict(l.split(None, 1) for l in open(TRAFFIC_FILE) if l.strip() and not l.startswith((" ", "#")))
        with open(ENGINE_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (kv.get("engine_source_sha256", "").strip() != sha or kv.get("pair_precision", "").strip() != prec
            or kv.get("kernel", "").strip() != kernel):
        return None
    return float(kv["traffic_bytes_per_launch"])


def _eval_roofline(pairs_kelvin, pairs_surface, avg_s, sym=0):
    t_min = (pairs_kelvin * (SLOTS_KELVIN_SYM if sym > 0 else SLOTS_KELVIN) + pairs_surface * SLOTS_SURFACE) / ISSUE_RATE
    pairs = pairs_kelvin + pairs_surface
    return {"bound": "alu", "achieved": pairs / avg_s / 1e9, "peak": pairs / t_min / 1e9, "unit": "Gpair/s",
            "frac": t_min / avg_s, "avg_launch_ms": avg_s * 1e3, "symmetric_block": sym}


def leg_field(args, checks) -> dict:
    """Potential, field and energy at the ions of the headline workload (N = 20000, a = 30,
    30% in the shell, P = 1600, M = 2400, the four parameter sets in one batched call):
    time per call and the field kernel against its ALU roofline; every ion's potential and field
    per system go to the oracle checks (relative L2 errors)."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c2()
    d, systems = wl.disc, wl.systems
    N, nsys = systems[0].n, len(systems)
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec)
             for s in systems]
    group = hs.Group(plans)
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off = torch.tensor(np.arange(nsys + 1) * N, dtype=torch.int64, device=dev)
    plan_of = torch.arange(nsys, dtype=torch.int32, device=dev)
    total = nsys * N

    def call():
        return group.field(off, xb, yb, zb, qb, total_n=total, max_n=N, plan_of=plan_of)

    call()
    torch.cuda.synchronize()
    assert group.stream_check() == 0
    steps = 10
    t0 = time.perf_counter()
    for _ in range(steps):
        phi, f, E = call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    group.profile(True)
    group.profile_read()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    st = group.profile_read()
    group.profile(False)
    inf = plans[0].info
    P, M = inf["P"], inf["M"]
    pk, ps = N * (N - 1) * nsys, N * P * nsys
    pairs = pk + ps + N * M * nsys
    ev = st["eval"][0] / steps * 1e-3
    t_min = (pk * SLOTS_FIELD_KELVIN + ps * SLOTS_FIELD_SURFACE) / ISSUE_RATE
    res = {"workload": "N=20000, a=30, 30% in the shell [a-1/2,a), P=1600, M=2400, p=20, 4 (eps1,eps2,kappa) sets, "
                       "potential + field + energy", "ms_per_call": ms, "gpairs_per_s": pairs / (ms * 1e-3) / 1e9,
           "stage_ms_per_call": {k: v[0] / steps for k, v in st.items()},
           "roofline": {"bound": "alu", "kernel": "k_eval_field (potential and field pair sums)",
                        "achieved": (pk + ps) / ev / 1e9, "peak": (pk + ps) / t_min / 1e9, "unit": "Gpair/s",
                        "frac": t_min / ev, "avg_launch_ms": ev * 1e3,
                        "peak_model": "%d / %d non-transcendental VALU instructions per Kelvin / surface pair" % (
                            SLOTS_FIELD_KELVIN, SLOTS_FIELD_SURFACE)}}
    if checks is not None:
        phi_h, f_h = phi.cpu().numpy(), f.cpu().numpy()

        def report(r):
            res["rel_err_phi_l2_max"] = max(r["rel_phi"])
            res["rel_err_field_l2_max"] = max(r["rel_field"])
            log(f"bench[field]: oracle: phi rel L2 {res['rel_err_phi_l2_max']:.2e}, "
                f"field rel L2 {res['rel_err_field_l2_max']:.2e}")

        checks.add("field", report, infos=[p.info for p in plans], systems=[(s.x, s.y, s.z, s.q) for s in systems],
                   phis=[phi_h[b * N:(b + 1) * N] for b in range(nsys)],
                   fields=[f_h[b * N:(b + 1) * N] for b in range(nsys)])
    for p in plans:
        p.close()
    log(f"bench[field]: {ms:.3f} ms/call, eval {ev * 1e3:.3f} ms ({res['roofline']['frac']:.2f} of its ALU peak)")
    return res


def leg_single_layer(args, checks) -> dict:
    """The headline workload (four parameter sets of N = 20000, one batched call per step) with
    the single-layer surface form (monopoles only, option dipole = 2) beside the default
    Green's-identity form: time per step, the evaluation launch, and the potentials and energies
    handed to the oracle checks (the oracle built with the same form)."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c2()
    d, systems = wl.disc, wl.systems
    N, nsys = systems[0].n, len(systems)
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off = torch.tensor(np.arange(nsys + 1) * N, dtype=torch.int64, device=dev)
    plan_of = torch.arange(nsys, dtype=torch.int32, device=dev)
    phi = torch.empty(nsys * N, dtype=torch.float64, device=dev)
    E = torch.empty(nsys, dtype=torch.float64, device=dev)
    res = {"workload": "N=20000, a=30, 30% in the shell [a-1/2,a), P=1600, M=2400, p=20, 4 (eps1,eps2,kappa) sets"}
    steps = 20
    for form, dip in (("green_identity", 0), ("single_layer", 2)):
        plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec, dipole=dip)
                 for s in systems]
        group = hs.Group(plans)

        def step():
            group.energy(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of, phi=phi, E=E)

        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < max(args.settle_s, 0.5):  # leave the idle clock state
            step()
            torch.cuda.synchronize()
        assert group.stream_check() == 0
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        group.profile(True)
        group.profile_read()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        st = group.profile_read()
        group.profile(False)
        res[form] = {"ms_per_step": ms, "eval_ms": st["eval"][0] / steps}
        log(f"bench[single_layer]: {form}: {ms:.4f} ms/step, evaluation {st['eval'][0] / steps:.4f} ms")
        if checks is not None:
            phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()

            def report(r, form=form):
                res[form]["rel_err_phi_l2_max"] = max(r["rel_phi"]["phi"])
                res[form]["rel_err_energy_max"] = max(r["rel_e"])
                log(f"bench[single_layer]: {form}: oracle phi rel L2 {res[form]['rel_err_phi_l2_max']:.2e}, "
                    f"energy {res[form]['rel_err_energy_max']:.2e}")

            checks.add("potentials", report, infos=[p.info for p in plans],
                       systems=[(s.x, s.y, s.z, s.q) for s in systems],
                       phis={"phi": [phi_h[b * N:(b + 1) * N] for b in range(nsys)]}, Es=[float(e) for e in E_h])
        for p in plans:
            p.close()
    return res


def leg_kirkwood(args, checks) -> dict:
    """The paper's comparison (Sec. 4.1) on the GPU: the C1 system (N = 200 uniform in a = 10,
    eps1 = 1, eps2 = 80, kappa = 0.1) by HSMA (FP64 pairs; P = 400, p = 10 and P = 1600, p = 20)
    and by the Kirkwood series truncated at order 40, each handed to the oracle checks against
    the converged series (the oracle's O2, not timed); then the time of the order-40 series on the N = 20000 shell
    system of the headline workload (first parameter set) beside HSMA's."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c1()
    s, ph = wl.systems[0], wl.systems[0].phys
    t = [torch.tensor(v, dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q)]
    res = {"workload": "C1: N=200 uniform in a=10, eps1=1, eps2=80, kappa=0.1; timing on N=20000, a=30, "
                       "30% in the shell, eps1=eps2=80, kappa=0.05"}
    out = {}
    for P, M in ((400, 600), (1600, 2400)):
        plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, P, M, pair_prec="fp64")
        phi = torch.empty(s.n, dtype=torch.float64, device=dev)
        plan.energy(*t, phi=phi)
        assert plan.stream_check() == 0
        out[f"hsma_p{plan.info['p']}_P{P}"] = phi.cpu().numpy()
        if P == 400:
            out["kirkwood_order40"] = plan.kirkwood(*t, order=40).cpu().numpy()
            assert plan.stream_check() == 0
        plan.close()
    if checks is not None:
        r = np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2)

        def report(errs):
            res["rel_err_l2_vs_converged_series"] = errs["all"]
            res["rel_err_l2_inner_ions_r_below_0.9a"] = errs["inner"]
            log("bench[kirkwood]: rel L2 vs the converged series, all ions / r < 0.9a: " +
                ", ".join(f"{k} {errs['all'][k]:.2e} / {errs['inner'][k]:.2e}" for k in errs["all"]))

        checks.add("series", report, physics=(ph.a, ph.eps1, ph.eps2, ph.kappa), system=(s.x, s.y, s.z, s.q),
                   outputs=out, inner=r < 0.9 * ph.a)
    wl2 = W.workload_c2()
    s2 = wl2.systems[0]
    p2 = hs.Plan(s2.phys.a, s2.phys.eps1, s2.phys.eps2, s2.phys.kappa, wl2.disc.P, wl2.disc.M)
    t2 = [torch.tensor(v, dtype=torch.float64, device=dev) for v in (s2.x, s2.y, s2.z, s2.q)]
    E = torch.empty(1, dtype=torch.float64, device=dev)
    times = {}
    for name, fn in (("kirkwood_order40_fp64", lambda: p2.kirkwood(*t2, order=40, E=E)),
                     ("hsma_fp32c", lambda: p2.energy(*t2, E=E))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) * 1e3 / 5
    assert p2.stream_check() == 0
    p2.close()
    res["ms_per_call_n20000"] = times
    log("bench[kirkwood]: N=20000: " + ", ".join(f"{k} {v:.2f} ms" for k, v in times.items()))
    return res


def leg_batched(args, checks) -> dict:
    """4096 configurations (a = 25, eps1 = 1, eps2 = 78.5, kappa = 0.3, P = 1024, M = 1536),
    N log-uniform in [100, 20000]: one batched call (shared plan, fit as MFMA GEMMs) per step,
    against the plain per-system path on the same systems."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wl = W.workload_c4()
    sizes = np.array([s.n for s in wl.systems], dtype=np.int64)
    off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = [np.concatenate([getattr(s, k) for s in wl.systems]) for k in "xyzq"]
    log(f"bench[batched]: {len(sizes)} systems, sum N = {off_h[-1]}, generated in {time.perf_counter() - t0:.1f} s")
    ph = wl.systems[0].phys
    plan = hs.Plan(ph.a, ph.eps1, ph.eps2, ph.kappa, wl.disc.P, wl.disc.M, pair_prec=args.prec)
    group = hs.Group([plan])
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off = torch.tensor(off_h, dtype=torch.int64, device=dev)
    nsys, total, max_n = len(sizes), int(off_h[-1]), int(sizes.max())
    phi = torch.empty(total, dtype=torch.float64, device=dev)
    E = torch.empty(nsys, dtype=torch.float64, device=dev)
    ws = hs.workspace(group.workspace_bytes(nsys, total, max_n), dev)

    def call():
        group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi, E=E, ws=ws)

    call()
    torch.cuda.synchronize()
    assert group.stream_check() == 0
    steps = 3
    t1 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / steps
    group.profile(True)
    group.profile_read()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    st = group.profile_read()
    group.profile(False)
    info = plan.info
    pk = float(np.sum(sizes * (sizes - 1)))
    ps = float(np.sum(sizes)) * info["P"]
    pc = float(np.sum(sizes)) * info["M"]
    # plain per-system path: one single-system call per configuration
    single_ws = hs.workspace(plan.workspace_bytes(max_n), dev)
    e1 = torch.empty(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for b in range(nsys):
        lo, hi = int(off_h[b]), int(off_h[b + 1])
        plan.energy(xb[lo:hi], yb[lo:hi], zb[lo:hi], qb[lo:hi], E=e1, ws=single_ws)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t2) * 1e3
    res = {
        "workload": "4096 configurations, N log-uniform in [100, 20000], a=25, eps1=1, eps2=78.5, kappa=0.3, "
                    "P=1024, M=1536, shared plan",
        "systems": nsys, "total_ions": total, "ms_per_call": ms, "systems_per_s": nsys / (ms * 1e-3),
        "gpairs_per_s": (pc + pk + ps) / (ms * 1e-3) / 1e9,
        "per_system_path_ms": ms_single, "per_system_path_systems_per_s": nsys / (ms_single * 1e-3),
        "stage_ms_per_call": {k: v[0] / steps for k, v in st.items()},
        "roofline": _eval_roofline(pk, ps, st["eval"][0] / steps * 1e-3, group.eval_kernel(nsys, total, max_n)),
    }
    # sampled systems for the oracle checks: the default route's potentials and energies here,
    # each fit route's potentials below
    rng = np.random.default_rng(0)
    pick = rng.choice(np.nonzero(sizes <= 3000)[0], 6, replace=False)
    phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()
    sampled = {"default": [phi_h[off_h[b]:off_h[b + 1]] for b in pick]}
    res["sampled_systems"] = [int(b) for b in pick]
    # The fit apply by each route on the same call: stage time, rate against the MFMA peak of its
    # type (the split-BF16 routes count their term products), and the sampled errors.
    K, P, M = info["K"], info["P"], info["M"]
    fit_flop = 2.0 * K * M * 2 * nsys + 2.0 * P * K * 2 * nsys
    routes = {}
    for mode, name, peak, mult in ((1, "gemv_fp32", None, 1), (2, "mfma_fp32", 157.3, 1),
                                   (3, "mfma_bf16x3", 2500.0, 3), (4, "mfma_bf16x6", 2500.0, 6)):
        group.set_fit(mode)
        call()
        group.profile(True)
        group.profile_read()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        fit_ms = group.profile_read()["fit"][0] / steps
        group.profile(False)
        r = {"fit_ms": fit_ms}
        if peak is not None:
            tf = fit_flop * mult / (fit_ms * 1e-3) / 1e12
            r.update({"tflops": tf, "peak_tflops": peak, "frac": tf / peak})
        phi_h = phi.cpu().numpy()
        sampled[name] = [phi_h[off_h[b]:off_h[b + 1]] for b in pick]
        routes[name] = r
        log(f"bench[batched]: fit {name}: {fit_ms:.3f} ms")
    group.set_fit(0)
    res["fit_routes"] = {"flop_per_call": fit_flop, **routes}
    if checks is not None:
        def report(r):
            res["rel_err_phi_l2_max_sampled"] = max(r["rel_phi"]["default"])
            res["rel_err_energy_max_sampled"] = max(r["rel_e"])
            for name in routes:
                routes[name]["rel_err_phi_l2_max_sampled"] = max(r["rel_phi"][name])
            log("bench[batched]: oracle on the sampled systems: max rel L2 " +
                ", ".join(f"{k} {max(v):.2e}" for k, v in r["rel_phi"].items()) +
                f"; energy {res['rel_err_energy_max_sampled']:.2e}")

        checks.add("potentials", report, infos=[info] * len(pick),
                   systems=[(wl.systems[b].x, wl.systems[b].y, wl.systems[b].z, wl.systems[b].q) for b in pick],
                   phis=sampled, Es=[float(E_h[b]) for b in pick])
    log(f"bench[batched]: {ms:.2f} ms/call, {res['systems_per_s']:.0f} systems/s "
        f"(per-system path {res['per_system_path_systems_per_s']:.0f})")
    return res


def leg_sweep(args, checks) -> dict:
    """Precision sweep on N = 1e6 ions uniform in a = 200 (charges +-1 and +-2, 2:1), eps1 = 1,
    eps2 = 80, kappa = 0.1, P = 6400, M = 9600 (p = 40): the whole path with FP32, compensated
    FP32 and FP64 pair sums (fit applied with FP32 GEMVs for the FP32 modes, FP64 GEMVs for FP64
    pairs), and the compensated FP32 path again with the fit applied as FP32 MFMA GEMMs and as
    split-BF16x3 and split-BF16x6 MFMA GEMMs.  The potentials of 256 sampled ions go to the oracle
    checks, the energies are compared with the FP64 run's; each run also reports its fit-stage time."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c3()
    s = wl.systems[0]
    d = wl.disc
    N = s.n
    x, y, z, q = (torch.tensor(v, dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 20))
    idx = np.sort(rng.choice(N, 256, replace=False))
    idx_d = torch.tensor(idx, dtype=torch.int64, device=dev)
    pairs = N * d.M + N * (N - 1) + N * d.P
    res = {"workload": "N=1e6 uniform in a=200, charges +-1/+-2 (2:1), eps1=1, eps2=80, kappa=0.1, "
                       "P=6400, M=9600, p=40", "pairs_per_call": pairs}
    runs = (("fp32", "fp32", 0), ("fp32c", "fp32c", 0), ("fp32c_fit_mfma_fp32", "fp32c", 2),
            ("fp32c_fit_mfma_bf16x3", "fp32c", 3), ("fp32c_fit_mfma_bf16x6", "fp32c", 4), ("fp64", "fp64", 0))
    route_name = {1: "gemv", 2: "mfma_fp32", 3: "mfma_bf16x3", 4: "mfma_bf16x6"}
    phis, Es = {}, {}
    plans = {}
    for label, prec, fit in runs:
        t0 = time.perf_counter()
        if prec not in plans:
            plans[prec] = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=prec)
        plan = plans[prec]
        t_plan = time.perf_counter() - t0
        plan.set_fit(fit)
        ws = hs.workspace(plan.workspace_bytes(N), dev)
        phi = torch.empty(N, dtype=torch.float64, device=dev)
        E = torch.empty(1, dtype=torch.float64, device=dev)
        plan.energy(x, y, z, q, phi=phi, E=E, ws=ws)
        torch.cuda.synchronize()
        assert plan.stream_check() == 0
        t1 = time.perf_counter()
        for _ in range(2):
            plan.energy(x, y, z, q, phi=phi, E=E, ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / 2
        plan.profile(True)
        plan.energy(x, y, z, q, phi=phi, E=E, ws=ws)
        st = plan.profile_read()
        plan.profile(False)
        phis[label] = phi[idx_d].cpu().numpy()
        Es[label] = float(E.cpu().numpy()[0])
        res[label] = {"ms_per_call": ms, "gpairs_per_s": pairs / (ms * 1e-3) / 1e9, "plan_s": t_plan, "E": Es[label],
                      "fit": route_name[plan.fit_route()] if prec != "fp64" else "gemv_fp64",
                      "fit_stage_ms": st["fit"][0]}
        log(f"bench[sweep]: {label}: {ms:.1f} ms/call ({pairs / (ms * 1e-3) / 1e9:.0f} GPairs/s), "
            f"fit {res[label]['fit']} {st['fit'][0]:.3f} ms, plan {t_plan:.2f} s")
        del ws, phi
    for label, _, _ in runs[:-1]:
        res[label]["rel_err_energy_vs_fp64"] = abs(Es[label] - Es["fp64"]) / abs(Es["fp64"])
    if checks is not None:
        def report(r):
            res["oracle_s"] = r["seconds"]
            for label, _, _ in runs:
                res[label]["rel_err_phi_l2_sampled"] = r["rel_phi"][label]
                res[label]["max_err_over_max_phi_sampled"] = r["max_over_max"][label]
            log(f"bench[sweep]: oracle on 256 sampled ions in {r['seconds']:.1f} s; rel L2 " +
                ", ".join(f"{lb} {res[lb]['rel_err_phi_l2_sampled']:.2e}" for lb, _, _ in runs))

        checks.add("sampled", report, info=plans["fp64"].info, system=(s.x, s.y, s.z, s.q), idx=idx, phis=phis)
    for plan in plans.values():
        plan.close()
    return res


def leg_accuracy(args, checks) -> dict:
    """The accuracy study of Sec. 4.1 (one unit charge, a = 1, eps1 = 2, eps2 = 80, kappa = 5) run
    by the library in FP64 pairs with the paper's own discretisation: the Gauss-Legendre check grid
    of 2p x (2p + 1) points on the interface and +-dy/2 point dipoles (dy = 1e-5 R_tau), up to
    p = 60 and F2 = 6765.  The GPU self energies go to the oracle checks against the converged
    Kirkwood series:
      fig2a: p = 30, F2 = 1597, tau in {0.05, 0.1, 0.15}, r_s from 0.1 to 0.98;
      fig2b: r_s = 0.9, tau = 0.1, F2 = 6765, p from 10 to 60;
      fig3:  r_s = 0.95, tau = 0.1, p in {15, 35, 55}, F2 in {610, 1597, 6765};
      fig4:  p = 20, F2 = 1597, r_s from 0.9 to 0.98, beside the Kirkwood series (on the GPU) at
             orders 20, 40 and 60.
    Plan set-up times (geometry build on the GPU) are reported too."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    a, eps1, eps2, kappa = 1.0, 2.0, 80.0, 5.0
    fib = {610: 377, 1597: 987, 6765: 4181}

    def plan(p, tau, F2):
        return hs.Plan(a, eps1, eps2, kappa, 2 * (F2 + 1), 2 * p * (2 * p + 1), p=p, tau=tau, rc_over_a=1.0,
                       F1=fib[F2], pair_prec="fp64", check_set=1, dipole=1, dy_over_Rtau=1e-5)

    def self_energy(pl, r_s, order=None):
        t = [torch.tensor(v, dtype=torch.float64, device=dev) for v in W.single_charge(r_s, a)]
        if order is None:
            e = float(pl.energy(*t).cpu().numpy()[0])
        else:
            e = 0.5 * float(pl.kirkwood(*t, order=order).cpu().numpy()[0])
        assert pl.stream_check() == 0
        return e

    rows = []  # (figure, label, r_s, E_self by the GPU)
    build_s = {}
    t_all = time.perf_counter()
    cases = [("fig2a", 30, tau, 1597, [0.1, 0.3, 0.5, 0.7, 0.8, 0.9, 0.92, 0.94, 0.95, 0.96, 0.97, 0.98])
             for tau in (0.05, 0.1, 0.15)]
    cases += [("fig2b", p, 0.1, 6765, [0.9]) for p in (10, 20, 30, 40, 50, 60)]
    cases += [("fig3", p, 0.1, F2, [0.95]) for p in (15, 35, 55) for F2 in (610, 1597, 6765)]
    cases += [("fig4", 20, 0.1, 1597, [0.9, 0.92, 0.94, 0.96, 0.98])]
    for fig, p, tau, F2, rs in cases:
        t0 = time.perf_counter()
        pl = plan(p, tau, F2)
        build_s[f"p{p}_F2_{F2}_tau{tau}"] = time.perf_counter() - t0
        label = f"hsma_p{p}_F2_{F2}_tau{tau}"
        for r_s in rs:
            rows.append((fig, label, r_s, self_energy(pl, r_s)))
            if fig == "fig4":
                for order in (20, 40, 60):
                    rows.append((fig, f"kirkwood_order{order}", r_s, self_energy(pl, r_s, order)))
        pl.close()
    res = {"workload": "one unit charge, a=1, eps1=2, eps2=80, kappa=5; Gauss-Legendre check grid on the "
                       "interface, point-pair dipoles dy=1e-5 R_tau, FP64 pairs",
           "plan_build_s": build_s, "seconds": time.perf_counter() - t_all}
    log(f"bench[accuracy]: {len(rows)} self energies from {len(cases)} plans in {res['seconds']:.1f} s "
        f"(largest plan build {max(build_s.values()):.2f} s)")
    if checks is not None:
        def report(refs):
            table = {}
            for fig, label, r_s, e in rows:
                table.setdefault(fig, {}).setdefault(label, {})[str(r_s)] = abs(e - refs[r_s])
            res["abs_err_self_energy"] = table
            res["ref_self_energy"] = {str(k): v for k, v in sorted(refs.items())}
            f2b = table["fig2b"]
            f3 = table["fig3"]
            f4 = table["fig4"]
            log("bench[accuracy]: fig2b r_s=0.9 error vs p: " +
                ", ".join(f"p{k.split('_')[1][1:]} {v['0.9']:.1e}" for k, v in f2b.items()))
            log("bench[accuracy]: fig3 r_s=0.95 relative error (p, F2): " +
                ", ".join(f"({k.split('_')[1][1:]}, {k.split('_')[3]}) {v['0.95'] / abs(refs[0.95]):.1e}"
                          for k, v in f3.items()))
            log("bench[accuracy]: fig4 max error over r_s in [0.9, 0.98]: " +
                ", ".join(f"{k} {max(v.values()):.1e}" for k, v in f4.items()))

        checks.add("self_energy", report, physics=(a, eps1, eps2, kappa), r_s=sorted({r[2] for r in rows}))
    return res


def leg_cpu_baseline(checks: OracleChecks) -> None:
    """The cpu_baseline leg: the only code in this file that runs the oracle.  It times the oracle
    on the headline workload (the cpu_baseline object, about ten seconds of host time) and computes
    the reference values of every accuracy check the other legs registered, handing each leg its
    errors.  Nothing here is timed as GPU work."""
    import numpy as np

    import oracle

    def params(i):
        return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"],
                             M=i["M"], tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=i["dipole"],
                             dy_over_Rtau=i["dy_over_Rtau"], check_set=i["check_set"])

    def rel(x, ref):
        return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))

    for kind, d, report in checks.jobs:
        if kind == "baseline":
            rel_phi, rel_e, secs, calls = [], [], 0.0, 0
            for i, (x, y, z, q), ph, e in zip(d["infos"], d["systems"], d["phis"], d["Es"]):
                t0 = time.perf_counter()
                ref = oracle.hsma_eval(params(i), x, y, z, q)
                secs += time.perf_counter() - t0
                calls += 1
                rel_phi.append(rel(ph, ref))
                e_ref = oracle.energy(q, ref)
                rel_e.append(abs(e - e_ref) / abs(e_ref))
            n = len(d["infos"])
            while secs < d["min_seconds"]:
                t0 = time.perf_counter()
                oracle.hsma_eval(params(d["infos"][calls % n]), *d["systems"][calls % n])
                secs += time.perf_counter() - t0
                calls += 1
            report({"rel_phi": rel_phi, "rel_e": rel_e, "calls": calls, "seconds": secs,
                    "cores": oracle.num_threads()})
        elif kind == "field":
            rp, rf = [], []
            for i, sysd, ph, f in zip(d["infos"], d["systems"], d["phis"], d["fields"]):
                ref_phi, ref_f = oracle.hsma_field(params(i), *sysd)
                rp.append(rel(ph, ref_phi))
                rf.append(rel(f, ref_f))
            report({"rel_phi": rp, "rel_field": rf})
        elif kind == "series":
            truth = oracle.kirkwood_eval(*d["physics"], *d["system"])
            inner = d["inner"]
            report({"all": {k: rel(v, truth) for k, v in d["outputs"].items()},
                    "inner": {k: rel(v[inner], truth[inner]) for k, v in d["outputs"].items()}})
        elif kind == "potentials":
            refs = [oracle.hsma_eval(params(i), *sysd) for i, sysd in zip(d["infos"], d["systems"])]
            rel_phi = {k: [rel(g, r) for g, r in zip(v, refs)] for k, v in d["phis"].items()}
            rel_e = []
            for sysd, r, e in zip(d["systems"], refs, d["Es"]):
                e_ref = oracle.energy(sysd[3], r)
                rel_e.append(abs(e - e_ref) / abs(e_ref))
            report({"rel_phi": rel_phi, "rel_e": rel_e})
        elif kind == "sampled":
            x, y, z, q = d["system"]
            idx = d["idx"]
            t0 = time.perf_counter()
            ref = oracle.hsma_eval(params(d["info"]), x, y, z, q, targets=np.stack([x[idx], y[idx], z[idx]], axis=1))
            secs = time.perf_counter() - t0
            report({"seconds": secs, "rel_phi": {k: rel(v, ref) for k, v in d["phis"].items()},
                    "max_over_max": {k: float(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))
                                     for k, v in d["phis"].items()}})
        elif kind == "self_energy":
            import workloads as W
            a = d["physics"][0]
            report({r_s: 0.5 * float(oracle.kirkwood_eval(*d["physics"], *W.single_charge(r_s, a))[0])
                    for r_s in d["r_s"]})
        else:
            raise ValueError(kind)


def leg_tree(args, checks) -> dict:
    """The treecode far field on N = 1e6 ions uniform in a = 200 (the precision-sweep system:
    charges +-1/+-2, eps1 = 1, eps2 = 80, kappa = 0.1, P = 6400, M = 9600, compensated FP32
    pairs): time per call for several (order, theta) beside the direct path, and the potentials
    of 256 sampled ions handed to the oracle checks."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c3()
    s = wl.systems[0]
    d = wl.disc
    N = s.n
    x, y, z, q = (torch.tensor(v, dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 20))
    idx = np.sort(rng.choice(N, 256, replace=False))
    idx_d = torch.tensor(idx, dtype=torch.int64, device=dev)
    plan = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec="fp32c")
    phi = torch.empty(N, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    res = {"workload": "N=1e6 uniform in a=200, charges +-1/+-2 (2:1), eps1=1, eps2=80, kappa=0.1, P=6400, M=9600, "
                       "p=40, compensated FP32 pairs"}
    sampled = {}
    runs = [("direct", None), ("tree_order4_theta0.5", (4, 0.5)), ("tree_order6_theta0.5", (6, 0.5)),
            ("tree_order6_theta0.4", (6, 0.4)), ("tree_order8_theta0.5", (8, 0.5)), ("tree_order6_theta0.3", (6, 0.3)),
            ("tree_order8_theta0.4", (8, 0.4))]
    for label, cfg in runs:
        if cfg is None:
            def call():
                plan.energy(x, y, z, q, phi=phi, E=E)
        else:
            def call(cfg=cfg):
                plan.energy_tree(x, y, z, q, order=cfg[0], theta=cfg[1], phi=phi, E=E)
        call()
        torch.cuda.synchronize()
        assert plan.stream_check() == 0
        t0 = time.perf_counter()
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 3
        sampled[label] = phi[idx_d].cpu().numpy()
        res[label] = {"ms_per_call": ms, "E": float(E.cpu().numpy()[0])}
        log(f"bench[tree]: {label}: {ms:.1f} ms/call")
    for label, _ in runs[1:]:
        res[label]["speedup_vs_direct"] = res["direct"]["ms_per_call"] / res[label]["ms_per_call"]
        res[label]["rel_err_energy_vs_direct"] = abs(res[label]["E"] - res["direct"]["E"]) / abs(res["direct"]["E"])
    if checks is not None:
        def report(r):
            for label, _ in runs:
                res[label]["rel_err_phi_l2_sampled"] = r["rel_phi"][label]
            log("bench[tree]: oracle on 256 sampled ions: rel L2 " +
                ", ".join(f"{lb} {r['rel_phi'][lb]:.2e}" for lb, _ in runs))

        checks.add("sampled", report, info=plan.info, system=(s.x, s.y, s.z, s.q), idx=idx, phis=sampled)
    plan.close()
    return res


def leg_serving(args) -> dict:
    """512 resident configurations (N log-uniform in [500, 50000], a ~ U[15, 40], kappa ~
    U[0.05, 1], eps1 = 1, eps2 = 78.5, P = 1024, M = 1536); requests 90% single-ion moves
    (ion and system uniform, displacement U([-1/2, 1/2]^3) kept inside, committed with
    probability 1/2) and 10% fresh full energies.  Capacity from a burst, then Poisson
    arrivals at 0.25, 0.5, 0.75, 0.9 and 1.1 of it; latency = done - submitted."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wl = W.workload_c5()
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, wl.disc.P, wl.disc.M) for s in wl.systems]
    dsl, esl = (int(v) for v in args.serving_slots.split(","))
    server = hs.Server(max_batch=512, delta_slots=dsl, energy_slots=esl)
    for p, s in zip(plans, wl.systems):
        t = [torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq"]
        server.add_system(p, *t)
    torch.cuda.synchronize()
    log(f"bench[serving]: {len(plans)} systems resident, {server.stats()['memory_used'] / 2**30:.2f} GiB, "
        f"set up in {time.perf_counter() - t0:.1f} s")
    rng = np.random.default_rng(1907017244)
    pos = [np.stack([s.x, s.y, s.z], axis=1).copy() for s in wl.systems]

    def stream(n):
        reqs = []
        for _ in range(n):
            b = int(rng.integers(len(pos)))
            if rng.random() < 0.1:
                reqs.append((hs.REQ_ENERGY, b, 0, 0, 0.0, 0.0, 0.0))
                continue
            k = int(rng.integers(len(pos[b])))
            new = W.random_move(rng, pos[b][k], wl.systems[b].phys.a)
            commit = int(rng.random() < 0.5)
            if commit:
                pos[b][k] = new
            reqs.append((hs.REQ_DELTA, b, commit, k, *new))
        return reqs

    def summarize(res, reqs, wall):
        lat = np.array([r.t_done - r.t_submit for r in res]) * 1e3
        dl = np.array([r.t_done - r.t_submit for r, q in zip(res, reqs) if q[0] == hs.REQ_DELTA]) * 1e3
        el = np.array([r.t_done - r.t_submit for r, q in zip(res, reqs) if q[0] == hs.REQ_ENERGY]) * 1e3
        assert all(r.status == 0 for r in res)
        return {"requests": len(res), "requests_per_s": len(res) / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "delta_p50_ms": float(np.percentile(dl, 50)),
                "delta_p99_ms": float(np.percentile(dl, 99)), "energy_p50_ms": float(np.percentile(el, 50)),
                "energy_p99_ms": float(np.percentile(el, 99))}

    n = args.serving_requests
    server.run_load(stream(500), np.zeros(500))  # warm-up
    reqs = stream(n)
    st0 = server.stats()
    res = server.run_load(reqs, np.zeros(n))
    st1 = server.stats()
    wall = max(r.t_done for r in res)
    burst = summarize(res, reqs, wall)
    cap = burst["requests_per_s"]
    out = {"workload": "512 resident configurations, N log-uniform in [500, 50000], a~U[15,40], kappa~U[0.05,1], "
                       "P=1024, M=1536; 90% single-ion moves (commit p=1/2), 10% fresh FP64 energies",
           "slots": {"moves": dsl, "energies": esl},
           "capacity_requests_per_s": cap, "burst": burst,
           "mean_batch": (st1["batched_requests"] - st0["batched_requests"]) / max(1, st1["batches"] - st0["batches"]),
           "loads": []}
    for f in (0.25, 0.5, 0.75, 0.9, 1.1):  # 1.1: overload, the queue grows over the run
        reqs = stream(n)
        arrival = np.cumsum(rng.exponential(1.0 / (f * cap), n))
        res = server.run_load(reqs, arrival)
        wall = max(r.t_done for r in res)
        d = summarize(res, reqs, wall)
        d["offered_fraction"] = f
        d["offered_requests_per_s"] = f * cap
        out["loads"].append(d)
        log(f"bench[serving]: load {f:.2f} x capacity: p50 {d['p50_ms']:.3f} ms, p99 {d['p99_ms']:.3f} ms "
            f"(moves {d['delta_p50_ms']:.3f} / {d['delta_p99_ms']:.3f} ms)")
    server.close()
    # plain per-system path: one synchronous single-ion query at a time on a resident system
    b = int(np.argmax([len(p) for p in pos]))
    s = wl.systems[b]
    t = [torch.tensor(v, dtype=torch.float64, device=dev) for v in (pos[b][:, 0], pos[b][:, 1], pos[b][:, 2], s.q)]
    one = hs.System(plans[b], *t)
    dE = torch.empty(1, dtype=torch.float64, device=dev)
    lat = []
    for i in range(300):
        k = int(rng.integers(len(pos[b])))
        new = W.random_move(rng, pos[b][k], s.phys.a)
        ta = time.perf_counter()
        one.delta_energy(k, new, out=dE)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ta)
    one.close()
    lat = np.array(lat[20:]) * 1e3
    out["per_system_path"] = {"system_ions": int(len(pos[b])), "delta_requests_per_s": float(1e3 / lat.mean()),
                              "delta_p50_ms": float(np.percentile(lat, 50)), "delta_p99_ms": float(np.percentile(lat, 99))}
    log(f"bench[serving]: capacity {cap:.0f} req/s (burst), per-system path {1e3 / lat.mean():.0f} req/s")
    return out


if __name__ == "__main__":
    sys.exit(main())
