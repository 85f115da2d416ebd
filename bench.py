#!/usr/bin/env python3
"""Benchmark of the HSMA reaction-potential hot path on one MI355X.

Headline workload: N = 1,000,000 ions uniform in a cavity of radius a = 200, charges +-1 and
+-2 (2:1, neutral), eps1 = 1, eps2 = 80, kappa = 0.1, P = 6,400 surface nodes, M = 9,600
check points (p = 40): the timing workload of Sec. 4.2 at its largest N.  One step = the
reaction energy E = 1/2 sum q_i Phi_i of the whole system (hsma_energy): Kelvin images, FP64
check sums, FP64 fit, FP64 energy pair sums (the symmetric energy kernel), fixed-order FP64
reduction.  Inputs are resident in HBM before timing starts.

Pairs per step = N*M (check) + N*(N-1) (Kelvin images, own image analytic) + N*P (surface
nodes) = 1.016e12.  value = pairs / time, in GPairs/s; systems/s = steps / time.  The energy
is compared with the oracle's full evaluation stored in tests/golden/c3_reference.json.

Prints one JSON line.  Accuracy against the FP64 CPU oracle is measured outside the timed
regions, by the cpu_baseline leg at the end, which also times the oracle on the host cores;
the other legs hand it their GPU results as plain arrays.
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

# Published MI355X vector peaks (dense): FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s.
PEAK_FP64, PEAK_FP32 = 78.6e12, 157.3e12
# Algorithmic flops of one pair term (its minimal FP arithmetic; a fused multiply-add counts 2):
#   Kelvin image: 3 sub, |d|^2 (mul + 2 fma: 5), reciprocal root 1, accumulate (fma: 2) = 11;
#   surface node: 3 sub, |d|^2 5, root 1, d.y_s 5, 1/r^2 1, monopole + dipole (2 fma: 4), 2 = 21;
#   check point: the Kelvin pair with a second accumulator = 13.
FLOP_KELVIN, FLOP_SURFACE, FLOP_CHECK = 11, 21, 13
# Potential and field of a pair (the field kernel): the potential's flops plus the gradient:
#   Kelvin image: 11 + r^-3 (2) + strength r^-3 (1) + three fma into E (6) = 20;
#   surface node: 21 + r^-2, r^-3 and the dipole factor (6) + two vector fma into E (12) = 39.
FLOP_FIELD_KELVIN, FLOP_FIELD_SURFACE = 20, 39
# VALU issue beside the roofline: the energy kernel's VALU instructions per launch (SQ_INSTS_VALU
# from the committed counter summary of the same engine source) over one FP64 wave instruction per
# 4 cycles on each of the 256 x 4 SIMDs at 2.4 GHz.
FP64_WAVE_ISSUE_RATE = 256 * 4 * 2.4e9 / 4
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "c3_reference.json")
PROFILE_DIR = os.path.join(ROOT, "profiles")
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
    ap.add_argument("--prec", default="fp32c", choices=["fp32", "fp32c", "fp64"],
                    help="pair precision of the potentials in the legs (energies always use FP64 pairs)")
    ap.add_argument("--no-oracle", action="store_true", help="skip the accuracy checks and the CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-stage HIP events")
    ap.add_argument("--legs", default="plan,c2,batched,serving,sweep,field,kirkwood,accuracy,single_layer,tree",
                    help="extra workloads after the headline one: plan, c2, batched, serving, sweep, field, kirkwood, "
                         "accuracy, single_layer, tree (comma list, or none)")
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up steps, so that the device has left its idle "
                         "clock state when timing starts")
    ap.add_argument("--serving-requests", type=int, default=20000)
    ap.add_argument("--serving-variants", default="0:1,-1:1",
                    help="request server settings to measure, comma-separated energy_workgroups:move_priority "
                         "(energy grid 0: one workgroup per compute unit, -1: no limit); the first is the headline")
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
    wl = W.workload_c3()
    s, d = wl.systems[0], wl.disc
    N = s.n
    t0 = time.perf_counter()
    plan = hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec)
    t_plan = time.perf_counter() - t0
    inf = plan.info
    M, P = inf["M"], inf["P"]
    x, y, z, q = (torch.tensor(v, dtype=torch.float64, device=dev) for v in (s.x, s.y, s.z, s.q))
    E = torch.empty(1, dtype=torch.float64, device=dev)
    ws = hs.workspace(plan.workspace_bytes(N), dev)
    stream = torch.cuda.current_stream()
    pairs_check, pairs_kelvin, pairs_surface = N * M, N * (N - 1), N * P
    pairs_step = pairs_check + pairs_kelvin + pairs_surface

    def step():
        plan.energy(x, y, z, q, E=E, stream=stream, ws=ws)

    log(f"bench: workload {wl.name}, N={N}, P={P}, M={M}, p={inf['p']}, energy (FP64 pairs), plan {t_plan:.2f} s")
    t_settle, settle_steps = time.perf_counter(), 0
    while time.perf_counter() - t_settle < args.settle_s:
        step()
        torch.cuda.synchronize()
        settle_steps += 1
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert plan.stream_check() == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    e_gpu = float(E.cpu().numpy()[0])
    log(f"bench: {ms:.3f} ms/step over {args.steps} steps, E = {e_gpu!r}")
    stages = {}
    prof_steps = min(args.steps, 5)
    if not args.no_profile:
        # per-stage HIP events on the launch stream, in a separate pass (events cost time of their own)
        plan.profile(True)
        plan.profile_read()
        for _ in range(prof_steps):
            step()
        torch.cuda.synchronize()
        stages = {k: list(v) for k, v in plan.profile_read().items()}
        plan.profile(False)
    out = {
        "metric": "GPairs/s and systems/s at <=1e-6 rel err vs FP64; p50/p99 dE latency",
        "value": pairs_step / (ms * 1e-3) / 1e9,
        "unit": "GPairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "N=1e6 ions uniform in a=200, charges +-1/+-2 (2:1, neutral), eps1=1, eps2=80, "
                               "kappa=0.1, P=6400, M=9600, p=40; reaction energy of the whole system per step",
                   "N": N, "P": P, "M": M, "p": inf["p"], "systems_per_step": 1,
                   "pairs_per_step": pairs_step, "energy_pairs": "fp64"},
        "systems_per_s": 1.0 / (ms * 1e-3),
        "settle": {"seconds": args.settle_s, "steps": settle_steps},
        "plan_s": t_plan,
    }
    with open(GOLDEN_C3) as f:
        golden = json.load(f)
    if golden["N"] == N and golden["P"] == P and golden["M"] == M:
        out["rel_err_energy"] = abs(e_gpu - golden["E"]) / abs(golden["E"])
        out["energy_reference"] = "tests/golden/c3_reference.json (oracle O1, full FP64 evaluation)"
        log(f"bench: energy vs the stored oracle evaluation: rel {out['rel_err_energy']:.2e}")
    if stages:
        ev_ms, ev_n = stages["eval"]
        avg = ev_ms / max(ev_n, 1) * 1e-3  # one energy-kernel launch per step
        flop = FLOP_KELVIN * pairs_kelvin + FLOP_SURFACE * pairs_surface
        valu = _measured_value("k_energy64", "sq_counters", "valu_instructions_per_launch")
        out["roofline"] = {
            "bound": "alu",
            "kernel": "k_energy64 (FP64 energy pair sums: symmetric Kelvin block pairs + surface chunks)",
            "achieved": flop / avg / 1e12,
            "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s",
            "frac": flop / avg / PEAK_FP64,
            "traffic": _measured_traffic("k_energy64", flop),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 256 MiB copy)",
            "algorithmic_bytes": 48 * N + 48 * P,
            "avg_launch_ms": avg * 1e3,
            "flop_per_launch": flop,
            "flop_model": "11 per Kelvin pair N(N-1), 21 per surface pair NP (algorithmic, both directions of a "
                          "pair counted); peak: published FP64 vector rate",
            "valu_instructions_per_launch": valu,
            "valu_issue_fraction": valu / avg / FP64_WAVE_ISSUE_RATE if valu else None,
        }
        out["stage_ms_per_step"] = {k: v[0] / prof_steps for k, v in stages.items()}
        log(f"bench: energy kernel {avg * 1e3:.2f} ms/launch, {out['roofline']['achieved']:.1f} TFLOP/s = "
            f"{out['roofline']['frac']:.3f} of the FP64 peak")
    del ws

    checks = None if args.no_oracle else OracleChecks()
    if checks is not None:
        def report_headline(r):
            out["cpu_baseline"] = {
                "value": r["pairs"] / r["seconds"] / 1e9,
                "unit": "GPairs/s",
                "cores": r["cores"],
                "kind": "oracle",
                "sample": "%d oracle (O1, FP64) evaluations of the headline system, each at 1000 sampled ions: "
                          "check sums of all 1e6 ions at the 9600 check points, Householder least squares, surface "
                          "strengths, Kelvin and surface sums at the 1000 ions (%.3g pairs in all)" % (r["calls"],
                                                                                                  r["pairs"]),
                "seconds": r["seconds"],
                "build": r["build"],
            }
            log(f"bench: cpu_baseline {out['cpu_baseline']['value']:.2f} GPairs/s on {r['cores']} threads "
                f"({r['seconds']:.1f} s, {r['build']})")

        checks.add("baseline_sampled", report_headline, info=inf, system=(s.x, s.y, s.z, s.q), targets=1000,
                   seed=W.SEED_BASE + 22, min_seconds=10.0)
    plan.close()
    legs = [l for l in args.legs.split(",") if l and l != "none"]
    if "plan" in legs:
        out["plan_build"] = leg_plan(args)
    if "c2" in legs:
        out["c2"] = leg_c2(args, checks)
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


def _measured_value(kernel: str, kind: str, key: str):
    """A per-launch figure of a kernel from its committed PMC summary (profiles/<kernel>_*<kind>.txt:
    its 'key value' lines), or None when no summary exists or the engine source changed since the
    counted run (its hash)."""
    import glob
    import hashlib
    try:
        with open(ENGINE_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        for path in sorted(glob.glob(os.path.join(PROFILE_DIR, f"{kernel}_*{kind}.txt"))):
            kv = dict(l.split(None, 1) for l in open(path) if l.strip() and not l.startswith((" ", "#")))
            if kv.get("engine_source_sha256", "").strip() == sha and kv.get("kernel", "").strip() == kernel:
                return float(kv[key])
    except (OSError, ValueError, KeyError):
        return None
    return None


def _measured_traffic(kernel: str, _flop=None):
    """HBM bytes per launch of a kernel from its committed PMC summary (profiles/<kernel>_*hbm_traffic.txt)."""
    return _measured_value(kernel, "hbm_traffic", "traffic_bytes_per_launch")


def _pot_roofline(pairs_kelvin, pairs_surface, avg_s, prec, kernel):
    """Roofline of a potential launch (Kelvin + surface pairs) against the published vector peak of
    its pair precision, with the algorithmic flops of FLOP_KELVIN / FLOP_SURFACE per pair."""
    peak = PEAK_FP64 if prec == "fp64" else PEAK_FP32
    flop = FLOP_KELVIN * pairs_kelvin + FLOP_SURFACE * pairs_surface
    return {"bound": "alu", "kernel": kernel, "achieved": flop / avg_s / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": flop / avg_s / peak, "avg_launch_ms": avg_s * 1e3, "flop_per_launch": flop}


def _energy_roofline(pairs_kelvin, pairs_surface, avg_s):
    flop = FLOP_KELVIN * pairs_kelvin + FLOP_SURFACE * pairs_surface
    return {"bound": "alu", "kernel": "k_energy64", "achieved": flop / avg_s / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": flop / avg_s / PEAK_FP64, "avg_launch_ms": avg_s * 1e3}


def leg_c2(args, checks) -> dict:
    """N = 20,000 ions with 30% in the shell r in [a - 1/2, a) of a cavity of radius a = 30,
    charges +-1 balanced, P = 1,600, M = 2,400, under the four parameter sets (eps1, eps2) in
    {(80, 80), (1, 80)} x kappa in {0.05, 0.5}, as one batched call of four systems: potentials
    alone (the pair precision of --prec), energies alone (FP64 pairs), and both; the potential
    kernel against its roofline; the plain per-system path on the same work."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c2()
    d = wl.disc
    systems = wl.systems
    N = systems[0].n
    nsys = len(systems)
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec)
             for s in systems]
    group = hs.Group(plans)
    cat = [np.concatenate([getattr(s, k) for s in systems]) for k in "xyzq"]
    xb, yb, zb, qb = (torch.tensor(v, dtype=torch.float64, device=dev) for v in cat)
    off = torch.tensor(np.arange(nsys + 1) * N, dtype=torch.int64, device=dev)
    plan_of = torch.arange(nsys, dtype=torch.int32, device=dev)
    phi = torch.empty(nsys * N, dtype=torch.float64, device=dev)
    E = torch.empty(nsys, dtype=torch.float64, device=dev)
    ws = hs.workspace(group.workspace_bytes(nsys, nsys * N, N), dev)
    inf = plans[0].info
    M, P = inf["M"], inf["P"]
    pk, ps, pc = N * (N - 1) * nsys, N * P * nsys, N * M * nsys
    pairs = pk + ps + pc
    calls = {
        "potentials": lambda: group.potential(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of,
                                              phi=phi, ws=ws),
        "energies": lambda: group.energy(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of, E=E,
                                         ws=ws),
        "potentials_and_energies": lambda: group.energy(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N,
                                                        plan_of=plan_of, phi=phi, E=E, ws=ws),
    }
    res = {"workload": "N=20000, a=30, 30% in the shell [a-1/2,a), +-1 charges, P=1600, M=2400, p=20, "
                       "4 (eps1,eps2,kappa) sets in one call", "pairs_per_call": pairs, "pair_precision": args.prec}
    steps = 20
    for name, call in calls.items():
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < max(args.settle_s, 0.5):  # leave the idle clock state
            call()
            torch.cuda.synchronize()
        assert group.stream_check() == 0
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        group.profile(True)
        group.profile_read()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        st = group.profile_read()
        group.profile(False)
        ev = st["eval"][0] / steps * 1e-3
        r = {"ms_per_call": ms, "gpairs_per_s": pairs / (ms * 1e-3) / 1e9,
             "stage_ms_per_call": {k: v[0] / steps for k, v in st.items()}}
        if name == "potentials":
            sym = group.eval_kernel(nsys, nsys * N, N)
            r["roofline"] = _pot_roofline(pk, ps, ev, args.prec, "k_kelvin_sym<%d>" % (sym // 64) if sym > 0
                                          else "k_eval")
            r["roofline"]["traffic"] = _measured_traffic("k_kelvin_sym4") if sym == 256 else None
        elif name == "energies":
            r["roofline"] = _energy_roofline(pk, ps, ev)
        res[name] = r
        log(f"bench[c2]: {name}: {ms:.4f} ms/call, evaluation {ev * 1e3:.4f} ms")
    # the plain per-system path on the same work, for comparison
    x, y, z, q = xb[:N], yb[:N], zb[:N], qb[:N]
    single_ws = [hs.workspace(p.workspace_bytes(N), dev) for p in plans]
    single_phi = [torch.empty(N, dtype=torch.float64, device=dev) for _ in plans]
    single_E = [torch.empty(1, dtype=torch.float64, device=dev) for _ in plans]

    def step_single():
        for p, w, ph, e in zip(plans, single_ws, single_phi, single_E):
            p.energy(x, y, z, q, phi=ph, E=e, ws=w)

    step_single()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        step_single()
    torch.cuda.synchronize()
    res["per_system_path_ms_per_call"] = (time.perf_counter() - t2) * 1e3 / steps
    if checks is not None:
        calls["potentials_and_energies"]()
        phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()

        def report(r):
            res["rel_err_phi_l2_max"] = max(r["rel_phi"]["phi"])
            res["rel_err_energy_max"] = max(r["rel_e"])
            log(f"bench[c2]: oracle: phi rel L2 {res['rel_err_phi_l2_max']:.2e}, energy "
                f"{res['rel_err_energy_max']:.2e}")

        checks.add("potentials", report, infos=[p.info for p in plans],
                   systems=[(s.x, s.y, s.z, s.q) for s in systems],
                   phis={"phi": [phi_h[b * N:(b + 1) * N] for b in range(nsys)]}, Es=[float(e) for e in E_h])
    for p in plans:
        p.close()
    return res


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

    def call_field_only():  # potential and field without the energy launch, for the kernel's roofline
        return group.field(off, xb, yb, zb, qb, total_n=total, max_n=N, plan_of=plan_of, E=False)

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
    for _ in range(steps):
        call_field_only()
    torch.cuda.synchronize()
    st_f = group.profile_read()
    group.profile(False)
    inf = plans[0].info
    P, M = inf["P"], inf["M"]
    pk, ps = N * (N - 1) * nsys, N * P * nsys
    pairs = pk + ps + N * M * nsys
    # the eval stage holds the energy launch's k_energy64 and the field launch's k_eval_field
    peak = PEAK_FP64 if args.prec == "fp64" else PEAK_FP32
    res = {"workload": "N=20000, a=30, 30% in the shell [a-1/2,a), P=1600, M=2400, p=20, 4 (eps1,eps2,kappa) sets, "
                       "potential + field + energy", "ms_per_call": ms, "gpairs_per_s": pairs / (ms * 1e-3) / 1e9,
           "stage_ms_per_call": {k: v[0] / steps for k, v in st.items()}}
    evf = st_f["eval"][0] / steps * 1e-3
    flop = FLOP_FIELD_KELVIN * pk + FLOP_FIELD_SURFACE * ps
    res["roofline"] = {"bound": "alu", "kernel": "k_eval_field (potential and field pair sums)",
                       "achieved": flop / evf / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": flop / evf / peak,
                       "avg_launch_ms": evf * 1e3, "flop_model": "20 per Kelvin pair, 39 per surface pair"}
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
    log(f"bench[field]: {ms:.3f} ms/call, field kernel {evf * 1e3:.3f} ms ({res['roofline']['frac']:.2f} of the "
        f"vector peak)")
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
            group.potential(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of, phi=phi)

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
        group.energy(off, xb, yb, zb, qb, total_n=nsys * N, max_n=N, plan_of=plan_of, E=E)
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
                     ("hsma_energy_fp64", lambda: p2.energy(*t2, E=E)),
                     ("hsma_potentials_fp32c", lambda: p2.potential(*t2))):
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
    N log-uniform in [100, 20000]: one batched call (shared plan) per step for the energies (FP64
    energy launch; systems/s) and one for the potentials (pair precision of --prec, fit as FP32 MFMA
    GEMMs), against the plain per-system path on the same systems."""
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
    info = plan.info
    pk = float(np.sum(sizes * (sizes - 1)))
    ps = float(np.sum(sizes)) * info["P"]
    pc = float(np.sum(sizes)) * info["M"]
    steps = 3

    def timed(call):
        call()
        torch.cuda.synchronize()
        assert group.stream_check() == 0
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
        return ms, {k: v[0] / steps for k, v in st.items()}

    def energies():
        group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max_n, E=E, ws=ws)

    def potentials():
        group.potential(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi, ws=ws)

    ms_e, st_e = timed(energies)
    ms_p, st_p = timed(potentials)
    # the library's timing-based tuner on both calls (energies first, then potentials), the tuned
    # calls timed, then each captured into a HIP graph and replayed
    default_settings = group.settings()
    tws = hs.workspace(group.autotune_workspace_bytes(nsys, total, max_n), dev)
    t_tune = time.perf_counter()
    tune_e = group.autotune(off, xb, yb, zb, qb, total_n=total, max_n=max_n, E=E, ws=tws, force=True)
    tune_p = group.autotune(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi, ws=tws, force=True)
    t_tune = time.perf_counter() - t_tune
    tuned_settings = group.settings()

    def trial_lines(r):
        out = []
        for tr in r["trials"]:
            diff = {k: v for k, v in tr["settings"].items() if v != default_settings[k]}
            out.append({"changed": diff, "ms": tr["ms"]})
        return out

    tune_e["trials"] = trial_lines(tune_e)
    tune_p["trials"] = trial_lines(tune_p)
    for name, r in (("energies", tune_e), ("potentials", tune_p)):
        log(f"bench[batched]: tuner, {name}: " + ", ".join(
            f"{' '.join(f'{k}={v}' for k, v in t['changed'].items()) or 'default'} {t['ms']:.2f}" for t in r["trials"]))

    def energies_t(stream=None):
        group.energy(off, xb, yb, zb, qb, total_n=total, max_n=max_n, E=E, ws=tws, stream=stream)

    def potentials_t(stream=None):
        group.potential(off, xb, yb, zb, qb, total_n=total, max_n=max_n, phi=phi, ws=tws, stream=stream)

    ms_e_t, _ = timed(energies_t)
    ms_p_t, _ = timed(potentials_t)

    def replay_ms(call):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            call(s)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            call(s)
        g.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        out_ms = (time.perf_counter() - t1) * 1e3 / steps
        assert group.stream_check() == 0
        return out_ms

    ms_e_g = replay_ms(energies_t)
    ms_p_g = replay_ms(potentials_t)
    log(f"bench[batched]: tuned in {t_tune:.1f} s: energies {ms_e:.2f} -> {ms_e_t:.2f} ms (graph replay {ms_e_g:.2f}), "
        f"potentials {ms_p:.2f} -> {ms_p_t:.2f} ms (graph replay {ms_p_g:.2f}); settings {tuned_settings}")
    # plain per-system path: one single-system energy call per configuration
    single_ws = hs.workspace(plan.workspace_bytes(max_n), dev)
    e1 = torch.empty(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for b in range(nsys):
        lo, hi = int(off_h[b]), int(off_h[b + 1])
        plan.energy(xb[lo:hi], yb[lo:hi], zb[lo:hi], qb[lo:hi], E=e1, ws=single_ws)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t2) * 1e3
    group.apply_settings(default_settings)
    energies()
    sym = group.eval_kernel(nsys, total, max_n)
    res = {
        "workload": "4096 configurations, N log-uniform in [100, 20000], a=25, eps1=1, eps2=78.5, kappa=0.3, "
                    "P=1024, M=1536, shared plan",
        "systems": nsys, "total_ions": total, "pairs_per_call": pc + pk + ps,
        "energies": {"ms_per_call": ms_e, "systems_per_s": nsys / (ms_e * 1e-3),
                     "gpairs_per_s": (pc + pk + ps) / (ms_e * 1e-3) / 1e9, "stage_ms_per_call": st_e,
                     "roofline": _energy_roofline(pk, ps, st_e["eval"] * 1e-3)},
        "potentials": {"ms_per_call": ms_p, "systems_per_s": nsys / (ms_p * 1e-3),
                       "gpairs_per_s": (pc + pk + ps) / (ms_p * 1e-3) / 1e9, "stage_ms_per_call": st_p,
                       "roofline": _pot_roofline(pk, ps, st_p["eval"] * 1e-3, args.prec,
                                                 "k_kelvin_sym<%d>" % (sym // 64) if sym > 0 else "k_eval")},
        "per_system_path_ms": ms_single, "per_system_path_systems_per_s": nsys / (ms_single * 1e-3),
        "tuned": {"default_settings": default_settings, "settings": tuned_settings, "tuning_s": t_tune,
                  "tuner_energies": tune_e, "tuner_potentials": tune_p,
                  "energies_ms_per_call": ms_e_t, "potentials_ms_per_call": ms_p_t,
                  "graph_replay": {"energies_ms_per_call": ms_e_g, "potentials_ms_per_call": ms_p_g,
                                   "energies_systems_per_s": nsys / (ms_e_g * 1e-3),
                                   "potentials_systems_per_s": nsys / (ms_p_g * 1e-3)}},
    }
    # sampled systems for the oracle checks: the default route's potentials and the energies here,
    # each fit route's potentials below
    rng = np.random.default_rng(0)
    pick = rng.choice(np.nonzero(sizes <= 3000)[0], 6, replace=False)
    phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()
    sampled = {"default": [phi_h[off_h[b]:off_h[b + 1]] for b in pick]}
    res["sampled_systems"] = [int(b) for b in pick]
    # The fit apply by each route on the potential call: stage time, rate against the MFMA peak of
    # its type (the split-BF16 routes count their term products), and the sampled errors.
    K, P, M = info["K"], info["P"], info["M"]
    fit_flop = 2.0 * K * M * 2 * nsys + 2.0 * P * K * 2 * nsys
    routes = {}
    for mode, name, peak, mult in ((1, "gemv_fp32", None, 1), (2, "mfma_fp32", 157.3, 1),
                                   (3, "mfma_bf16x3", 2500.0, 3), (4, "mfma_bf16x6", 2500.0, 6)):
        group.set_fit(mode)
        _, st = timed(potentials)
        fit_ms = st["fit"]
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
    log(f"bench[batched]: energies {ms_e:.2f} ms/call ({res['energies']['systems_per_s']:.0f} systems/s), "
        f"potentials {ms_p:.2f} ms/call; per-system path {res['per_system_path_systems_per_s']:.0f} systems/s")
    return res


def leg_sweep(args, checks) -> dict:
    """Precision sweep on N = 1e6 ions uniform in a = 200 (charges +-1 and +-2, 2:1), eps1 = 1,
    eps2 = 80, kappa = 0.1, P = 6400, M = 9600 (p = 40): the whole path with FP32, compensated
    FP32 and FP64 pair sums (fit applied with FP32 GEMVs for the FP32 modes, FP64 GEMVs for FP64
    pairs), and the compensated FP32 path again with the fit applied as FP32 MFMA GEMMs and as
    split-BF16x3 and split-BF16x6 MFMA GEMMs.  The potentials of 256 sampled ions go to the oracle
    checks; each run also reports its fit-stage time.  Potentials only (hsma_potential): the
    energies, FP64 in every mode, are the headline's."""
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
    phis = {}
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
        plan.potential(x, y, z, q, phi=phi, ws=ws)
        torch.cuda.synchronize()
        assert plan.stream_check() == 0
        t1 = time.perf_counter()
        for _ in range(2):
            plan.potential(x, y, z, q, phi=phi, ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / 2
        plan.profile(True)
        plan.potential(x, y, z, q, phi=phi, ws=ws)
        st = plan.profile_read()
        plan.profile(False)
        phis[label] = phi[idx_d].cpu().numpy()
        res[label] = {"ms_per_call": ms, "gpairs_per_s": pairs / (ms * 1e-3) / 1e9, "plan_s": t_plan,
                      "fit": route_name[plan.fit_route()] if prec != "fp64" else "gemv_fp64",
                      "fit_stage_ms": st["fit"][0],
                      "roofline": _pot_roofline(N * (N - 1), N * d.P, st["eval"][0] * 1e-3, prec, "evaluation")}
        log(f"bench[sweep]: {label}: {ms:.1f} ms/call ({pairs / (ms * 1e-3) / 1e9:.0f} GPairs/s), "
            f"fit {res[label]['fit']} {st['fit'][0]:.3f} ms, plan {t_plan:.2f} s")
        del ws, phi
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


def leg_plan(args) -> dict:
    """Plan set-up time (geometry on the GPU: nodes, bases, normal equations, Cholesky factor and
    the blocked triangular solves for the pseudo-inverse) for the C2 geometry (a = 30, P = 1600,
    M = 2400, p = 20), the C3 geometry (a = 200, P = 6400, M = 9600, p = 40) and the C3 geometry
    at p = 60 (K = 3721).  Each is built fresh: no other plan holds its geometry."""
    import torch

    import paper_1907_01724_amd as hs

    torch.cuda.synchronize()
    out = {}
    for label, a, P, M, p in (("c2_p20_K441", 30.0, 1600, 2400, None), ("c3_p40_K1681", 200.0, 6400, 9600, None),
                              ("c3_p60_K3721", 200.0, 6400, 9600, 60)):
        t0 = time.perf_counter()
        pl = hs.Plan(a, 1.0, 80.0, 0.1, P, M, p=p)
        torch.cuda.synchronize()
        out[label + "_ms"] = (time.perf_counter() - t0) * 1e3
        pl.close()
        log(f"bench[plan]: {label}: {out[label + '_ms']:.1f} ms")
    return out


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

    # The timed oracle is the same C source built for the host it runs on (-O3 -march=native, no
    # fast-math), in a scratch directory; the accuracy references use the same build.
    build = "gcc -O2 (oracle/__init__.py build)"
    try:
        import tempfile
        native = os.path.join(tempfile.mkdtemp(prefix="hsma_oracle_"), "libhsma_oracle_native.so")
        flags = oracle.build_native(native)
        oracle.use_library(native)
        build = "gcc " + " ".join(flags)
    except Exception as e:  # keep the default build
        log(f"bench: native oracle build failed ({e}); timing the default build")

    def params(i):
        return oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"],
                             M=i["M"], tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"], dipole=i["dipole"],
                             dy_over_Rtau=i["dy_over_Rtau"], check_set=i["check_set"])

    def rel(x, ref):
        return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))

    for kind, d, report in checks.jobs:
        if kind == "baseline_sampled":
            # whole oracle evaluations at 1000 sampled ions each (check sums of all ions, the fit,
            # Kelvin and surface sums at the sample), repeated with fresh samples for at least 10 s
            x, y, z, q = d["system"]
            i = d["info"]
            n = len(x)
            rng = np.random.Generator(np.random.PCG64(d["seed"]))
            secs, pairs, calls = 0.0, 0.0, 0
            while secs < d["min_seconds"]:
                idx = np.sort(rng.choice(n, d["targets"], replace=False))
                t0 = time.perf_counter()
                oracle.hsma_eval(params(i), x, y, z, q, targets=np.stack([x[idx], y[idx], z[idx]], axis=1))
                secs += time.perf_counter() - t0
                pairs += float(n) * i["M"] + float(len(idx)) * (n + i["P"])
                calls += 1
            report({"seconds": secs, "pairs": pairs, "calls": calls, "cores": oracle.num_threads(), "build": build})
        elif kind == "baseline":
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
            ("tree_order8_theta0.4", (8, 0.4)), ("tree_order8_theta0.35", (8, 0.35)), ("tree_order8_theta0.3", (8, 0.3)),
            ("tree_order10_theta0.5", (10, 0.5)), ("tree_order10_theta0.45", (10, 0.45)),
            ("tree_order10_theta0.4", (10, 0.4))]
    for label, cfg in runs:
        if cfg is None:
            def call():
                plan.potential(x, y, z, q, phi=phi)
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
        if cfg is None:
            plan.energy(x, y, z, q, E=E)  # the direct energy, FP64 pairs
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
    probability 1/2) and 10% fresh full energies.  For each request-server setting (--serving-variants:
    the full energies' grid and the move kernels' wave priority): capacity from a burst, then Poisson
    arrivals at 0.25, 0.5, 0.75, 0.9 and 1.1 of that capacity, the same requests and the same
    unit-rate arrival gaps for every setting; latency = done - submitted.  Then the plain per-system
    path (each request run alone, synchronously, on its resident system) under the first setting's
    arrival streams."""
    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wl = W.workload_c5()
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, wl.disc.P, wl.disc.M) for s in wl.systems]
    dsl, esl = (int(v) for v in args.serving_slots.split(","))
    tens = [[torch.tensor(getattr(s, k), dtype=torch.float64, device=dev) for k in "xyzq"] for s in wl.systems]
    rng = np.random.default_rng(1907017244)
    pos = [np.stack([s.x, s.y, s.z], axis=1).copy() for s in wl.systems]
    n = args.serving_requests
    fractions = (0.25, 0.5, 0.75, 0.9, 1.1)

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

    def summarize(lat_s, kinds, wall):
        lat = np.asarray(lat_s) * 1e3
        kinds = np.asarray(kinds)
        dl, el = lat[kinds == hs.REQ_DELTA], lat[kinds == hs.REQ_ENERGY]
        return {"requests": len(lat), "requests_per_s": len(lat) / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "delta_p50_ms": float(np.percentile(dl, 50)),
                "delta_p99_ms": float(np.percentile(dl, 99)), "energy_p50_ms": float(np.percentile(el, 50)),
                "energy_p99_ms": float(np.percentile(el, 99))}

    # one request sequence for every variant: warm-up (a short stream, then a full burst, so that
    # the device's clocks have settled), the measured burst, then one stream per offered load
    warm, warm_burst, burst_reqs = stream(500), stream(n), stream(n)
    loads = [(f, stream(n), np.cumsum(rng.exponential(1.0, n))) for f in fractions]
    out = {"workload": "512 resident configurations, N log-uniform in [500, 50000], a~U[15,40], kappa~U[0.05,1], "
                       "P=1024, M=1536; 90% single-ion moves (commit p=1/2), 10% fresh FP64 energies",
           "slots": {"moves": dsl, "energies": esl}, "server": []}
    cap_ref = None
    for ewg, prio in ((int(a), int(b)) for a, b in (v.split(":") for v in args.serving_variants.split(","))):
        server = hs.Server(max_batch=512, delta_slots=dsl, energy_slots=esl, energy_workgroups=ewg,
                           move_priority=prio)
        for p, t in zip(plans, tens):
            server.add_system(p, *t)
        torch.cuda.synchronize()
        label = f"energy_workgroups={ewg} move_priority={prio}"
        log(f"bench[serving]: {label}: {len(plans)} systems resident, {server.stats()['memory_used'] / 2**30:.2f} GiB, "
            f"set up in {time.perf_counter() - t0:.1f} s")
        server.run_load(warm, np.zeros(len(warm)))
        server.run_load(warm_burst, np.zeros(n))
        st0 = server.stats()
        res = server.run_load(burst_reqs, np.zeros(n))
        st1 = server.stats()
        assert all(r.status == 0 for r in res)
        burst = summarize([r.t_done - r.t_submit for r in res], [q[0] for q in burst_reqs], max(r.t_done for r in res))
        cap = burst["requests_per_s"]
        cap_ref = cap if cap_ref is None else cap_ref
        d_out = {"energy_workgroups": ewg, "move_priority": prio, "capacity_requests_per_s": cap, "burst": burst,
                 "mean_batch": (st1["batched_requests"] - st0["batched_requests"]) / max(1, st1["batches"] - st0["batches"]),
                 "loads": []}
        log(f"bench[serving]: {label}: capacity {cap:.0f} req/s (burst)")
        for f, reqs_f, gaps in loads:
            res = server.run_load(reqs_f, gaps / (f * cap))
            assert all(r.status == 0 for r in res)
            d = summarize([r.t_done - r.t_submit for r in res], [q[0] for q in reqs_f], max(r.t_done for r in res))
            d["offered_fraction"] = f
            d["offered_requests_per_s"] = f * cap
            d_out["loads"].append(d)
            log(f"bench[serving]: {label}: load {f:.2f} x {cap:.0f} req/s: p50 {d['p50_ms']:.3f} ms, p99 "
                f"{d['p99_ms']:.3f} ms (moves {d['delta_p50_ms']:.3f} / {d['delta_p99_ms']:.3f} ms, energies "
                f"{d['energy_p50_ms']:.3f} / {d['energy_p99_ms']:.3f} ms)")
        server.close()
        out["server"].append(d_out)
    streams = [(f, r, g / (f * cap_ref)) for f, r, g in loads]
    # the plain per-system path under the same arrival streams: each request alone, synchronously,
    # on its resident system, in arrival order (a request that arrives while another runs waits)
    systems = [hs.System(p, *t) for p, t in zip(plans, tens)]
    ws = hs.workspace(max(s.workspace_bytes() for s in systems), dev)
    dE = torch.empty(1, dtype=torch.float64, device=dev)
    E1 = torch.empty(1, dtype=torch.float64, device=dev)
    plain = {"loads": []}
    for f, reqs_f, arrival in streams:
        m = min(n, 2000)  # bounded: the plain path cannot keep up at these rates and its queue grows
        lat, kinds = [], []
        tb = time.perf_counter()
        for (kind, b, commit, k, x, y, z), ta in zip(reqs_f[:m], arrival[:m]):
            while time.perf_counter() - tb < ta:
                pass
            if kind == hs.REQ_DELTA:
                systems[b].delta_energy(k, (x, y, z), out=dE)
                if commit:
                    systems[b].commit(k, (x, y, z))
                torch.cuda.synchronize()
            else:
                systems[b].full_energy(out=E1, ws=ws)
            lat.append(time.perf_counter() - tb - ta)
            kinds.append(kind)
        d = summarize(lat, kinds, time.perf_counter() - tb)
        d["offered_fraction"] = f
        d["offered_requests_per_s"] = f * cap_ref
        plain["loads"].append(d)
        log(f"bench[serving]: per-system path: load {f:.2f}: p50 {d['p50_ms']:.3f} ms, p99 {d['p99_ms']:.3f} ms "
            f"(moves {d['delta_p50_ms']:.3f} / {d['delta_p99_ms']:.3f} ms), first {m} requests")
    # and its unloaded service rate: one synchronous move query at a time on the largest system
    b = int(np.argmax([len(p) for p in pos]))
    lat = []
    for i in range(300):
        k = int(rng.integers(len(pos[b])))
        new = W.random_move(rng, pos[b][k], wl.systems[b].phys.a)
        ta = time.perf_counter()
        systems[b].delta_energy(k, new, out=dE)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ta)
    lat = np.array(lat[20:]) * 1e3
    plain.update({"system_ions": int(len(pos[b])), "delta_requests_per_s_alone": float(1e3 / lat.mean()),
                  "delta_p50_ms_alone": float(np.percentile(lat, 50)), "delta_p99_ms_alone": float(np.percentile(lat, 99))})
    for sysm in systems:
        sysm.close()
    out["per_system_path"] = plain
    return out


if __name__ == "__main__":
    sys.exit(main())
