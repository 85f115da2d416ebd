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
timed region; the oracle is also timed on the host cores (cpu_baseline).
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

# Derived ALU ceiling of the evaluation kernel (pairs/s): 256 CUs x 4 SIMDs x 16 lanes
# issue 256*64 lane-instructions per cycle at 2.4 GHz.  A Kelvin pair needs 7 full-rate
# FP32 VALU instructions (3 sub, 1 mul, 2 fma for |d|^2, 1 fma to accumulate) and one
# v_rsq_f32, a transcendental issued at a quarter of the full rate (4 slots).
CU, LANES, CLOCK = 256, 64, 2.4e9
ISSUE_RATE = CU * LANES * CLOCK              # lane-instructions / s
SLOTS_PER_PAIR = 7 + 4                        # full-rate + transcendental
PEAK_PAIRS = ISSUE_RATE / SLOTS_PER_PAIR      # 3.57e12 pairs / s


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32c", choices=["fp32", "fp32c", "fp64"])
    ap.add_argument("--no-oracle", action="store_true", help="skip the accuracy check and the CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-stage HIP events")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        return 2

    import numpy as np
    import torch

    import paper_1907_01724_amd as hs
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload_c2()
    d = wl.disc
    systems = wl.systems
    s0 = systems[0]
    N = s0.n
    x, y, z, q = (torch.tensor(v, dtype=torch.float64, device=dev) for v in (s0.x, s0.y, s0.z, s0.q))
    plans = [hs.Plan(s.phys.a, s.phys.eps1, s.phys.eps2, s.phys.kappa, d.P, d.M, pair_prec=args.prec)
             for s in systems]
    phis = [torch.empty(N, dtype=torch.float64, device=dev) for _ in plans]
    Es = [torch.empty(1, dtype=torch.float64, device=dev) for _ in plans]
    wss = [hs.workspace(p.workspace_bytes(N), dev) for p in plans]
    stream = torch.cuda.current_stream()
    inf = plans[0].info
    M, P = inf["M"], inf["P"]
    pairs_check = N * M
    pairs_kelvin = N * (N - 1)
    pairs_surface = N * P
    pairs_sys = pairs_check + pairs_kelvin + pairs_surface
    pairs_step = pairs_sys * len(plans)

    def step():
        for p, ph, e, w in zip(plans, phis, Es, wss):
            p.energy(x, y, z, q, phi=ph, E=e, stream=stream, ws=w[1])

    log(f"bench: workload {wl.name}, N={N}, P={P}, M={M}, p={inf['p']}, prec={args.prec}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for p in plans:
        assert p.stream_check() == 0
    if not args.no_profile:
        for p in plans:
            p.profile(True)
            p.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    stages = {}
    if not args.no_profile:
        for p in plans:
            for k, (t, c) in p.profile_read().items():
                a = stages.setdefault(k, [0.0, 0])
                a[0] += t
                a[1] += c
            p.profile(False)
    log(f"bench: {ms:.4f} ms/step over {args.steps} steps")

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
        "systems_per_s": len(plans) / (ms * 1e-3),
    }
    if stages:
        ev_ms, ev_n = stages["eval"]
        avg = ev_ms / max(ev_n, 1) * 1e-3
        eval_pairs = pairs_kelvin + pairs_surface
        achieved = eval_pairs / avg
        out["roofline"] = {
            "bound": "alu",
            "kernel": "k_eval (evaluation pair sums)",
            "achieved": achieved / 1e9,
            "peak": PEAK_PAIRS / 1e9,
            "unit": "Gpair/s",
            "frac": achieved / PEAK_PAIRS,
            "traffic": None,
            "avg_launch_ms": avg * 1e3,
            "peak_model": "256 CU x 64 lanes x 2.4 GHz / (7 VALU + 4-slot v_rsq_f32) per pair",
        }
        out["stage_ms_per_step"] = {k: v[0] / args.steps for k, v in stages.items()}

    if not args.no_oracle:
        import oracle
        worst_phi, worst_e = 0.0, 0.0
        for p, ph, e, s in zip(plans, phis, Es, systems):
            i = p.info
            prm = oracle.Params(a=i["a"], eps1=i["eps1"], eps2=i["eps2"], kappa=i["kappa"], p=i["p"], P=i["P"],
                                M=i["M"], tau=i["tau"], rc_over_a=i["rc"] / i["a"], F1=i["F1"])
            t2 = time.perf_counter()
            ref = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q)
            t3 = time.perf_counter()
            got = ph.cpu().numpy()
            worst_phi = max(worst_phi, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
            e_ref = oracle.energy(s.q, ref)
            worst_e = max(worst_e, abs(float(e.cpu().numpy()[0]) - e_ref) / abs(e_ref))
            if "cpu_baseline" not in out:
                out["cpu_baseline"] = {
                    "value": pairs_sys / (t3 - t2) / 1e9,
                    "unit": "GPairs/s",
                    "cores": oracle.num_threads(),
                    "kind": "oracle",
                    "sample": "one of the four parameter sets (eps1=80, eps2=80, kappa=0.05), all N ions: "
                              "FP64 direct check sums, Householder least squares, Kelvin and surface sums",
                    "seconds": t3 - t2,
                }
        out["rel_err_phi_l2_max"] = worst_phi
        out["rel_err_energy_max"] = worst_e
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
