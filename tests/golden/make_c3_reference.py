"""Write ``c3_reference.json``: the oracle's reaction energy and potentials of the full
N = 10^6 workload (10^6 ions uniform in a cavity of radius 200, a 2:1 mix of +-1 and +-2
charges, eps1 = 1, eps2 = 80, kappa = 0.1, P = 6400 surface nodes, M = 9600 check points,
p = 40; the timing workload of Sec. 4.2 at its largest N).

Only ``oracle`` (O1: HSMA with direct FP64 sums, Algorithm 1) and the seeded input
generator ``workloads`` are called.  The sums take about 10^12 FP64 pairs: some 25 minutes
on 8 host threads.  Stored, with the workload's seed:

* E = 1/2 sum_i q_i Phi_i over all ions, and its Kelvin-image and surface-image parts;
* the L2 norm of Phi over all ions;
* Phi at 2048 ions drawn with a fixed seed;
* four projections sum_i w_i Phi_i with seeded standard-normal weights w, which a wrong
  potential anywhere among the 10^6 ions changes.

Run from the repository root:  python tests/golden/make_c3_reference.py
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c3_reference.json")
SAMPLE_SEED = 20240613
NSAMPLE = 2048
PROJ_SEEDS = (11, 12, 13, 14)
CHUNK = 25_000


def main() -> None:
    t_start = time.time()
    wl = W.workload_c3()
    s = wl.systems[0]
    ph, d = s.phys, wl.disc
    prm = oracle.Params(ph.a, ph.eps1, ph.eps2, ph.kappa, d.p, d.P, d.M, tau=d.tau, rc_over_a=d.rc_over_a)
    n = s.n
    pos = np.stack([s.x, s.y, s.z], axis=1)

    # steps 1-4 once (check fields, fit, surface strengths) with the first chunk of targets
    phi0, dg = oracle.hsma_eval(prm, s.x, s.y, s.z, s.q, targets=pos[:CHUNK], diag=True)
    phi_k = np.zeros(n)
    phi_s = np.zeros(n)
    phi_k[:CHUNK] = dg["kelvin"]
    phi_s[:CHUNK] = phi0 - dg["kelvin"]
    print(f"fit done, first chunk in {time.time() - t_start:.0f} s", flush=True)
    for c0 in range(CHUNK, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        tg = pos[c0:c1]
        phi_k[c0:c1] = oracle.kelvin_potential(prm, s.x, s.y, s.z, s.q, tg)
        phi_s[c0:c1] = oracle.surface_potential(prm, dg["nodes"], dg["Q"], dg["D"], tg)
        print(f"targets {c1}/{n} after {time.time() - t_start:.0f} s", flush=True)
    phi = phi_k + phi_s

    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    idx = np.sort(rng.choice(n, NSAMPLE, replace=False))
    proj = []
    for sd in PROJ_SEEDS:
        w = np.random.Generator(np.random.PCG64(sd)).standard_normal(n)
        proj.append({"seed": sd, "value": math.fsum(w * phi)})
    rec = {
        "workload": wl.name,
        "recipe": "workloads.workload_c3(): seed 1907017240 + 2, N = 10^6 uniform in a = 200, "
                  "charges +-1/+-2 in a 2:1 mix, eps1 = 1, eps2 = 80, kappa = 0.1",
        "N": n, "a": ph.a, "eps1": ph.eps1, "eps2": ph.eps2, "kappa": ph.kappa,
        "P": d.P, "M": d.M, "p": d.p, "tau": d.tau, "rc_over_a": d.rc_over_a, "F1": prm.f1(),
        "oracle": "O1 (oracle/hsma_oracle.c), FP64 direct sums; final sums by math.fsum",
        "E": 0.5 * math.fsum(s.q * phi),
        "E_kelvin": 0.5 * math.fsum(s.q * phi_k),
        "E_surface": 0.5 * math.fsum(s.q * phi_s),
        "phi_l2": math.sqrt(math.fsum(phi * phi)),
        "sample_seed": SAMPLE_SEED,
        "sample_idx": [int(i) for i in idx],
        "sample_phi": [float(v) for v in phi[idx]],
        "projections": proj,
        "threads": oracle.num_threads(),
        "seconds": round(time.time() - t_start, 1),
    }
    with open(OUT + ".tmp", "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT}: E = {rec['E']!r} in {rec['seconds']} s", flush=True)


if __name__ == "__main__":
    main()
