"""Write f2_stability.json: the float64 oracle's view of the minimum thickness
for a stable vortex (Sec. IV.A-B, Fig. f-v-LoR), by the protocol of
experiments.thiele_sweep.stability_scan:

* Permalloy, a = 2 nm; R = 30 nm with L = 2 nm (below the minimum thickness)
  and L = 5 nm (above it);
* static: constrained relaxations (the oracle's relax, constraint over the
  cells within 4 lambda_ex of X, tolerance 1e-9) from the vortex ansatz at
  X = (0, 0) and X = (4 nm, 0), both nudged by 1e-3 a; kt = 2 (U(x) - U(0))
  / x^2 with x the core distance of the displaced state (units of a);
* dynamic: a vortex relaxed at X = (R/2, 0) = (15 nm, 0), released with
  alpha = 0.02 (RK4, dtau = 0.04) for 50000 steps (tau = 2000) with the core
  position sampled every 500 steps: the least-squares slope of its distance
  from the centre (nm per unit tau) over the samples where a +1 vortex is
  found, the first and last such distance, and whether the vortex is found in
  every sample.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_f2_stability_golden.py      (several minutes on 8 cores)
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402
import torch  # noqa: E402

import llg_inputs as li  # noqa: E402
import oracle  # noqa: E402
from oracle.dynamics import rk4_step  # noqa: E402
from oracle.observables import energy, vortex_core_position  # noqa: E402
from oracle.relax import relax  # noqa: E402

A_NM = 2.0
GEOMS = [(30.0, 2.0), (30.0, 5.0)]
DTAU, N_STEPS, EVERY = 0.04, 50000, 500


def relaxed(d, prm, X, lam):
    m0 = torch.tensor(li.vortex_ansatz(d.D, X / A_NM + 1e-3, 1e-3), dtype=torch.float64)
    m, *_ = relax(m0, d, prm, (X, 0.0), tol=1e-9, max_sweeps=200000, cutoff_nm=4.0 * lam)
    return m


def main():
    t0 = time.time()
    mat = oracle.Material()
    lam = oracle.units.exchange_length(mat) * 1e9
    c = (A_NM / lam) ** 2
    out = {"protocol": __doc__.split("\n\n")[1], "lambda_ex_nm": lam, "c": c, "dtau": DTAU, "n_steps": N_STEPS,
           "sample_every": EVERY, "geometries": []}
    for R, L in GEOMS:
        d = oracle.Disk(R, L, A_NM)
        prm = oracle.Params(c=c)
        Us, cores = [], []
        for X in (0.0, 4.0):
            m = relaxed(d, prm, X, lam)
            Us.append(energy(m, d, prm)[0])
            cores.append(vortex_core_position(m, d, lam))
        x = math.hypot(cores[1][0], cores[1][1]) / A_NM
        kt = 2.0 * (Us[1] - Us[0]) / (x * x)
        m = relaxed(d, prm, R / 2, lam)
        c0 = vortex_core_position(m, d, lam)
        dyn = oracle.Params(alpha=0.02, c=c, dtau=DTAU)
        t, rad, found = [], [], []
        for s in range(N_STEPS // EVERY):
            m = rk4_step(m, d, dyn, EVERY)
            xc, yc, _, _, flag = vortex_core_position(m, d, lam)
            t.append((s + 1) * EVERY * DTAU)
            rad.append(math.hypot(xc, yc))
            found.append(flag > 0)
        t, rad, found = np.array(t), np.array(rad), np.array(found)
        drift = float(np.polyfit(t[found], rad[found], 1)[0]) if found.sum() >= 2 else None
        out["geometries"].append({"R_nm": R, "L_nm": L, "U0": Us[0], "Ux": Us[1], "x_cells": x, "kt": kt,
                                  "start_radius_nm": float(math.hypot(c0[0], c0[1])),
                                  "drift_nm_per_tau": drift,
                                  "end_radius_nm": float(rad[found][-1]) if found.any() else None,
                                  "vortex_kept": bool(found.all())})
        print(R, L, out["geometries"][-1], f"{time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "f2_stability.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
