"""Write f2_thiele.json: the float64 oracle's static stiffness and gyrotropic
rate for two disks of the geometry sweep of Sec. IV.A-B, by the protocol the
library's sweep uses (experiments.thiele_sweep):

* Permalloy, a = 2 nm; R = 30 nm with L = 10 nm and L = 20 nm;
* constrained relaxation (the oracle's relax, constraint over the cells within
  4 lambda_ex of X, tolerance 1e-9) from the vortex ansatz at X = (0, 0) and
  X = (4 nm, 0) (= 2a, the displacement of eq. Ux), both nudged by 1e-3 a;
* kt = 2 (U(x) - U(0)) / x^2 with x the core distance of the displaced
  relaxed state (units of a, energies in J);
* RK4 at dtau = 0.04 from the displaced relaxed state: alpha = 0.02 for 2500
  steps, then alpha = 0 for 25000 steps with the core position sampled every
  250 steps; Omega = slope of the unwrapped azimuth of the samples (rad per
  unit tau), orbit radius = mean distance (nm).
Calls only the oracle and the seeded input generator.

    python tests/golden/make_f2_golden.py      (a few minutes on 8 cores)
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
GEOMS = [(30.0, 10.0), (30.0, 20.0)]
DTAU, N_DAMP, N_FREE, EVERY = 0.04, 2500, 25000, 250


def main():
    t0 = time.time()
    mat = oracle.Material()
    lam = oracle.units.exchange_length(mat) * 1e9
    c = (A_NM / lam) ** 2
    out = {"protocol": __doc__.split("\n\n")[1], "lambda_ex_nm": lam, "c": c, "dtau": DTAU, "n_damp": N_DAMP,
           "n_free": N_FREE, "sample_every": EVERY, "geometries": []}
    for R, L in GEOMS:
        d = oracle.Disk(R, L, A_NM)
        prm = oracle.Params(c=c)
        states, Us, cores = [], [], []
        for X in (0.0, 4.0):
            m0 = torch.tensor(li.vortex_ansatz(d.D, X / A_NM + 1e-3, 1e-3), dtype=torch.float64)
            m, _, it, res, C = relax(m0, d, prm, (X, 0.0), tol=1e-9, max_sweeps=200000, cutoff_nm=4.0 * lam)
            states.append(m)
            Us.append(energy(m, d, prm)[0])
            cores.append(vortex_core_position(m, d, lam))
        x = math.hypot(cores[1][0], cores[1][1]) / A_NM
        kt = 2.0 * (Us[1] - Us[0]) / (x * x)
        m = rk4_step(states[1], d, oracle.Params(alpha=0.02, c=c, dtau=DTAU), N_DAMP)
        free = oracle.Params(alpha=0.0, c=c, dtau=DTAU)
        pos = []
        for s in range(N_FREE // EVERY):
            m = rk4_step(m, d, free, EVERY)
            xc, yc, *_ = vortex_core_position(m, d, lam)
            pos.append((xc, yc))
        pos = np.array(pos)
        t = (np.arange(len(pos)) + 1) * EVERY * DTAU
        ang = np.unwrap(np.arctan2(pos[:, 1], pos[:, 0]))
        om = float(np.polyfit(t, ang, 1)[0])
        out["geometries"].append({"R_nm": R, "L_nm": L, "U0": Us[0], "Ux": Us[1], "x_cells": x, "kt": kt,
                                  "omega": om, "orbit_radius_nm": float(np.hypot(pos[:, 0], pos[:, 1]).mean()),
                                  "revolutions": float(abs(ang[-1] - ang[0]) / (2 * math.pi))})
        print(R, L, out["geometries"][-1], f"{time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "f2_thiele.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
