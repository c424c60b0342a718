"""Write c2_thiele.json: the float64 oracle's static potential and free
gyration of the gyrotropic disk (Permalloy R = 100 nm, L = 20 nm, a = 2 nm;
D = 100, FFT 256):

* constrained relaxation (the oracle's relax, constraint over the cells within
  4 lambda_ex of X, tolerance 1e-8) from the vortex ansatz at X = (x, 0) for
  x = 0, 2, ..., 20 nm, each nudged by 1e-3 a;
* U(X) - U(0) (units of J) and the relaxed core distances r (units of a), and
  the least-squares fit U - U(0) = kt r^2/2 + k4 r^4/4 (Sec. IV.B, eq. Ux);
* RK4 at alpha = 0, dtau = 0.04 from the state relaxed at X = 10 nm, 2000
  steps, the core position every 100 steps.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_c2_golden.py       (long: tens of minutes on 8 cores)
"""
from __future__ import annotations

import json
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

A_NM, R_NM, L_NM = 2.0, 100.0, 20.0
XS = [2.0 * k for k in range(11)]


def main():
    t0 = time.time()
    lam = oracle.units.exchange_length(oracle.Material()) * 1e9
    c = (A_NM / lam) ** 2
    d = oracle.Disk(R_NM, L_NM, A_NM)
    prm = oracle.Params(c=c)
    rs, Us, sweeps, state10 = [], [], [], None
    for X in XS:
        m0 = torch.tensor(li.vortex_ansatz(d.D, X / A_NM + 1e-3, 1e-3), dtype=torch.float64)
        m, _, it, res, C = relax(m0, d, prm, (X, 0.0), tol=1e-8, max_sweeps=400000, cutoff_nm=4.0 * lam)
        xc, yc, *_ = vortex_core_position(m, d, lam)
        rs.append(float(np.hypot(xc, yc) / A_NM))
        Us.append(energy(m, d, prm)[0])
        sweeps.append(int(it))
        if X == 10.0:
            state10 = m
        print(f"X = {X} nm: r = {rs[-1] * A_NM:.4f} nm, U = {Us[-1]:.10f}, {it} sweeps, res {res:.1e}, "
              f"{time.time() - t0:.0f} s", flush=True)
    r = np.array(rs)
    dU = np.array(Us) - Us[0]
    A = np.stack([0.5 * r[1:] ** 2, 0.25 * r[1:] ** 4], axis=1)
    kt, k4 = np.linalg.lstsq(A, dU[1:], rcond=None)[0]
    free = oracle.Params(alpha=0.0, c=c, dtau=0.04)
    m = state10
    path = []
    for s in range(20):
        m = rk4_step(m, d, free, 100)
        xc, yc, *_ = vortex_core_position(m, d, lam)
        path.append([xc, yc])
    print(f"kt = {kt:.6f}, k4 = {k4:.4e}, path done {time.time() - t0:.0f} s", flush=True)
    out = {"protocol": __doc__.split("\n\n")[1], "lambda_ex_nm": lam, "c": c, "X_nm": XS, "r_cells": rs,
           "dU": dU.tolist(), "sweeps": sweeps, "kt": float(kt), "k4": float(k4), "dtau": 0.04,
           "path_every": 100, "path_nm": path}
    with open(os.path.join(HERE, "c2_thiele.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
