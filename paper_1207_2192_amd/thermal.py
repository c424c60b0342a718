"""Thermal vortex statistics of an ensemble of replicas (Sec. V-VI of the paper).

Runs `replicas` independent Heun trajectories of one Permalloy disk at
temperature T in one persistent launch per sample interval, records the vortex
core position of every replica every `sample_every` steps, and compares, after
an equilibration fraction, the core-radius and core-speed statistics with the
Boltzmann forms of a harmonic potential U = kt r^2/2 whose stiffness kt comes
from constrained relaxations of the same disk (static fit of U(r), Sec. IV.B):

  <r^2> = 2 T_eff / kt,   p(r) = (kt/T_eff) r exp(-kt r^2 / (2 T_eff)),
  speed V = Omega r with Omega = kt/(2 pi)  ->  <V^2> = 2 T_eff kt / (2 pi)^2,

in simulation units (lengths in a, energies in J = 2AL, time in t0), with
T_eff = (1 + alpha^2) T for the paper's noise amplitude (or T with the FD
factor).  Everything runs in lib_llgdisk; numpy only reduces the samples.

    python -m paper_1207_2192_amd.thermal --replicas 64 --steps 500000
prints progress lines and one JSON report.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

import llg_inputs as li

from .api import Disk, LLGParams, params_from_si


def static_stiffness(R, L, a, c, lam, Xs, tol=2e-6):
    """kt, k4 from U(r) - U(0) = kt r^2/2 + k4 r^4/4 over relaxed core positions (r in a)."""
    batch = Disk.batch([R] * len(Xs), [L] * len(Xs), a)
    D = batch.D[0]
    m = batch.pack([torch.tensor(li.vortex_ansatz(D, X / a + 1e-3, 1e-3), dtype=torch.float32, device="cuda")
                    .reshape(-1) for X in Xs])
    p = LLGParams(c=c)
    out = batch.relax(m, [(X, 0.0) for X in Xs], p, tol=tol, max_sweeps=400000, cutoff_nm=4 * lam).cpu()
    batch.check()
    U = batch.energy(m, p).cpu()[:, 0].double().numpy()
    core = batch.vortex_core_position(m, lam).cpu().double().numpy()
    r = np.hypot(core[:, 0], core[:, 1]) / a
    A = np.stack([0.5 * r[1:] ** 2, 0.25 * r[1:] ** 4], axis=1)
    kt, k4 = np.linalg.lstsq(A, U[1:] - U[0], rcond=None)[0]
    return float(kt), float(k4), r, U - U[0], out[:, 2].numpy()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--R", type=float, default=250.0)
    ap.add_argument("--L", type=float, default=20.0)
    ap.add_argument("--a", type=float, default=2.0)
    ap.add_argument("--T", type=float, default=300.0)
    ap.add_argument("--alpha", type=float, default=0.1)
    ap.add_argument("--dt", type=float, default=0.02, help="time step (ps)")
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--steps", type=int, default=500000)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--equil", type=float, default=0.4, help="fraction of the run discarded as equilibration")
    ap.add_argument("--seed", type=int, default=20120827)
    ap.add_argument("--fd-factor", action="store_true")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    PY = li.PERMALLOY
    p, lam = params_from_si(PY["A"], PY["Ms"], PY["gamma"], args.a, args.L, args.dt, args.T, args.alpha)
    p.renorm = True
    p.fd_factor = args.fd_factor
    t0 = time.perf_counter()
    Xs = [0.0, 2.0, 4.0, 6.0, 8.0, 10.0]
    kt, k4, r_rel, dU, sweeps = static_stiffness(args.R, args.L, args.a, p.c, lam, Xs)
    print(f"# static fit: kt = {kt:.6f}, k4 = {k4:.3e} (relaxed cores at {np.round(r_rel * args.a, 3)} nm, "
          f"{int(sweeps.max())} sweeps, {time.perf_counter() - t0:.1f} s)", flush=True)

    n = args.replicas
    disk = Disk.batch([args.R] * n, [args.L] * n, args.a)
    D = disk.D[0]
    m = torch.tensor(np.concatenate([li.vortex_ansatz(D, 0.01, 0.013).reshape(-1)] * n), dtype=torch.float32,
                     device="cuda")
    prms = [p] * n
    disk.autotune(m.clone(), prms, "heun", probe_steps=20)
    k = args.sample_every
    n_samp = args.steps // k
    samples = torch.empty(n_samp, n, 2, dtype=torch.float64, device="cuda")
    t1 = time.perf_counter()
    for s in range(n_samp):
        disk.heun_step(m, k, prms, seed=args.seed, step0=s * k, replica=0)
        samples[s] = disk.vortex_core_position(m, lam)[:, :2]
        if (s + 1) % max(1, n_samp // 20) == 0:
            torch.cuda.synchronize()
            print(f"# {(s + 1) * k} steps, {time.perf_counter() - t1:.1f} s", flush=True)
    torch.cuda.synchronize()
    disk.check()
    run_s = time.perf_counter() - t1
    xy = samples.cpu().numpy() / args.a                       # [n_samp, n, 2] in a
    first = int(args.equil * n_samp)
    eq = xy[first:]
    r = np.hypot(eq[..., 0], eq[..., 1]).ravel()
    # core speed from displacements over `lag` samples: short lags see the thermal jitter of
    # the core position, long lags the gyrotropic drift
    speeds = {}
    for lag in (1, 10, 50):
        if eq.shape[0] > lag:
            d = (eq[lag:] - eq[:-lag]) / (lag * k * p.dtau)
            speeds[lag] = np.hypot(d[..., 0], d[..., 1]).ravel()
    T_eff = p.temp * (1.0 if args.fd_factor else 1.0 + args.alpha ** 2)
    r2_pred = 2.0 * T_eff / kt
    v2_pred = 2.0 * T_eff * kt / (2.0 * math.pi) ** 2
    # Kolmogorov distance of r against the Rayleigh law F(r) = 1 - exp(-kt r^2 / (2 T_eff))
    rs = np.sort(r)
    F = 1.0 - np.exp(-kt * rs ** 2 / (2.0 * T_eff))
    emp = np.arange(1, rs.size + 1) / rs.size
    ks = float(np.max(np.abs(emp - F)))
    hist, edges = np.histogram(r, bins=12, range=(0.0, 3.0 * math.sqrt(r2_pred)), density=True)
    mid = 0.5 * (edges[1:] + edges[:-1])
    pr = kt / T_eff * mid * np.exp(-kt * mid ** 2 / (2.0 * T_eff))
    report = {
        "disk": {"R_nm": args.R, "L_nm": args.L, "a_nm": args.a, "D": D, "cells": disk.n_cells[0]},
        "ensemble": {"replicas": n, "steps": args.steps, "sample_every": k, "T_K": args.T, "alpha": args.alpha,
                     "dtau": p.dtau, "T_scaled": p.temp, "T_eff": T_eff, "equilibration_fraction": args.equil},
        "static": {"kt": kt, "k4": k4, "relaxed_core_nm": (r_rel * args.a).tolist(), "dU": dU.tolist()},
        "radius": {"r2_measured_a2": float(np.mean(r ** 2)), "r2_predicted_a2": r2_pred,
                   "ratio": float(np.mean(r ** 2) / r2_pred), "ks_distance_rayleigh": ks,
                   "hist_r_a": mid.tolist(), "hist_p_measured": hist.tolist(), "hist_p_boltzmann": pr.tolist()},
        "speed": {"v2_gyrotropic_predicted": v2_pred,
                  "by_lag": {str(lag * k): {"v2_measured": float(np.mean(v ** 2)),
                                            "ratio": float(np.mean(v ** 2) / v2_pred)}
                             for lag, v in speeds.items()}},
        "timing": {"run_s": run_s, "cell_steps_per_s": disk.n_cells[0] * n * args.steps / run_s},
    }
    print(json.dumps(report), flush=True)
    return report


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
