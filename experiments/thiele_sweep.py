"""Static stiffness and gyrotropic frequency over disk geometries (Sec. IV.A-B).

For every (R, L) of the sweep, one ragged batch relaxes the vortex with its
core held at the centre and at x = 2a (and at further points for a fit),
giving k_F from eq. Ux; a second ragged batch releases the vortices relaxed at
(2a, 0) with alpha = 0.02 until tau = 1000, then at alpha = 0, and the
gyrotropic rate is the slope of the unwrapped azimuth of the core over the
following periods (the paper's procedure).  Reported per geometry: k_F/L in
units of A/a^2 (= 2 kt), Omega_G measured and the Thiele value kt/(2 pi) of
eq. OG, f_G in GHz for Permalloy; and over the sweep the slope of k_F/L
against L/R (eq. kFlinear: about 1/4) and of |Omega_G| against kt/(2 pi)
(unit slope, Fig. nu-v-kFoL).

The stability scan (--stability) probes the minimum thickness for a stable
vortex (Fig. f-v-LoR: f_G falls to zero there) over thinner films: the sign of
the static stiffness from relaxations at 0 and 2a, and the paper's dynamic
check — a vortex relaxed near half the radius, released with alpha = 0.02,
must move the way the Thiele equation gives for a restoring force (spiral
inwards) — reported as the radial drift of the core and whether it is kept.

    python -m experiments.thiele_sweep [--quick] [--stability]
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

from experiments.analysis import gyration_rate, stiffness_fit, stiffness_two_point, thiele_rate
from experiments.common import A_NM, PY, material, relax_batch, sample_cores
from paper_1207_2192_amd import Disk, LLGParams

RADII = [30.0, 60.0, 90.0, 120.0]
F0_GHZ = PY["gamma"] * 2.0 * PY["A"] / ((A_NM * 1e-9) ** 2 * PY["Ms"]) / 1e9   # 1/t0 in GHz
THICK = [5.0, 10.0, 20.0]


def run(geoms, *, dtau=0.04, tau_damped=1000.0, periods=6.0, max_steps=1_200_000, every=250, extra_X=(4.0, 8.0),
        n_free=None, autotune=True, log=print):
    t0 = time.perf_counter()
    _, lam = material(10.0)
    n = len(geoms)
    # ---- static: U at X = 0, 2a and further points, one ragged batch
    Xs = [0.0, 2 * A_NM] + [x for x in extra_X if x != 2 * A_NM]
    R_l, L_l, X_l = [], [], []
    for R, L in geoms:
        for X in Xs:
            R_l.append(R)
            L_l.append(L)
            X_l.append((X, 0.0))
    batch, m, out, U, core = relax_batch(R_l, L_l, X_l, lam)
    log(f"# relaxed {len(R_l)} states, max sweeps {int(out[:, 2].max())}, max residual {out[:, 3].max():.1e} "
        f"({time.perf_counter() - t0:.1f} s)")
    res = []
    starts = []
    for g, (R, L) in enumerate(geoms):
        rows = slice(g * len(Xs), (g + 1) * len(Xs))
        Ug, cg = U[rows], core[rows]
        r = np.hypot(cg[:, 0], cg[:, 1]) / A_NM
        kt2 = stiffness_two_point(Ug[0], Ug[1], r[1])
        kt, k4 = stiffness_fit(r[1:], Ug[1:] - Ug[0])
        res.append(dict(R_nm=R, L_nm=L, L_over_R=L / R, kt_two_point=kt2, kt_fit=kt, k4_fit=k4,
                        kF_over_L=2.0 * kt2, core_at_2a_nm=float(r[1] * A_NM), vortex_found=bool(cg[1, 4] > 0),
                        relax_sweeps=int(out[g * len(Xs) + 1, 2]), relax_residual=float(out[g * len(Xs) + 1, 3])))
        starts.append(batch.unpack(m, g * len(Xs) + 1).reshape(-1).clone())
    batch.close()
    # ---- dynamics: all geometries in one ragged batch from their relaxed (2a, 0) states
    dyn = Disk.batch([R for R, _ in geoms], [L for _, L in geoms], A_NM)
    mdyn = torch.cat(starts).contiguous()
    cs = [material(L)[0].c for _, L in geoms]
    kmin = min(max(r["kt_two_point"], 1e-4) for r in res)
    tauG = 4 * math.pi ** 2 / kmin
    n_damp = int(round(tau_damped / dtau))
    if n_free is None:
        n_free = min(max_steps, int(periods * tauG / dtau) // every * every)
    damped = [LLGParams(alpha=0.02, c=c, dtau=dtau) for c in cs]
    free = [LLGParams(alpha=0.0, c=c, dtau=dtau) for c in cs]
    if autotune:
        dyn.autotune(mdyn.clone(), free, "rk4", probe_steps=100)
    dyn.rk4_step(mdyn, n_damp, damped)
    t1 = time.perf_counter()
    t, cores = sample_cores(dyn, mdyn, n_free, every, lambda s0, k: dyn.rk4_step(mdyn, k, free), lam)
    log(f"# {n_damp} damped + {n_free} free RK4 steps of {n} disks in {time.perf_counter() - t1:.1f} s "
        f"(plan {dyn.launch_shape()})")
    tt = t * dtau
    for g, r in enumerate(res):
        x, y, found = cores[:, g, 0] / A_NM, cores[:, g, 1] / A_NM, cores[:, g, 4]
        r["vortex_kept"] = bool(found.min() > 0)
        if r["vortex_kept"] and r["vortex_found"]:
            om, rad, rev = gyration_rate(tt, x, y)
            r.update(omega_measured=om, orbit_radius_nm=rad * A_NM, revolutions=rev,
                     omega_thiele=thiele_rate(r["kt_two_point"]), ratio=om / thiele_rate(r["kt_two_point"]),
                     fG_GHz=abs(om) / (2 * math.pi) * F0_GHZ)
        else:
            r.update(omega_measured=None, ratio=None)
    dyn.close()
    ok = [r for r in res if r.get("ratio") is not None and r["revolutions"] > 1.0]
    summary = {}
    if len(ok) >= 3:
        lr = np.array([r["L_over_R"] for r in ok])
        kl = np.array([r["kF_over_L"] for r in ok])
        summary["kF_over_L_vs_L_over_R_slope"] = float(np.polyfit(lr, kl, 1)[0])
        thin = lr <= 0.2
        if thin.sum() >= 3:        # the range where eq. kFlinear is meant to hold
            summary["kF_over_L_vs_L_over_R_slope_LR_le_0.2"] = float(np.polyfit(lr[thin], kl[thin], 1)[0])
        kx = np.array([-r["omega_thiele"] for r in ok])
        ky = np.array([-r["omega_measured"] for r in ok])
        summary["omega_vs_thiele_slope_through_0"] = float((kx * ky).sum() / (kx * kx).sum())
    return {"geometries": res, "summary": summary, "dtau": dtau, "tau_damped": tau_damped,
            "free_steps": n_free, "sample_every": every, "wall_s": time.perf_counter() - t0}


def stability_scan(geoms, *, dtau=0.04, tau=4000.0, every=500, start_frac=0.5, log=print):
    """Per (R, L): the two-point stiffness kt (eq. Ux) of relaxations at 0 and 2a, and
    the radial drift of a vortex relaxed at (start_frac R, 0) and released with
    alpha = 0.02 for tau: the least-squares slope of r(t) over the run (nm per unit
    tau), the first and last core radius, and whether a +1 vortex is still found."""
    t0 = time.perf_counter()
    _, lam = material(10.0)
    n = len(geoms)
    R_l = [R for R, _ in geoms for _ in (0, 1)]
    L_l = [L for _, L in geoms for _ in (0, 1)]
    X_l = [(X, 0.0) for _ in geoms for X in (0.0, 2 * A_NM)]
    batch, m, out, U, core = relax_batch(R_l, L_l, X_l, lam)
    batch.close()
    res = []
    for g, (R, L) in enumerate(geoms):
        r1 = math.hypot(core[2 * g + 1, 0], core[2 * g + 1, 1]) / A_NM
        res.append(dict(R_nm=R, L_nm=L, L_over_R=L / R, kt_two_point=stiffness_two_point(U[2 * g], U[2 * g + 1], r1),
                        vortex_found_static=bool(core[2 * g, 4] > 0 and core[2 * g + 1, 4] > 0),
                        relax_residual=float(max(out[2 * g, 3], out[2 * g + 1, 3]))))
    log(f"# static: {2 * n} relaxations ({time.perf_counter() - t0:.1f} s)")
    # dynamic check from a vortex relaxed near half the radius
    starts = [(start_frac * R, 0.0) for R, _ in geoms]
    batch, m, out, U, core0 = relax_batch([R for R, _ in geoms], [L for _, L in geoms], starts, lam)
    prm = [LLGParams(alpha=0.02, c=material(L)[0].c, dtau=dtau) for _, L in geoms]
    nsteps = int(round(tau / dtau)) // every * every
    t1 = time.perf_counter()
    t, cores = sample_cores(batch, m, nsteps, every, lambda s0, k: batch.rk4_step(m, k, prm), lam)
    log(f"# dynamic: {nsteps} damped RK4 steps of {n} disks from r = {start_frac} R "
        f"({time.perf_counter() - t1:.1f} s)")
    batch.close()
    tt = t * dtau
    for g, r in enumerate(res):
        found = cores[:, g, 4] > 0
        rad = np.hypot(cores[:, g, 0], cores[:, g, 1])
        r["start_radius_nm"] = float(math.hypot(core0[g, 0], core0[g, 1]))
        r["vortex_kept"] = bool(found.all())
        if found.sum() >= 2:
            slope = float(np.polyfit(tt[found], rad[found], 1)[0])
            r.update(drift_nm_per_tau=slope, end_radius_nm=float(rad[found][-1]))
        else:
            r.update(drift_nm_per_tau=None, end_radius_nm=None)
        r["stable"] = bool(r["kt_two_point"] > 0 and r["vortex_kept"] and (r["drift_nm_per_tau"] or 0.0) < 0.0)
    return {"geometries": res, "dtau": dtau, "tau": tau, "start_frac": start_frac,
            "wall_s": time.perf_counter() - t0}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="two radii only, shorter runs")
    ap.add_argument("--periods", type=float, default=6.0)
    ap.add_argument("--stability", action="store_true",
                    help="scan thinner films (L = 1..5 nm) for the minimum thickness of a stable vortex")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.stability:
        geoms = [(R, L) for R in RADII for L in (1.0, 2.0, 3.0, 4.0, 5.0)]
        rep = stability_scan(geoms, log=lambda s: print(s, flush=True))
        for r in rep["geometries"]:
            print(f"# R={r['R_nm']:.0f} L={r['L_nm']:.0f}: kt={r['kt_two_point']:.5f} drift={r['drift_nm_per_tau']} "
                  f"r {r['start_radius_nm']:.1f} -> {r['end_radius_nm']} kept={r['vortex_kept']} "
                  f"stable={r['stable']}", flush=True)
        print(json.dumps(rep), flush=True)
        return rep
    geoms = [(R, L) for R in RADII for L in THICK]
    if args.quick:
        geoms = [(30.0, 10.0), (30.0, 20.0), (60.0, 20.0)]
    rep = run(geoms, periods=args.periods, log=lambda s: print(s, flush=True))
    print(json.dumps(rep), flush=True)
    return rep


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
