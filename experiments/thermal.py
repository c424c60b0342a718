"""Thermal vortex statistics and power spectra (Sec. V.A-V.C) on ensembles of
thermal replicas.

For each disk geometry the static stiffness kt comes from constrained
relaxations of the same disk (Sec. IV.B, eq. Ux); every (geometry,
temperature) gets `replicas` independent Heun trajectories (Philox streams
per replica and cell) that start from the vortex relaxed at the centre, all
in one batched persistent launch per sampling interval.  The core position
is sampled between launches, the float64 <m> series on the device at every
`series_every` steps.  After an equilibration fraction:

* radial statistics against eq. r2 (<r^2> = 2 T_eff / kt) and eq. pr (the
  Rayleigh law, with its Kolmogorov distance and a histogram);
* rotational speed V = r |d theta/dt| (azimuth rate over a quarter of the
  Thiele period) against f(V) = p(V/omega)/omega with omega = kt/(2 pi),
  i.e. <V^2> = 2 T_eff kt / (2 pi)^2;
* the mean gyration rate against the static Thiele rate;
* the Bartlett power spectrum of <m_x> (segments through llg_power_spectrum
  on the device, averaged over segments and replicas): the gyrotropic line
  and, in the larger disks, the spin-wave doublet (Sec. V.B).
Units: lengths in a, energies in J = 2AL, time in t0; T_eff = (1 + alpha^2) T
for the paper's noise amplitude.

    python -m experiments.thermal --geom 30:5 --geom 30:10 --temps 150 300 --replicas 16 --tau 250000
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

from experiments.analysis import (angular_momentum_rate, radial_statistics, rayleigh_cdf, ks_distance,
                                  rotational_speeds, stiffness_fit, stiffness_two_point, thiele_rate)
from experiments.common import A_NM, PY, material, relax_batch, segment_spectra
from paper_1207_2192_amd import Disk, LLGParams

F0_GHZ = PY["gamma"] * 2.0 * PY["A"] / ((A_NM * 1e-9) ** 2 * PY["Ms"]) / 1e9   # 1/t0 in GHz


def static_stiffness(geoms, lam, Xs=(0.0, 2.0, 4.0, 6.0, 8.0)):
    R_l = [R for R, L in geoms for _ in Xs]
    L_l = [L for R, L in geoms for _ in Xs]
    X_l = [(X, 0.0) for _ in geoms for X in Xs]
    batch, m, out, U, core = relax_batch(R_l, L_l, X_l, lam)
    res, centred = [], []
    for g in range(len(geoms)):
        rows = slice(g * len(Xs), (g + 1) * len(Xs))
        r = np.hypot(core[rows, 0], core[rows, 1]) / A_NM
        dU = U[rows] - U[rows][0]
        kt, k4 = stiffness_fit(r[1:], dU[1:])
        kt2 = stiffness_two_point(0.0, dU[2], r[2])           # eq. Ux at x = 2a (X = 4 nm)
        res.append(dict(kt=kt, k4=k4, kt_two_point=kt2, r_relaxed_nm=(r * A_NM).tolist(), dU=dU.tolist(),
                        sweeps_max=int(out[rows, 2].max())))
        centred.append(batch.unpack(m, g * len(Xs)).reshape(-1).clone())
    batch.close()
    return res, centred


def run(geoms, temps, *, replicas=16, alpha=0.02, dtau=0.04, tau=250000.0, every=250, series_every=50,
        equil=0.2, seed=20120827, seg=4096, fd_factor=False, log=print):
    t0 = time.perf_counter()
    _, lam = material(10.0)
    stat, centred = static_stiffness(geoms, lam)
    log(f"# static stiffness: " + ", ".join(f"R={R} L={L}: kt={s['kt']:.5f} (two-point {s['kt_two_point']:.5f})"
                                         for (R, L), s in zip(geoms, stat)) + f" ({time.perf_counter() - t0:.1f} s)")
    groups = [(gi, T) for gi in range(len(geoms)) for T in temps]
    R_l, L_l, prms, starts = [], [], [], []
    for gi, T in groups:
        R, L = geoms[gi]
        p, _ = material(L, 0.0, T, alpha)
        p.dtau = dtau
        p.renorm = True
        p.fd_factor = fd_factor
        for _ in range(replicas):
            R_l.append(R)
            L_l.append(L)
            prms.append(p)
            starts.append(centred[gi])
    disk = Disk.batch(R_l, L_l, A_NM)
    m = torch.cat(starts).contiguous()
    disk.autotune(m.clone(), prms, "heun", probe_steps=40)
    nsteps = int(round(tau / dtau)) // every * every
    S = nsteps // every
    per = every // series_every
    cores = torch.empty(S, disk.n, 5, dtype=torch.float64, device="cuda")
    series = torch.empty(S * per, disk.n, 4, dtype=torch.float64, device="cuda")
    t1 = time.perf_counter()
    last = t1
    for s in range(S):
        series[s * per:(s + 1) * per] = disk.heun_series(m, every, prms, series_every, seed=seed, step0=s * every)
        cores[s] = disk.vortex_core_position(m, lam)
        if time.perf_counter() - last > 30.0:
            torch.cuda.synchronize()
            last = time.perf_counter()
            log(f"# {(s + 1) * every} / {nsteps} steps, {last - t1:.0f} s")
    torch.cuda.synchronize()
    disk.check()
    run_s = time.perf_counter() - t1
    log(f"# {nsteps} Heun steps of {disk.n} disks in {run_s:.1f} s ({sum(disk.n_cells) * nsteps / run_s:.3e} "
        f"cell-steps/s, plan {disk.launch_shape()})")
    c = cores.cpu().numpy()
    t = (np.arange(S) + 1) * every * dtau
    first = int(equil * S)
    # spectra of <m_x> on the device: segments of the equilibrated part of every replica
    sx = series[int(equil * S * per):, :, 0].contiguous()
    P, nseg = segment_spectra(sx, seg)
    freqs = np.arange(seg // 2 + 1) / (seg * series_every * dtau)
    # the gyrotropic line from four times longer segments (finer resolution, fewer segments)
    seg_l = 4 * seg
    P_l, nseg_l = segment_spectra(sx, seg_l) if sx.shape[0] >= seg_l else (None, 0)
    freqs_l = np.arange(seg_l // 2 + 1) / (seg_l * series_every * dtau)
    report = {"geometries": [], "alpha": alpha, "dtau": dtau, "tau": nsteps * dtau, "replicas": replicas,
              "sample_every": every, "series_every": series_every, "equilibration_fraction": equil,
              "fd_factor": fd_factor, "run_s": run_s, "cell_steps_per_s": sum(disk.n_cells) * nsteps / run_s,
              "f0_GHz": F0_GHZ}
    for q, (gi, T) in enumerate(groups):
        R, L = geoms[gi]
        cols = slice(q * replicas, (q + 1) * replicas)
        p = prms[q * replicas]
        T_eff = p.temp * (1.0 if fd_factor else 1.0 + alpha ** 2)
        kt = stat[gi]["kt"]
        x, y = c[first:, cols, 0] / A_NM, c[first:, cols, 1] / A_NM
        lost = int((c[first:, cols, 4] < 0.5).sum())
        r = np.hypot(x, y)
        radial = radial_statistics(r, kt, T_eff)
        # rotation: mean azimuth rate, and speeds over a quarter of the Thiele period
        om_thiele = thiele_rate(kt)
        lag = max(1, int(round(0.25 * 2 * math.pi / abs(om_thiele) / (every * dtau))))
        V, w = rotational_speeds(t[first:], x, y, lag)
        om_mean = float(np.mean(w))
        om_L = angular_momentum_rate(t[first:], x, y, 1)
        v2_pred = 2.0 * T_eff * kt / (2 * math.pi) ** 2
        # V = |Omega| r with the r^2-weighted rate (f(V) = p(V/Omega)/Omega), and the raw
        # per-sample speeds r |d theta/dt| over the lag
        VL = abs(om_L) * r
        speed = {"lag_tau": lag * every * dtau, "v2_predicted": v2_pred,
                 "v2_from_rate": float(np.mean(VL ** 2)), "ratio_from_rate": float(np.mean(VL ** 2) / v2_pred),
                 "ks_distance_from_rate": ks_distance(VL, lambda v: rayleigh_cdf(v / abs(om_thiele), kt, T_eff)),
                 "v2_raw": float(np.mean(V ** 2)), "ratio_raw": float(np.mean(V ** 2) / v2_pred),
                 "omega_r2_weighted": om_L, "omega_mean_azimuth_rate": om_mean, "omega_thiele": om_thiele,
                 "omega_ratio": om_L / om_thiele}
        Pq = P[cols].mean(axis=0)
        lo = (freqs > 0) & (freqs < 0.004)
        hi = (freqs > 0.004) & (freqs < 0.02)
        kg = int(np.argmax(np.where(lo, Pq, -1)))
        nu_g, res_g = float(freqs[kg]), float(freqs[1])
        if P_l is not None:
            Pl = P_l[cols].mean(axis=0)
            lo_l = (freqs_l > 0) & (freqs_l < 0.004)
            kl = int(np.argmax(np.where(lo_l, Pl, -1)))
            nu_g, res_g = float(freqs_l[kl]), float(freqs_l[1])
            if 1 <= kl < len(Pl) - 1:          # parabola through the log power of the peak and its neighbours
                a_, b_, c_ = np.log(Pl[kl - 1:kl + 2])
                den = a_ - 2 * b_ + c_
                if den < 0:
                    nu_g = float(freqs_l[kl] + 0.5 * (a_ - c_) / den * freqs_l[1])
        spec = {"segment": seg, "segments_per_replica": nseg, "resolution": float(freqs[1]),
                "gyrotropic_segment": seg_l if P_l is not None else seg, "gyrotropic_resolution": res_g,
                "gyrotropic_peak_nu": nu_g, "gyrotropic_peak_GHz": nu_g * F0_GHZ,
                "gyrotropic_thiele_GHz": abs(om_thiele) / (2 * math.pi) * F0_GHZ,
                "nu": freqs[:int(0.02 / freqs[1]) + 1].tolist(), "power": Pq[:int(0.02 / freqs[1]) + 1].tolist()}
        if hi.any():
            idx = np.where(hi)[0]
            ph = Pq[idx]
            # the two largest local maxima above the gyrotropic band
            loc = [i for i in range(1, len(idx) - 1) if ph[i] >= ph[i - 1] and ph[i] >= ph[i + 1]]
            loc = sorted(loc, key=lambda i: -ph[i])[:2]
            spec["high_peaks_GHz"] = sorted(float(freqs[idx[i]] * F0_GHZ) for i in loc)
        report["geometries"].append({"R_nm": R, "L_nm": L, "T_K": T, "T_scaled": p.temp, "T_eff": T_eff,
                                     "static": stat[gi], "radial": radial, "speed": speed, "spectrum": spec,
                                     "samples": int(r.size), "vortex_lost_samples": lost})
        log(f"# R={R} L={L} T={T} K: <r^2>/pred = {radial['ratio']:.3f}, KS = {radial['ks_distance']:.3f}, "
            f"<V^2>/pred = {speed['ratio_from_rate']:.3f}, Omega/Thiele = {speed['omega_ratio']:.3f}, "
            f"f_G peak {spec['gyrotropic_peak_GHz']:.3f} GHz (Thiele {spec['gyrotropic_thiele_GHz']:.3f}), "
            f"high peaks {spec.get('high_peaks_GHz')}")
    disk.close()
    report["wall_s"] = time.perf_counter() - t0
    return report


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--geom", action="append", default=None, help="R:L in nm (repeatable); default 30:5")
    ap.add_argument("--temps", type=float, nargs="+", default=[300.0])
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--alpha", type=float, default=0.02)
    ap.add_argument("--dtau", type=float, default=0.04)
    ap.add_argument("--tau", type=float, default=250000.0)
    ap.add_argument("--every", type=int, default=250, help="steps between core-position samples")
    ap.add_argument("--series-every", type=int, default=50, help="steps between <m> samples")
    ap.add_argument("--segment", type=int, default=4096)
    ap.add_argument("--equil", type=float, default=0.2)
    ap.add_argument("--fd-factor", action="store_true")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    geoms = [tuple(float(v) for v in g.split(":")) for g in (args.geom or ["30:5"])]
    rep = run(geoms, args.temps, replicas=args.replicas, alpha=args.alpha, dtau=args.dtau, tau=args.tau,
              every=args.every, series_every=args.series_every, equil=args.equil, seg=args.segment,
              fd_factor=args.fd_factor, log=lambda s: print(s, flush=True))
    print(json.dumps(rep), flush=True)
    return rep


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
