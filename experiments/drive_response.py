"""Vortex response to a driven external field (the time-dependent h_ext of
eq. Hmm and eq. Bi).

1. Resonance sweep: the vortex relaxed at the centre of one disk is driven by
   an in-plane field h_ac x-hat sin(2 pi f tau) at `n_freq` frequencies around
   the Thiele gyrotropic frequency kt/(2 pi)^2 (kt from the disk's
   constrained relaxations, Sec. IV.B), every frequency a disk of one ragged
   batch with its own parameters, so the whole sweep is one persistent launch
   per sampling interval.  After `settle` drive periods of the slowest
   frequency, the amplitude of <m_x> (float64 series on the device) over the
   rest of the run gives the response curve; its maximum should sit at the
   gyrotropic frequency.
2. Pulse ring-down: a Gaussian in-plane field pulse displaces the vortex; at
   alpha = 0 afterwards the <m_x> series is transformed on the device
   (llg_power_spectrum) and its peak is the gyrotropic frequency.

    python -m experiments.drive_response [--R 30 --L 10]
prints one JSON report.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from experiments.analysis import stiffness_two_point
from experiments.common import A_NM, PY, material, relax_batch
from paper_1207_2192_amd import Disk, LLGParams, power_spectrum

F0_GHZ = PY["gamma"] * 2.0 * PY["A"] / ((A_NM * 1e-9) ** 2 * PY["Ms"]) / 1e9


def run(R=30.0, L=10.0, *, n_freq=16, span=(0.5, 1.6), h_ac=0.004, alpha=0.05, dtau=0.04, settle=6.0,
        measure=6.0, every=50, log=print):
    t0 = time.perf_counter()
    p0, lam = material(L)
    c = p0.c
    batch, m, out, U, core = relax_batch([R, R], [L, L], [(0.0, 0.0), (4.0, 0.0)], lam)
    x = math.hypot(core[1, 0], core[1, 1]) / A_NM
    kt = stiffness_two_point(U[0], U[1], x)
    centred = batch.unpack(m, 0).reshape(-1).clone()
    batch.close()
    fG = kt / (2 * math.pi) ** 2                       # cycles per unit tau
    freqs = np.linspace(span[0], span[1], n_freq) * fG
    # ---- 1. resonance sweep, one disk per drive frequency
    disk = Disk.batch([R] * n_freq, [L] * n_freq, A_NM)
    mm = centred.repeat(n_freq).contiguous()
    prms = [LLGParams(alpha=alpha, c=c, dtau=dtau, hac=(h_ac, 0.0, 0.0), freq=float(f)) for f in freqs]
    n_settle = int(settle / freqs.min() / dtau) // every * every
    n_meas = int(measure / freqs.min() / dtau) // every * every
    for q in prms:
        q.tau0 = 0.0
    disk.rk4_step(mm, n_settle, prms)
    for q in prms:
        q.tau0 = n_settle * dtau
    ser = disk.rk4_series(mm, n_meas, prms, every)
    disk.check()
    mx = ser[:, :, 0].cpu().numpy()
    amp = 0.5 * (mx.max(axis=0) - mx.min(axis=0))
    k = int(np.argmax(amp))
    sweep = {"f_thiele": fG, "f_thiele_GHz": fG * F0_GHZ, "freqs": freqs.tolist(), "amplitude": amp.tolist(),
             "f_peak": float(freqs[k]), "f_peak_GHz": float(freqs[k] * F0_GHZ), "peak_over_thiele": float(freqs[k] / fG),
             "settle_steps": n_settle, "measure_steps": n_meas}
    log(f"# resonance: peak at {freqs[k] / fG:.3f} x the Thiele frequency ({freqs[k] * F0_GHZ:.3f} GHz), "
        f"{time.perf_counter() - t0:.1f} s")
    disk.close()
    # ---- 2. pulse ring-down at alpha = 0
    one = Disk.build(R, L, A_NM)
    m1 = centred.clone()
    w = 20.0
    pulse = LLGParams(alpha=0.0, c=c, dtau=dtau, hpulse=(0.05, 0.0, 0.0), tpulse=4 * w, wpulse=w)
    n_pulse = int(8 * w / dtau)
    one.rk4_step(m1, n_pulse, pulse)
    N = 1 << 10                                          # 16 periods
    e2 = max(1, int(round(1.0 / (64 * fG * dtau))))     # about 64 samples per gyration period
    n_ring = N * e2
    ring = one.rk4_series(m1, n_ring, LLGParams(alpha=0.0, c=c, dtau=dtau, tau0=n_pulse * dtau), e2)
    one.check()
    P = power_spectrum(ring[:, 0, 0].contiguous(), True, "hann").cpu().numpy()
    nu = np.arange(N // 2 + 1) / (N * e2 * dtau)
    kk = int(np.argmax(P[1:])) + 1
    ringdown = {"sample_every": e2, "samples": N, "resolution": float(nu[1]), "f_peak": float(nu[kk]),
                "f_peak_GHz": float(nu[kk] * F0_GHZ), "peak_over_thiele": float(nu[kk] / fG)}
    log(f"# ring-down: spectral peak at {nu[kk] / fG:.3f} x the Thiele frequency ({nu[kk] * F0_GHZ:.3f} GHz)")
    one.close()
    return {"R_nm": R, "L_nm": L, "kt": kt, "alpha": alpha, "h_ac": h_ac, "sweep": sweep, "ringdown": ringdown,
            "wall_s": time.perf_counter() - t0}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--R", type=float, default=30.0)
    ap.add_argument("--L", type=float, default=10.0)
    ap.add_argument("--n-freq", type=int, default=16)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    rep = run(args.R, args.L, n_freq=args.n_freq, log=lambda s: print(s, flush=True))
    print(json.dumps(rep), flush=True)
    return rep


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
