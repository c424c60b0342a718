"""Thermal statistics of Sec. V (experiments.thermal) on the GPU.

* Pathwise parity of the thermal ensembles: the campaign geometries (R = 30 nm
  with L = 5 and 10 nm, R = 120 nm with L = 20 nm) at 150 K and 300 K,
  alpha = 0.02, dtau = 0.04, one ragged batch with one Philox stream per disk,
  against the float64 oracle's Heun steps of each disk.
* Boltzmann statistics at a short, stated horizon: 64 replicas of the
  R = 30 nm, L = 5 nm disk at 300 K, started from the centred relaxed vortex,
  with strong damping (alpha = 0.5, noise with the fluctuation-dissipation
  factor so that equilibrium is at T) so that the gyration amplitude
  equilibrates within about 700 tau: 1e4 tau (2.5e5 steps), the first 40 %
  discarded.  <r^2> must lie within 25 % of 2T/kt (eq. r2; kt from the
  disk's own relaxations at T = 0, which the thermal softening the paper
  reports lowers by some 10 %) and the radial distribution within a
  Kolmogorov distance of 0.15 of the Rayleigh law of eq. pr (about 300
  effectively independent samples; the samples are correlated, so no p-value
  is claimed)."""
import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.dynamics import heun_step as o_heun

pytestmark = pytest.mark.gpu


def test_thermal_ensembles_match_oracle_pathwise():
    from experiments.common import material
    from paper_1207_2192_amd import Disk
    geoms = [(30.0, 5.0), (30.0, 10.0), (120.0, 20.0)]
    entries = [(R, L, T) for R, L in geoms for T in (150.0, 300.0)]
    disk = Disk.batch([e[0] for e in entries], [e[1] for e in entries])
    starts = [li.vortex_ansatz(D, 1.5, -0.5) for D in disk.D]
    m = torch.tensor(np.concatenate([s.reshape(-1) for s in starts]), dtype=torch.float32, device="cuda")
    prms = []
    for R, L, T in entries:
        p, _ = material(L, 0.0, T, 0.02)
        p.dtau, p.renorm = 0.04, True
        prms.append(p)
    disk.heun_step(m, 3, prms, seed=20120827, step0=777, replica=10)
    disk.check()
    for k, (R, L, T) in enumerate(entries):
        od = oracle.Disk(R, L)
        p = prms[k]
        op = oracle.Params(alpha=p.alpha, c=p.c, temp=p.temp, dtau=p.dtau, renorm=True)
        x0 = od.apply_mask(torch.tensor(starts[k], dtype=torch.float32).double())
        ref = o_heun(x0, od, op, seed=20120827, step0=777, replica=10 + k, nsteps=3)
        got = disk.unpack(m, k).double().cpu()
        print(R, L, T, float((got - ref).abs().max()))
        assert float((got - ref).abs().max()) <= 5e-6


def test_boltzmann_statistics_short_horizon():
    from experiments.thermal import run
    rep = run([(30.0, 5.0)], [300.0], replicas=64, alpha=0.5, dtau=0.04, tau=10000.0, every=250,
              series_every=50, equil=0.4, seg=256, fd_factor=True)
    g = rep["geometries"][0]
    print({k: g["radial"][k] for k in ("r2_measured", "r2_predicted", "ratio", "ks_distance")}, g["static"]["kt"])
    assert g["vortex_lost_samples"] == 0
    assert 0.7 < g["static"]["kt"] / (5.0 / (8 * 30.0)) < 1.3        # loose law kt ~ L/(8R)
    assert 0.75 < g["radial"]["ratio"] < 1.25
    assert g["radial"]["ks_distance"] < 0.15
