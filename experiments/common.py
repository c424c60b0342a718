"""GPU pipelines shared by the studies: batched constrained relaxations, core
trajectories sampled between launches, and on-device spectra of the <m>
series.  Everything runs through lib_llgdisk's Python binding."""
from __future__ import annotations

import math

import numpy as np
import torch

import llg_inputs as li
from paper_1207_2192_amd import Disk, LLGParams, params_from_si, power_spectrum

A_NM = 2.0
PY = li.PERMALLOY


def material(L_nm, dt_ps=0.0, T_K=0.0, alpha=0.0):
    """(LLGParams, lambda_ex_nm) for Permalloy at thickness L."""
    return params_from_si(PY["A"], PY["Ms"], PY["gamma"], A_NM, L_nm, dt_ps, T_K, alpha)


def pack_starts(batch: Disk, X_nm):
    """Vortex ansatz states (core width 2.5 a) at the (x, y) targets, nudged off the grid symmetry point."""
    return batch.pack([torch.tensor(li.vortex_ansatz(batch.D[k], X[0] / A_NM + 1e-3, X[1] / A_NM + 1e-3),
                                    dtype=torch.float32, device="cuda").reshape(-1) for k, X in enumerate(X_nm)])


def relax_batch(R_nm, L_nm, X_nm, lam_nm, *, tol=2e-6, max_sweeps=400000):
    """Relax one disk per entry with its core held at X (nm): returns (handle, states,
    relax record [n, 8], U [n] in J, core [n, 5]).  The constraint acts over the cells
    within 4 lambda_ex of X (the core-position definition of Sec. IV)."""
    batch = Disk.batch(R_nm, L_nm, A_NM)
    m = pack_starts(batch, X_nm)
    prm = []
    for L in L_nm:
        p, _ = material(L)
        prm.append(LLGParams(c=p.c))
    out = batch.relax(m, X_nm, prm, tol=tol, max_sweeps=max_sweeps, cutoff_nm=4.0 * lam_nm).cpu().numpy()
    batch.check()
    U = batch.energy(m, prm).cpu().numpy()[:, 0]
    core = batch.vortex_core_position(m, lam_nm).cpu().numpy()
    return batch, m, out, U, core


def sample_cores(disk: Disk, m, nsteps, every, step_fn, lam_nm, hint=True):
    """Run nsteps in launches of `every` steps (step_fn(n0, k) advances m by k steps
    from step n0) and sample the core position after each launch; returns
    (t_steps [S], cores [S, n, 5]) as numpy.  With hint, every sample uses the
    previous core position to choose among several +1 plaquettes."""
    import time
    S = nsteps // every
    cores = torch.empty(S, disk.n, 5, dtype=torch.float64, device="cuda")
    prev = None
    last = time.perf_counter()
    for s in range(S):
        step_fn(s * every, every)
        c = disk.vortex_core_position(m, lam_nm, hint_nm=prev)
        cores[s] = c
        if hint and s % 50 == 49:        # refresh the hint now and then (a host copy)
            prev = [tuple(v) for v in c[:, :2].cpu().numpy().tolist()]
            if time.perf_counter() - last > 30.0:
                last = time.perf_counter()
                print(f"# {(s + 1) * every} / {S * every} steps", flush=True)
    torch.cuda.synchronize()
    disk.check()
    return (np.arange(1, S + 1) * every), cores.cpu().numpy()


def segment_spectra(x: torch.Tensor, seg: int):
    """Bartlett spectrum on the device: x [samples, k] float64 (CUDA); the
    non-overlapping length-seg segments of every column go through
    llg_power_spectrum (mean removed, no window) and are averaged:
    returns (P [k, seg/2 + 1], segments per column)."""
    S, k = x.shape
    n = S // seg
    segs = x[:n * seg].t().contiguous().reshape(k * n, seg)
    P = power_spectrum(segs, True, "none").reshape(k, n, seg // 2 + 1).mean(dim=1)
    return P.cpu().numpy(), n
