"""Parity at the benchmarked sizes and launch shapes: the 64-replica Heun batch
(R = 250 nm, P = 512) and the 256-disk ragged RK4 batch in the plans the tuner
picks for them, with sampled disks checked against the float64 oracle, for a
few steps and for the benchmark's 20-step launch; and the largest supported
box (D = 256, P = 512).

Trajectory tolerance: 2.5e-6 absolute on |m| = 1 per step taken (the few-step
bound of the parity tests), so 5e-5 after the 20 steps of a timed launch."""
import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.demag import demag_fft
from oracle.dynamics import heun_step as o_heun, llg_rhs as o_rhs, rk4_step as o_rk4

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


@pytest.mark.parametrize("pol,nsteps", [(1, 2), (3, 2), (3, 20)])
def test_heun_replicas_full_size(pol, nsteps):
    from paper_1207_2192_amd import Disk, params_from_si
    n, R, L = 64, 250.0, 20.0
    disk = Disk.batch([R] * n, [L] * n)
    disk.tune(4, [4] * n, pol)                  # the benchmark's plans: 256 workgroups x 768 threads
    assert disk.launch_shape()[:2] == (4, 256)
    D = disk.D[0]
    PY = li.PERMALLOY
    p, _ = params_from_si(PY["A"], PY["Ms"], PY["gamma"], 2.0, L, 0.02, 300.0, 0.1)
    p.renorm = True
    m0 = li.vortex_ansatz(D, 0.01, 0.013)
    m = torch.tensor(np.concatenate([m0.reshape(-1)] * n), dtype=torch.float32, device="cuda")
    seed, step0 = 20120827, 4000
    disk.heun_step(m, nsteps, [p] * n, seed=seed, step0=step0, replica=0)
    disk.check()
    od = oracle.Disk(R, L)
    op = oracle.Params(alpha=p.alpha, c=p.c, dtau=p.dtau, temp=p.temp, renorm=True)
    m32 = od.apply_mask(torch.tensor(m0, dtype=torch.float32).double())
    for k in (0, 17, 63):                          # each replica draws its own noise stream
        ref = o_heun(m32, od, op, seed=seed, step0=step0, replica=k, nsteps=nsteps)
        got = disk.unpack(m, k).view(3, D, D).double().cpu()
        print(f"replica {k}, {nsteps} steps: max err {float((got - ref).abs().max()):.2e}", flush=True)
        assert float((got - ref).abs().max()) <= 2.5e-6 * nsteps
    # replicas differ (independent noise), and |m| = 1 inside the disk
    assert not torch.equal(disk.unpack(m, 0), disk.unpack(m, 1))
    nrm = torch.linalg.vector_norm(disk.unpack(m, 5).view(3, D, D).double().cpu(), dim=0)[od.mask]
    assert float((nrm - 1).abs().max()) < 1e-6


@pytest.mark.parametrize("pol,nsteps", [(1, 3), (3, 3), (3, 20)])
def test_ragged_batch_full_size(pol, nsteps):
    from paper_1207_2192_amd import Disk, LLGParams
    ens = li.ragged_ensemble(256)
    disk = Disk.batch([e.R_nm for e in ens], [e.L_nm for e in ens])
    disk.tune(1, None, pol)                        # one-group workgroups, the library's counts
    m0s = [li.vortex_ansatz(disk.D[k], ens[k].x0_nm / 2.0 + 0.01, ens[k].y0_nm / 2.0) for k in range(disk.n)]
    m = torch.tensor(np.concatenate([x.reshape(-1) for x in m0s]), dtype=torch.float32, device="cuda")
    p = LLGParams(alpha=0.02, c=C_PY, dtau=0.04)
    disk.rk4_step(m, nsteps, [p] * disk.n)
    disk.check()
    Ds = np.array(disk.D)
    pick = [int(np.argmin(Ds)), int(np.argmax(Ds)), 7, 128, 200]
    for k in pick:
        od = oracle.Disk(ens[k].R_nm, ens[k].L_nm)
        m32 = od.apply_mask(torch.tensor(m0s[k], dtype=torch.float32).double())
        ref = o_rk4(m32, od, oracle.Params(alpha=0.02, c=C_PY, dtau=0.04), nsteps)
        got = disk.unpack(m, k).view(3, disk.D[k], disk.D[k]).double().cpu()
        print(f"disk {k} (D={disk.D[k]}, P={disk.P[k]}), {nsteps} steps: max err "
              f"{float((got - ref).abs().max()):.2e}", flush=True)
        assert float((got - ref).abs().max()) <= 2.5e-6 * nsteps


def test_largest_box_fields():
    from paper_1207_2192_amd import Disk, LLGParams
    R, L = 256.0, 20.0
    disk = Disk.build(R, L)
    D = disk.D[0]
    assert (D, disk.P[0]) == (256, 512)
    od = oracle.Disk(R, L)
    m0 = li.smooth_random_field(D, 8)
    m = torch.tensor(m0, dtype=torch.float32, device="cuda").reshape(-1).contiguous()
    m32 = od.apply_mask(m.view(3, D, D).double().cpu())
    H = disk.demag_field(m).view(3, D, D).double().cpu()
    ref = demag_fft(m32, od)
    assert float((H - ref).abs().max() / ref.abs().max()) <= 1e-5
    p = LLGParams(alpha=0.05, c=C_PY, hext=(0.01, 0.0, -0.02))
    f = disk.rhs(m, p).view(3, D, D).double().cpu()
    fr = o_rhs(m32, od, oracle.Params(alpha=0.05, c=C_PY, hext=(0.01, 0.0, -0.02)))
    assert float((f - fr).abs().max() / fr.abs().max()) <= 1e-5
