"""Small-disk trajectory: the float32 GPU RK4 run against the float64 oracle
over 2000 steps (Permalloy R = 30 nm, L = 10 nm, a = 2 nm, alpha = 0.01,
dt = 0.05 ps; vortex with a 5 nm Gaussian core at X = (5 nm, 0)).  Reports and
bounds the trajectory error, the core-position error, the energy change and
the |m| drift (renormalisation off)."""
import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.dynamics import rk4_step as o_rk4
from oracle.observables import energy as o_energy, vortex_core_position as o_core

pytestmark = pytest.mark.gpu


def test_small_disk_trajectory_against_float64():
    from paper_1207_2192_amd import Disk, params_from_si
    R, L, a = 30.0, 10.0, 2.0
    PY = li.PERMALLOY
    p, lam = params_from_si(PY["A"], PY["Ms"], PY["gamma"], a, L, 0.05, 0.0, 0.01)
    disk = Disk.build(R, L, a)
    D = disk.D[0]
    od = oracle.Disk(R, L, a)
    m0 = li.vortex_ansatz(D, 5.0 / a, 0.0, core_width=2.5)
    m = torch.tensor(m0, dtype=torch.float32, device="cuda").reshape(-1).contiguous()
    op = oracle.Params(alpha=p.alpha, c=p.c, dtau=p.dtau)
    mo = od.apply_mask(torch.tensor(m0))
    e0 = o_energy(mo, od, op)[0]
    err_m, err_rc, core_gpu, core_ref = 0.0, 0.0, [], []
    for chunk in range(20):
        disk.rk4_step(m, 100, p)
        mo = o_rk4(mo, od, op, 100)
        g = m.view(3, D, D).double().cpu()
        err_m = max(err_m, float((g - mo).abs().max()))
        cg = [float(v) for v in disk.vortex_core_position(m, lam).cpu()[0]]
        cr = o_core(mo, od, lam)
        core_gpu.append((cg[0], cg[1]))
        core_ref.append(cr[:2])
        err_rc = max(err_rc, float(np.hypot(cg[0] - cr[0], cg[1] - cr[1])))
    disk.check()
    eg = disk.energy(m, p).cpu()[0, 0].item()
    er = o_energy(mo, od, op)[0]
    norm = torch.linalg.vector_norm(m.view(3, D, D).double().cpu(), dim=0)[od.mask]
    drift = float((norm - 1).abs().max())
    print(f"\n2000 RK4 steps: max |m_gpu - m_f64| = {err_m:.2e}, max core-position error = {err_rc:.2e} nm, "
          f"energy {e0:.6f} -> {er:.6f} (gpu {eg:.6f}), |m| drift {drift:.2e}; "
          f"core moved from {core_ref[0]} to {core_ref[-1]} nm")
    # the damped gyration moved the core by more than the error bounds below
    assert np.hypot(core_ref[-1][0] - core_ref[0][0], core_ref[-1][1] - core_ref[0][1]) > 0.5
    assert err_m <= 2e-4
    assert err_rc <= 5e-3
    assert abs(eg - er) <= 1e-5 * abs(er)
    assert er < e0                      # damping
    assert drift <= 1e-4                # RK4 error without renormalisation
