"""Failure detection forced from the host, with every kernel ending normally:
a non-finite state raises the device flag that llg_check reports, and a
group-barrier wait given a tiny poll budget (llg_debug_spin_limit) records a
timeout and leaves the kernel; in both cases the handle keeps working and the
next launch with clean inputs and the default budget gives the reference
result bit for bit."""
import numpy as np
import pytest
import torch

import llg_inputs as li

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").reshape(-1).contiguous()


@pytest.mark.parametrize("integrator", ["rk4", "heun"])
def test_non_finite_state_is_reported(integrator):
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd._lib import LLGError
    disk = Disk.build(30.0, 10.0)
    D = disk.D[0]
    m0 = dev(li.vortex_ansatz(D, 1.0, 2.0))
    p = LLGParams(alpha=0.05, c=C_PY, dtau=0.04, temp=0.01 if integrator == "heun" else 0.0, renorm=True)

    def step(m):
        if integrator == "rk4":
            disk.rk4_step(m, 3, p)
        else:
            disk.heun_step(m, 3, p, seed=5, step0=0)

    ref = m0.clone()
    step(ref)
    disk.check()
    bad = m0.clone()
    bad.view(3, D, D)[0, D // 2, D // 2] = float("nan")     # a cell inside the disk
    step(bad)
    with pytest.raises(LLGError, match="non-finite"):
        disk.check()
    again = m0.clone()
    step(again)
    disk.check()                                             # the flag was cleared by the report
    assert torch.equal(again, ref)


def test_barrier_timeout_is_reported_and_the_handle_recovers():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd._lib import LLGError
    disk = Disk.batch([100.0, 60.0], [20.0, 10.0])
    # more workgroups than row tiles: the idle ones wait at every barrier
    disk.tune(2, [40, 20], 0)
    m0 = disk.pack([dev(li.vortex_ansatz(D, 2.0, -1.0)) for D in disk.D])
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04)] * disk.n
    ref = m0.clone()
    disk.rk4_step(ref, 4, p)
    disk.check()
    disk.debug_spin_limit(1)
    scratch = m0.clone()
    disk.rk4_step(scratch, 4, p)
    with pytest.raises(LLGError, match="barrier"):
        disk.check()
    disk.debug_spin_limit(0)
    m = m0.clone()
    disk.rk4_step(m, 4, p)
    disk.check()
    assert torch.equal(m, ref)
