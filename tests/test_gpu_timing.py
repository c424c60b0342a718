"""Opt-in launch timing of the C ABI (llg_timing / llg_last_launch_ms): off by
default, kept per kind of launch, and each figure lies inside the stream-event
interval that brackets the same call (the library's events sit right around
the cooperative kernel, after the barrier reset)."""
import numpy as np
import pytest
import torch

import llg_inputs as li

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


def test_launch_timing_per_kind():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd._lib import LLGError
    disk = Disk.batch([61.0, 100.0], [12.0, 20.0])
    m = disk.pack([torch.tensor(li.vortex_ansatz(D, 2.0, 1.0), dtype=torch.float32, device="cuda").reshape(-1)
                   for D in disk.D])
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04, temp=0.01, renorm=True)] * disk.n
    disk.rk4_step(m, 5, p)
    with pytest.raises(LLGError):
        disk.last_launch_ms("rk4")              # timing is off by default
    disk.timing(True)
    with pytest.raises(LLGError):
        disk.last_launch_ms("rk4")              # nothing timed since enabling
    stream = torch.cuda.current_stream()
    for kind, call in (("rk4", lambda: disk.rk4_step(m, 200, p)),
                       ("heun", lambda: disk.heun_step(m, 100, p, seed=3, step0=0)),
                       ("energy", lambda: disk.energy(m, p))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        outer = e0.elapsed_time(e1)
        ms = disk.last_launch_ms(kind)
        print(kind, ms, outer, flush=True)
        assert 0.0 < ms <= outer
        if kind != "energy":                    # a long launch is most of its call
            assert ms >= 0.8 * outer
    # the integrators' figures are kept while other kinds run
    t_rk4 = disk.last_launch_ms("rk4")
    disk.energy(m, p)
    assert disk.last_launch_ms("rk4") == t_rk4
    disk.timing(False)
    with pytest.raises(LLGError):
        disk.last_launch_ms("heun")
    disk.check()
