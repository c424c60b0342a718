"""Ragged batches as executable hipGraphs and the device-side Heun step counter:
every replay is checked against the same steps taken by eager calls, with
unrelated eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

import llg_inputs as li

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


def ragged():
    from paper_1207_2192_amd import Disk
    Rs, Ls = [30.0, 44.0, 60.0], [10.0, 6.0, 15.0]
    disk = Disk.batch(Rs, Ls)
    m = torch.tensor(np.concatenate([li.vortex_ansatz(D, 2.0 + k, -1.0).reshape(-1) for k, D in enumerate(disk.D)]),
                     dtype=torch.float32, device="cuda")
    return disk, m


def other_work():
    x = torch.randn(1 << 20, device="cuda")
    y = (x * x).sum()
    torch.cuda.synchronize()
    return float(y)


def test_rk4_graph_replays_match_eager_calls():
    from paper_1207_2192_amd import LLGParams
    disk, m0 = ragged()
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04)] * disk.n
    mg, me = m0.clone(), m0.clone()
    g = disk.graph("rk4", mg, 15, p)
    for rep in range(3):
        g.launch()
        other_work()
        disk.rk4_step(me, 15, p)
        torch.cuda.synchronize()
        disk.check()
        assert torch.equal(mg, me), rep
    assert not torch.equal(mg, m0)
    g.close()


def test_heun_graph_continues_the_noise_stream():
    from paper_1207_2192_amd import LLGParams
    disk, m0 = ragged()
    p = [LLGParams(alpha=0.1, c=C_PY, dtau=0.0266, temp=0.008, renorm=True)] * disk.n
    mg, me = m0.clone(), m0.clone()
    disk.set_step(1000)
    g = disk.graph("heun", mg, 10, p, seed=77, replica=5)
    for rep in range(3):
        g.launch()
        other_work()
        # the eager path with explicit step indices; the counter is untouched by it
        disk.heun_step(me, 10, p, seed=77, step0=1000 + 10 * rep, replica=5)
        torch.cuda.synchronize()
        disk.check()
        assert torch.equal(mg, me), rep
    assert disk.get_step() == 1030
    g.close()


def test_eager_heun_with_the_step_counter_equals_explicit_steps():
    from paper_1207_2192_amd import LLGParams
    disk, m0 = ragged()
    p = [LLGParams(alpha=0.1, c=C_PY, dtau=0.0266, temp=0.008, renorm=True)] * disk.n
    m1, m2 = m0.clone(), m0.clone()
    disk.set_step(5)
    disk.heun_step(m1, 7, p, seed=3, step0=None)
    disk.heun_step(m1, 3, p, seed=3, step0=None)
    disk.heun_step(m2, 10, p, seed=3, step0=5)
    torch.cuda.synchronize()
    disk.check()
    assert disk.get_step() == 15
    assert torch.equal(m1, m2)


def test_graph_keeps_its_launch_plan_across_a_retune():
    # a graph copies the plan (workgroup maps, descriptors, partial sums) at creation:
    # re-planning the handle afterwards must neither disturb nor invalidate it
    from paper_1207_2192_amd import LLGParams
    disk, m0 = ragged()
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04)] * disk.n
    mg, me = m0.clone(), m0.clone()
    g = disk.graph("rk4", mg, 12, p)
    shape0 = disk.launch_shape()
    for rep, (ug, wg, pol) in enumerate([(2, [1, 2, 3], 1), (4, None, 3), (1, [5, 1, 2], 2)]):
        disk.tune(ug, wg, pol)
        assert disk.launch_shape() != shape0 or rep > 0
        g.launch()
        other_work()
        disk.rk4_step(me, 12, p)        # eager steps under the new plan
        torch.cuda.synchronize()
        disk.check()
        # the radix schedule of the plans differs, so equal to float rounding only
        assert float((mg - me).abs().max()) <= 1e-5, rep
        me.copy_(mg)
    g.close()
