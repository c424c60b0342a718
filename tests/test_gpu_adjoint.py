"""GPU adjoint: llg_rk4_record / llg_rk4_vjp / llg_core_position_vjp and the
CoreTrajectory autograd Function against the float64 oracle's autograd
gradient and against finite differences."""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.dynamics import heun_step as o_heun, rk4_step as o_rk4
from oracle.observables import core_centroid, vortex_core_position as o_core

pytestmark = pytest.mark.gpu
C_PY = 0.14298555
LAM = 5.28906


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").reshape(-1).contiguous()


# up to P = 128, the P = 256 instance of the R = 80 nm adjoint workload, and P = 512
@pytest.mark.parametrize("R,L,nsteps,pol", [(15.0, 5.0, 3, 0), (30.0, 10.0, 5, 0), (61.0, 12.0, 2, 0),
                                            (30.0, 10.0, 5, 3), (80.0, 10.0, 3, 0), (80.0, 10.0, 2, 1),
                                            (250.0, 20.0, 1, 0)])
def test_rk4_vjp_matches_oracle(R, L, nsteps, pol):
    # pol 3: the recording integrator runs lane-group columns, the adjoint kernel its own strategy
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.build(R, L)
    disk.tune(1, None, pol)
    D = disk.D[0]
    od = oracle.Disk(R, L)
    m0 = li.smooth_random_field(D, 4)
    yb = li.random_unit_field(D, 9)
    p = LLGParams(alpha=0.07, c=C_PY, dtau=0.05, hext=(0.02, -0.01, 0.03))
    m = dev(m0)
    m32 = m.view(3, D, D).double().cpu()
    rec = torch.empty(8 * nsteps * disk.state_size, dtype=torch.float32, device="cuda")
    disk.rk4_record(m, nsteps, p, rec)
    ybar = dev(yb * od.mask.numpy())
    pgrad = torch.zeros(2, dtype=torch.float64, device="cuda")
    disk.rk4_vjp(rec, nsteps, ybar, pgrad, p)
    disk.check()
    # oracle: autograd of <yb, y_N(m0, alpha, c)>
    mr = m32.clone().requires_grad_(True)
    a = torch.tensor(0.07, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    yN = o_rk4(mr, od, oracle.Params(alpha=a, c=c, dtau=0.05, hext=(0.02, -0.01, 0.03)), nsteps)
    L_ = (yN * torch.tensor(yb) * od.mask).sum()
    gm, ga, gc = torch.autograd.grad(L_, (mr, a, c))
    gm = od.apply_mask(gm)
    got = ybar.view(3, D, D).double().cpu()
    assert float((got - gm).abs().max()) <= 1e-5 * float(gm.abs().max())
    assert abs(float(pgrad[0]) - float(ga)) <= 1e-5 * abs(float(ga)) + 1e-6
    assert abs(float(pgrad[1]) - float(gc)) <= 1e-5 * abs(float(gc)) + 1e-6


@pytest.mark.parametrize("R,L,nsteps,renorm,fd", [(15.0, 5.0, 4, False, False), (30.0, 10.0, 6, True, False),
                                                  (41.0, 8.0, 3, True, True), (80.0, 10.0, 2, True, False),
                                                  (250.0, 20.0, 1, True, False)])
def test_heun_vjp_matches_oracle(R, L, nsteps, renorm, fd):
    # reverse pass of Heun steps with the noise replayed, against autograd through the oracle
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.build(R, L)
    D = disk.D[0]
    od = oracle.Disk(R, L)
    m0 = li.smooth_random_field(D, 6)
    yb = li.random_unit_field(D, 3)
    kw = dict(alpha=0.1, c=C_PY, dtau=0.03, temp=0.02, renorm=renorm, fd_factor=fd, hext=(0.01, 0.02, -0.01))
    p = LLGParams(**kw)
    seed, step0, rep = 99, 1234, 3
    m = dev(m0)
    m32 = m.view(3, D, D).double().cpu()
    rec = torch.empty(4 * nsteps * disk.state_size, dtype=torch.float32, device="cuda")
    disk.heun_record(m, nsteps, p, rec, seed=seed, step0=step0, replica=rep)
    ybar = dev(yb * od.mask.numpy())
    pgrad = torch.zeros(2, dtype=torch.float64, device="cuda")
    disk.heun_vjp(rec, nsteps, ybar, pgrad, p, seed=seed, step0=step0, replica=rep)
    disk.check()
    mr = m32.clone().requires_grad_(True)
    a = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    okw = dict(kw, alpha=a, c=c)
    yN = o_heun(mr, od, oracle.Params(**okw), seed=seed, step0=step0, replica=rep, nsteps=nsteps)
    # the recorded forward is the ordinary Heun step
    assert float((m.view(3, D, D).double().cpu() - yN.detach()).abs().max()) <= 5e-6
    L_ = (yN * torch.tensor(yb) * od.mask).sum()
    gm, ga, gc = torch.autograd.grad(L_, (mr, a, c))
    gm = od.apply_mask(gm)
    got = ybar.view(3, D, D).double().cpu()
    assert float((got - gm).abs().max()) <= 2e-5 * float(gm.abs().max())
    assert abs(float(pgrad[0]) - float(ga)) <= 2e-5 * abs(float(ga)) + 1e-6
    assert abs(float(pgrad[1]) - float(gc)) <= 2e-5 * abs(float(gc)) + 1e-6


def test_core_position_vjp_matches_oracle():
    from paper_1207_2192_amd import Disk
    disk = Disk.build(40.0, 10.0)
    D = disk.D[0]
    od = oracle.Disk(40.0, 10.0)
    m0 = li.vortex_ansatz(D, 3.3, -1.7)
    m = dev(m0)
    core = disk.vortex_core_position(m, LAM)
    rbar = torch.tensor([[0.7, -1.3]], dtype=torch.float64, device="cuda")
    mbar = torch.zeros_like(m)
    disk.core_position_vjp(m, LAM, core, rbar, mbar)
    c = core.cpu()[0]
    mr = m.view(3, D, D).double().cpu().requires_grad_(True)
    rc = core_centroid(mr, od, LAM, float(c[2]), float(c[3]), True)
    (g,) = torch.autograd.grad((rc * torch.tensor([0.7, -1.3], dtype=torch.float64)).sum(), mr)
    got = mbar.view(3, D, D).double().cpu()
    assert float((got - g).abs().max()) <= 1e-6 * float(g.abs().max())


def _oracle_loss(m0, alpha, c, od, n_seg, seg, target, frozen_sets):
    prm = oracle.Params(alpha=alpha, c=c, dtau=0.04)
    m = m0
    rcs = []
    for s in range(n_seg + 1):
        if s > 0:
            m = o_rk4(m, od, prm, seg)
        fr = frozen_sets[s]
        rcs.append(core_centroid(m, od, LAM, fr[2], fr[3], fr[4] > 0))
    rc = torch.stack(rcs)
    return ((rc - target) ** 2).sum()


def test_trajectory_gradient_matches_oracle_and_finite_differences():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory
    R, L = 30.0, 10.0
    disk = Disk.build(R, L)
    D = disk.D[0]
    od = oracle.Disk(R, L)
    n_seg, seg = 4, 25
    m0_np = li.vortex_ansatz(D, 2.6, 0.4)
    m0 = dev(m0_np)
    base = LLGParams(alpha=0.01, c=C_PY, dtau=0.04)
    target = torch.tensor([[2.0 * math.cos(0.1 * k), 2.0 * math.sin(0.1 * k)] for k in range(n_seg + 1)],
                          dtype=torch.float64)
    m0g = m0.clone().requires_grad_(True)
    a = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    rc = core_trajectory(m0g, a, c, disk, base, n_seg, seg, LAM)
    loss = ((rc - target.cuda()) ** 2).sum()
    loss.backward()
    disk.check()
    # oracle gradient with the same frozen core sets (taken from the GPU forward)
    frozen = []
    m32 = m0.view(3, D, D).double().cpu()
    mo = m32.clone()
    for s in range(n_seg + 1):
        if s > 0:
            mo = o_rk4(mo, od, oracle.Params(alpha=0.01, c=C_PY, dtau=0.04), seg)
        frozen.append(o_core(mo, od, LAM))
    mr = m32.clone().requires_grad_(True)
    ao = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    co = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    Lo = _oracle_loss(mr, ao, co, od, n_seg, seg, target, frozen)
    gm, ga, gc = torch.autograd.grad(Lo, (mr, ao, co))
    assert abs(float(loss) - float(Lo)) <= 1e-4 * abs(float(Lo))
    got_m = m0g.grad.view(3, D, D).double().cpu()
    gm = od.apply_mask(gm)
    assert float((got_m - gm).abs().max()) <= 2e-3 * float(gm.abs().max())
    assert abs(float(a.grad) - float(ga)) <= 2e-3 * abs(float(ga))
    assert abs(float(c.grad) - float(gc)) <= 2e-3 * abs(float(gc))
    # central finite differences of the float64 oracle, h = 1e-4
    h = 1e-4
    fa = (_oracle_loss(m32, 0.01 + h, C_PY, od, n_seg, seg, target, frozen)
          - _oracle_loss(m32, 0.01 - h, C_PY, od, n_seg, seg, target, frozen)) / (2 * h)
    fc = (_oracle_loss(m32, 0.01, C_PY + h, od, n_seg, seg, target, frozen)
          - _oracle_loss(m32, 0.01, C_PY - h, od, n_seg, seg, target, frozen)) / (2 * h)
    assert abs(float(a.grad) - float(fa)) <= 5e-3 * abs(float(fa))
    assert abs(float(c.grad) - float(fc)) <= 5e-3 * abs(float(fc))


def test_heun_trajectory_gradient_matches_oracle():
    # checkpointed Heun trajectory at T > 0 with renormalisation, noise replayed in the backward pass
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory
    R, L = 30.0, 10.0
    disk = Disk.build(R, L)
    D = disk.D[0]
    od = oracle.Disk(R, L)
    n_seg, seg = 3, 10
    seed, step0, rep = 5, 700, 1
    m0 = dev(li.vortex_ansatz(D, 2.6, 0.4))
    kw = dict(alpha=0.05, c=C_PY, dtau=0.03, temp=0.01, renorm=True)
    base = LLGParams(**kw)
    target = torch.tensor([[2.0 * math.cos(0.1 * k), 2.0 * math.sin(0.1 * k)] for k in range(n_seg + 1)],
                          dtype=torch.float64)
    m0g = m0.clone().requires_grad_(True)
    a = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    rc = core_trajectory(m0g, a, c, disk, base, n_seg, seg, LAM, noise=(seed, step0, rep))
    loss = ((rc - target.cuda()) ** 2).sum()
    loss.backward()
    disk.check()

    def o_step(x, s, alpha=0.05, cc=C_PY):
        return o_heun(x, od, oracle.Params(**dict(kw, alpha=alpha, c=cc)), seed=seed, step0=step0 + s * seg,
                      replica=rep, nsteps=seg)

    m32 = m0.view(3, D, D).double().cpu()
    frozen, mo = [], m32.clone()
    for s in range(n_seg + 1):
        if s > 0:
            mo = o_step(mo, s - 1)
        frozen.append(o_core(mo, od, LAM))
    mr = m32.clone().requires_grad_(True)
    ao = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    co = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
    x, Lo = mr, 0.0
    for s in range(n_seg + 1):
        if s > 0:
            x = o_step(x, s - 1, ao, co)
        f = frozen[s]
        rcs = core_centroid(x, od, LAM, f[2], f[3], f[4] >= 1)
        Lo = Lo + ((rcs - target[s]) ** 2).sum()
    gm, ga, gc = torch.autograd.grad(Lo, (mr, ao, co))
    assert abs(float(loss) - float(Lo)) <= 1e-4 * abs(float(Lo))
    got_m = m0g.grad.view(3, D, D).double().cpu()
    gm = od.apply_mask(gm)
    assert float((got_m - gm).abs().max()) <= 2e-3 * float(gm.abs().max())
    assert abs(float(a.grad) - float(ga)) <= 2e-3 * abs(float(ga))
    assert abs(float(c.grad) - float(gc)) <= 2e-3 * abs(float(gc))
