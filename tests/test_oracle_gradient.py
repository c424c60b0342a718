"""Oracle pin for the gradient oracle: torch autograd through the float64
oracle (RK4 trajectory + frozen-set core centroid) against central finite
differences of the same oracle."""
import numpy as np
import torch

import llg_inputs as li
from oracle import Disk, Params
from oracle.dynamics import heun_step, rk4_step
from oracle.observables import core_centroid, vortex_core_position

LAM = 5.28906


def loss_fn(m0, alpha, c, disk, nsteps, frozen):
    prm = Params(alpha=alpha, c=c, dtau=0.06)
    m = rk4_step(m0, disk, prm, nsteps)
    rc = core_centroid(m, disk, LAM, frozen[2], frozen[3], True)
    tgt = torch.tensor([3.0, -1.0], dtype=torch.float64)
    return ((rc - tgt) ** 2).sum()


def test_autograd_matches_finite_differences():
    d = Disk(10.0, 5.0, 2.0)
    m0 = torch.tensor(li.vortex_ansatz(d.D, 1.3, -0.4), dtype=torch.float64)
    n = 12
    mN = rk4_step(m0, d, Params(alpha=0.05, c=0.143, dtau=0.06), n)
    frozen = vortex_core_position(mN, d, LAM)
    assert frozen[4] >= 1
    m0r = m0.clone().requires_grad_(True)
    a = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(0.143, dtype=torch.float64, requires_grad=True)
    L = loss_fn(m0r, a, c, d, n, frozen)
    gm, ga, gc = torch.autograd.grad(L, (m0r, a, c))
    h = 1e-6
    fa = (loss_fn(m0, 0.05 + h, 0.143, d, n, frozen) - loss_fn(m0, 0.05 - h, 0.143, d, n, frozen)) / (2 * h)
    fc = (loss_fn(m0, 0.05, 0.143 + h, d, n, frozen) - loss_fn(m0, 0.05, 0.143 - h, d, n, frozen)) / (2 * h)
    assert abs(float(ga) - float(fa)) <= 1e-6 * max(1.0, abs(float(fa)))
    assert abs(float(gc) - float(fc)) <= 1e-6 * max(1.0, abs(float(fc)))
    rng = np.random.default_rng(0)
    idx = np.argwhere(d.mask.numpy())
    for k in rng.choice(len(idx), 5, replace=False):
        j, i = idx[k]
        for comp in range(3):
            mp, mn = m0.clone(), m0.clone()
            mp[comp, j, i] += h
            mn[comp, j, i] -= h
            fd = (loss_fn(mp, 0.05, 0.143, d, n, frozen) - loss_fn(mn, 0.05, 0.143, d, n, frozen)) / (2 * h)
            assert abs(float(gm[comp, j, i]) - float(fd)) <= 1e-6 * max(1.0, abs(float(fd)))


def heun_loss(m0, alpha, c, disk, nsteps, v, renorm, fd):
    prm = Params(alpha=alpha, c=c, dtau=0.03, temp=0.02, renorm=renorm, fd_factor=fd)
    m = heun_step(m0, disk, prm, seed=11, step0=40, replica=2, nsteps=nsteps)
    return (m * v).sum()


def test_heun_autograd_matches_finite_differences():
    # the gradient w.r.t. alpha includes the noise amplitude sigma(alpha)
    d = Disk(8.0, 4.0, 2.0)
    m0 = torch.tensor(li.smooth_random_field(d.D, 2), dtype=torch.float64)
    v = torch.tensor(li.random_unit_field(d.D, 5), dtype=torch.float64) * d.mask
    for renorm, fd in ((False, False), (True, True)):
        m0r = m0.clone().requires_grad_(True)
        a = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
        c = torch.tensor(0.143, dtype=torch.float64, requires_grad=True)
        L = heun_loss(m0r, a, c, d, 5, v, renorm, fd)
        gm, ga, gc = torch.autograd.grad(L, (m0r, a, c))
        h = 1e-6
        fa = (heun_loss(m0, 0.2 + h, 0.143, d, 5, v, renorm, fd) - heun_loss(m0, 0.2 - h, 0.143, d, 5, v, renorm, fd)) / (2 * h)
        fc = (heun_loss(m0, 0.2, 0.143 + h, d, 5, v, renorm, fd) - heun_loss(m0, 0.2, 0.143 - h, d, 5, v, renorm, fd)) / (2 * h)
        assert abs(float(ga) - float(fa)) <= 1e-6 * max(1.0, abs(float(fa)))
        assert abs(float(gc) - float(fc)) <= 1e-6 * max(1.0, abs(float(fc)))
        # the noise path matters: without it the alpha gradient changes
        prm0 = Params(alpha=0.2, c=0.143, dtau=0.03, temp=0.02, renorm=renorm, fd_factor=fd)
        assert prm0.sigma() > 0
        idx = np.argwhere(d.mask.numpy())
        for k in np.random.default_rng(1).choice(len(idx), 3, replace=False):
            j, i = idx[k]
            for comp in range(3):
                mp, mn = m0.clone(), m0.clone()
                mp[comp, j, i] += h
                mn[comp, j, i] -= h
                fd_ = (heun_loss(mp, 0.2, 0.143, d, 5, v, renorm, fd) - heun_loss(mn, 0.2, 0.143, d, 5, v, renorm, fd)) / (2 * h)
                assert abs(float(gm[comp, j, i]) - float(fd_)) <= 1e-6 * max(1.0, abs(float(fd_)))
