"""Oracle pins: effective induction, LLG right-hand side, RK4 and Heun
(Sec. III) against brute force, closed forms and invariants."""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
from oracle import Disk, Params
from oracle.dynamics import (effective_field, exchange_field, heun_step, heun_step_replicas,
                             llg_rhs, rk4_step, torque)
from oracle.greens import self_factors
from oracle.observables import energy

C_PY = 0.14298555   # a^2/lambda_ex^2 for Permalloy at a = 2 nm


def unit(D, seed):
    return torch.from_numpy(li.random_unit_field(D, seed))


def smooth(D, seed):
    return torch.from_numpy(li.smooth_random_field(D, seed))


def test_exchange_matches_neighbour_loop():
    d = Disk(9, 4, 2.0)
    m = unit(d.D, 5)
    b = exchange_field(m, d)
    M = d.mask.numpy()
    ref = np.zeros((3, d.D, d.D))
    for j in range(d.D):
        for i in range(d.D):
            if not M[j, i]:
                continue
            for dj, di in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                jj, ii = j + dj, i + di
                if 0 <= jj < d.D and 0 <= ii < d.D and M[jj, ii]:
                    ref[:, j, i] += m[:, jj, ii].numpy()
    assert np.abs(b.numpy() - ref).max() < 1e-15


def test_uniform_state_exchange_counts_neighbours():
    d = Disk(11, 4, 2.0)
    m = torch.zeros(3, d.D, d.D, dtype=torch.float64)
    m[1] = 1.0
    b = exchange_field(m, d)
    M = d.mask.to(torch.float64)
    cnt = torch.zeros_like(M)
    cnt[1:] += M[:-1]; cnt[:-1] += M[1:]; cnt[:, 1:] += M[:, :-1]; cnt[:, :-1] += M[:, 1:]
    assert torch.equal(b[1], cnt * M)


@pytest.mark.parametrize("hext", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.5)])
def test_induction_is_minus_energy_gradient(hext):
    # b_i = -dE/dm_i (eq. Bi from eq. Hmm): finite differences of the energy.
    d = Disk(8, 6, 2.0)
    prm = Params(c=C_PY, hext=hext)
    m = unit(d.D, 9)
    b = effective_field(m, d, prm)
    eps = 1e-6
    idx = torch.nonzero(d.mask)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(idx), 8, replace=False):
        j, i = (int(t) for t in idx[k])
        for c in range(3):
            mp, mn = m.clone(), m.clone()
            mp[c, j, i] += eps
            mn[c, j, i] -= eps
            g = (energy(mp, d, prm)[0] - energy(mn, d, prm)[0]) / (2 * eps)
            assert abs(g + float(b[c, j, i])) < 1e-7


def test_rhs_invariants():
    d = Disk(10, 5, 2.0)
    prm = Params(alpha=0.3, c=C_PY, hext=(0.1, 0.0, -0.2))
    m = unit(d.D, 2)
    b = effective_field(m, d, prm)
    f = llg_rhs(m, d, prm)
    M = d.mask
    assert float((m * f).sum(0)[M].abs().max()) < 1e-13          # |m| preserved
    mxb = torch.linalg.cross(m, b, dim=0)
    bf = (b * f).sum(0)[M]
    assert float((bf - prm.alpha * (mxb * mxb).sum(0)[M]).abs().max()) < 1e-12  # dE/dtau <= 0
    f0 = llg_rhs(m, d, Params(alpha=0.0, c=C_PY, hext=prm.hext))
    assert float((b * f0).sum(0)[M].abs().max()) < 1e-12
    assert float(f[:, ~M].abs().max()) == 0.0


def test_single_cell_precession_closed_form():
    # One cell (D = 1) in a field along z feels h - (N_z - N_x) m_z along z:
    # m_z is conserved and the in-plane angle turns at omega = c (h - (N_z - N_x) m_z),
    # clockwise for omega > 0 under dm/dtau = m x b.
    d = Disk(1.0, 6.0, 2.0)
    nx, nz = self_factors(d.ell)
    h = 0.8
    prm = Params(alpha=0.0, c=C_PY, hext=(0, 0, h), dtau=0.01)
    th0, ph0 = 1.0, 0.3
    m0 = torch.tensor([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)],
                      dtype=torch.float64).view(3, 1, 1)
    n = 2000
    m = rk4_step(m0, d, prm, n)
    om = prm.c * (h - (nz - nx) * math.cos(th0))
    ph = ph0 - om * n * prm.dtau
    ref = torch.tensor([math.sin(th0) * math.cos(ph), math.sin(th0) * math.sin(ph), math.cos(th0)],
                       dtype=torch.float64).view(3, 1, 1)
    assert float((m - ref).abs().max()) < 1e-10


def test_rk4_is_fourth_order():
    d = Disk(12, 10, 2.0)
    prm = Params(alpha=0.05, c=C_PY)
    m0 = smooth(d.D, 7)
    T = 1.6
    ref = rk4_step(m0, d, Params(alpha=0.05, c=C_PY, dtau=T / 256), 256)
    errs = []
    for n in (8, 16, 32):
        y = rk4_step(m0, d, Params(alpha=0.05, c=C_PY, dtau=T / n), n)
        errs.append(float((y - ref).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 13 < r2 < 19, errs


def test_energy_conserved_without_damping():
    # At alpha = 0 the dynamics conserves the energy; RK4 leaves only its
    # truncation error, which must be tiny at dtau = 0.04 (Sec. III.A) and
    # fall at least 14x when dtau is halved (fourth order or better).
    d = Disk(20, 10, 2.0)
    m0 = torch.from_numpy(li.vortex_ansatz(d.D, 2.3, 1.1))
    drift = []
    for dt in (0.04, 0.02):
        prm = Params(alpha=0.0, c=C_PY, dtau=dt)
        e0 = energy(m0, d, prm)[0]
        e1 = energy(rk4_step(m0, d, prm, int(round(60 / dt))), d, prm)[0]
        drift.append(abs(e1 - e0) / abs(e0))
    assert drift[0] < 2e-9
    assert drift[0] / drift[1] > 14


def test_energy_decays_with_damping():
    d = Disk(16, 8, 2.0)
    prm = Params(alpha=0.1, c=C_PY, dtau=0.04)
    m = smooth(d.D, 3)
    es = [energy(m, d, prm)[0]]
    for _ in range(20):
        m = rk4_step(m, d, prm, 10)
        es.append(energy(m, d, prm)[0])
    assert all(b < a for a, b in zip(es, es[1:]))


def test_norm_drift_small_without_renormalisation():
    d = Disk(16, 8, 2.0)
    prm = Params(alpha=0.01, c=C_PY, dtau=0.04)
    m = smooth(d.D, 8)
    y = rk4_step(m, d, prm, 200)
    n = torch.linalg.vector_norm(y, dim=0)[d.mask]
    assert float((n - 1).abs().max()) < 1e-6
    y = rk4_step(m, d, Params(alpha=0.01, c=C_PY, dtau=0.04, renorm=True), 200)
    n = torch.linalg.vector_norm(y, dim=0)[d.mask]
    assert float((n - 1).abs().max()) < 1e-14


def test_heun_zero_temperature_is_second_order():
    d = Disk(12, 10, 2.0)
    m0 = smooth(d.D, 5)
    T = 0.8
    ref = rk4_step(m0, d, Params(alpha=0.05, c=C_PY, dtau=T / 64), 64)
    errs = []
    for n in (8, 16, 32):
        y = heun_step(m0, d, Params(alpha=0.05, c=C_PY, dtau=T / n), seed=1, step0=0, nsteps=n)
        errs.append(float((y - ref).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.5 < r2 < 4.5, errs


def test_heun_restart_is_bitwise_identical():
    d = Disk(8, 5, 2.0)
    prm = Params(alpha=0.1, c=C_PY, temp=0.05, dtau=0.02, renorm=True)
    m0 = smooth(d.D, 1)
    a = heun_step(m0, d, prm, seed=77, step0=10, replica=3, nsteps=6)
    b = heun_step(m0, d, prm, seed=77, step0=10, replica=3, nsteps=2)
    b = heun_step(b, d, prm, seed=77, step0=12, replica=3, nsteps=4)
    assert torch.equal(a, b)
    c = heun_step(m0, d, prm, seed=77, step0=10, replica=4, nsteps=6)
    assert not torch.equal(a, c)


def _langevin_mz(h, c, nx, nz, temp):
    # <m_z> for p(m_z) ~ exp(-E/T), E/J = -c h m_z + (c/2)(N_z - N_x) m_z^2 on [-1, 1]
    from scipy.integrate import quad
    E = lambda z: -c * h * z + 0.5 * c * (nz - nx) * z * z
    Z = quad(lambda z: math.exp(-E(z) / temp), -1, 1)[0]
    return quad(lambda z: z * math.exp(-E(z) / temp), -1, 1)[0] / Z


@pytest.mark.parametrize("fd", [False, True])
def test_heun_macrospin_reaches_boltzmann(fd):
    # A single cell in a field along z relaxes to the Boltzmann distribution of
    # its energy.  With noise variance 2 alpha T dtau in the Landau-Lifshitz
    # form the equilibrium temperature is (1 + alpha^2) T; dividing the
    # variance by (1 + alpha^2) restores T.
    d = Disk(1.0, 6.0, 2.0)
    nx, nz = self_factors(d.ell)
    alpha, temp, h = 1.0, 0.25, 4.0
    prm = Params(alpha=alpha, c=C_PY, hext=(0, 0, h), temp=temp, dtau=0.02, renorm=True, fd_factor=fd)
    B = 1500
    m = torch.zeros(B, 3, 1, 1, dtype=torch.float64)
    m[:, 2] = 1.0
    m = heun_step_replicas(m, d, prm, seed=2024, step0=0, replicas=range(B), nsteps=300)
    acc = []
    for k in range(12):
        m = heun_step_replicas(m, d, prm, seed=2024, step0=300 + 50 * k, replicas=range(B), nsteps=50)
        acc.append(float(m[:, 2].mean()))
    got = float(np.mean(acc))
    teff = temp if fd else (1 + alpha ** 2) * temp
    want = _langevin_mz(h, C_PY, nx, nz, teff)
    other = _langevin_mz(h, C_PY, nx, nz, (1 + alpha ** 2) * temp if fd else temp)
    assert abs(got - want) < 0.02, (got, want, other)
    assert abs(got - want) < 0.5 * abs(want - other)
