"""Oracle pins for the time-dependent external field h_ext(tau) (eq. Hmm and
eq. Bi with a driven field; the reading in oracle/units.py and
oracle/dynamics.py): the field formula at hand-picked times, the closed-form
precession of one cell in a driven axial field, and the orders of RK4 and of
the zero-temperature Heun step with a driven field, which hold only when each
stage takes the field at its own time."""
import math

import pytest
import torch

import llg_inputs as li
from oracle import Disk, Params
from oracle.dynamics import heun_step, rk4_step
from oracle.greens import self_factors
from oracle.observables import energy

C_PY = 0.14298555


def test_field_formula():
    p = Params(hext=(0.1, 0.0, -0.2), hac=(0.0, 0.3, 0.0), freq=0.25, phase=0.5,
               hpulse=(0.0, 0.0, 0.4), tpulse=3.0, wpulse=2.0)
    for tau in (0.0, 1.0, 3.0, 7.5):
        s = math.sin(2 * math.pi * 0.25 * tau + 0.5)
        g = math.exp(-((tau - 3.0) ** 2) / 8.0)
        h = p.field_at(tau)
        assert abs(h[0] - 0.1) < 1e-15
        assert abs(h[1] - 0.3 * s) < 1e-15
        assert abs(h[2] - (-0.2 + 0.4 * g)) < 1e-15
    assert Params(hext=(1.0, 2.0, 3.0)).field_at(123.0) == (1.0, 2.0, 3.0)


def test_single_cell_in_a_driven_axial_field():
    # one cell: m_z is conserved and the in-plane angle turns at
    # omega(tau) = c (h_z(tau) - (N_z - N_x) m_z); its integral is closed-form
    d = Disk(1.0, 6.0, 2.0)
    nx, nz = self_factors(d.ell)
    h0, h1, f, ph, hp, tp, w = 0.5, 0.3, 0.004, 0.7, 0.6, 25.0, 6.0
    prm = Params(alpha=0.0, c=C_PY, hext=(0, 0, h0), hac=(0, 0, h1), freq=f, phase=ph,
                 hpulse=(0, 0, hp), tpulse=tp, wpulse=w, dtau=0.01, tau0=3.0)
    th0, ph0 = 1.1, -0.4
    m0 = torch.tensor([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)],
                      dtype=torch.float64).view(3, 1, 1)
    n = 5000
    m = rk4_step(m0, d, prm, n)
    t0, t1 = 3.0, 3.0 + n * 0.01
    integ = (h0 - (nz - nx) * math.cos(th0)) * (t1 - t0)
    integ += h1 * (math.cos(2 * math.pi * f * t0 + ph) - math.cos(2 * math.pi * f * t1 + ph)) / (2 * math.pi * f)
    integ += hp * w * math.sqrt(math.pi / 2) * (math.erf((t1 - tp) / (math.sqrt(2) * w))
                                                - math.erf((t0 - tp) / (math.sqrt(2) * w)))
    phi = ph0 - C_PY * integ
    ref = torch.tensor([math.sin(th0) * math.cos(phi), math.sin(th0) * math.sin(phi), math.cos(th0)],
                       dtype=torch.float64).view(3, 1, 1)
    assert float((m - ref).abs().max()) < 1e-10


def _drive(dtau):
    return Params(alpha=0.05, c=C_PY, dtau=dtau, hext=(0.02, 0.0, 0.0), hac=(0.0, 0.4, 0.3), freq=0.9,
                  phase=0.2, hpulse=(0.5, -0.2, 0.0), tpulse=0.4, wpulse=0.15, tau0=0.1)


def test_rk4_with_a_driven_field_is_fourth_order():
    d = Disk(8, 6, 2.0)
    m0 = torch.from_numpy(li.smooth_random_field(d.D, 2))
    T = 0.8
    errs = []
    ref = rk4_step(m0, d, _drive(T / 320), 320)
    for n in (20, 40):
        errs.append(float((rk4_step(m0, d, _drive(T / n), n) - ref).abs().max()))
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


def test_zero_temperature_heun_with_a_driven_field_is_second_order():
    d = Disk(8, 6, 2.0)
    m0 = torch.from_numpy(li.smooth_random_field(d.D, 4))
    T = 0.8
    ref = rk4_step(m0, d, _drive(T / 400), 400)
    errs = [float((heun_step(m0, d, _drive(T / n), seed=1, step0=0, nsteps=n) - ref).abs().max())
            for n in (40, 80)]
    assert 3.2 < errs[0] / errs[1] < 4.8, errs


def test_energy_takes_the_field_at_tau0():
    d = Disk(10, 5, 2.0)
    m = torch.from_numpy(li.smooth_random_field(d.D, 7))
    p = _drive(0.01)
    e = energy(m, d, p)
    h = p.field_at(p.tau0)
    e_const = energy(m, d, Params(alpha=p.alpha, c=p.c, hext=h))
    assert abs(e[0] - e_const[0]) < 1e-12 and abs(e[3] - e_const[3]) < 1e-12
