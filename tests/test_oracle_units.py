"""Oracle pins: the unit system and collective-coordinate relations against the
numbers the paper prints (tests/golden/paper_numbers.txt, each with its section)."""
import math
import os

import pytest

from oracle import Material
from oracle import collective as col
from oracle.units import KB, MU0, dimensionless

HERE = os.path.dirname(__file__)


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_numbers.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, val, tol = line.split()[:3]
            out[name] = (float(val), float(tol))
    return out


G = _golden()
PY = Material()
A_NM = 2.0


def close(name, got):
    val, tol = G[name]
    assert abs(got - val) <= tol * abs(val), f"{name}: {got} vs paper {val} (rel tol {tol})"


def test_units_permalloy():
    d = dimensionless(PY, A_NM, 5.0, T_K=300.0)
    close("lambda_ex_nm", d["lambda_ex_nm"])
    close("mu0Ms_T", d["mu0Ms"])
    close("t0_ps", d["t0_ps"])
    close("J_zJ_L5", d["J"] * 1e21)
    close("kT_zJ_300K", KB * 300 * 1e21)
    close("temp_L5_300K", d["temp"])
    close("freq_unit_GHz", MU0 / (4 * math.pi) * PY.gamma * PY.Ms / 1e9)
    close("kT_over_Aa_300K", KB * 300 / (PY.A * A_NM * 1e-9))


def test_units_printed_with_rounded_exchange_length():
    # The paper quotes B0 and f0 from lambda_ex rounded to 5.3 nm:
    # B0 = (lambda_ex/a)^2 mu0 Ms (eq. for B0 in Sec. III.A).
    lam = 5.3
    B0 = (lam / A_NM) ** 2 * MU0 * PY.Ms
    close("B0_T", B0)
    close("f0_THz", PY.gamma * B0 / 1e12)
    # the exact formula 2A/(a^2 Ms) agrees with the rounded one to the rounding
    d = dimensionless(PY, A_NM, 5.0)
    assert abs(d["B0"] - 2 * PY.A / ((A_NM * 1e-9) ** 2 * PY.Ms)) < 1e-12
    assert abs(d["B0"] / B0 - (d["lambda_ex_nm"] / lam) ** 2) < 1e-12


def test_period_conversion():
    d = dimensionless(PY, A_NM, 5.0)
    # printed with t0 rounded to 0.75 ps
    close("period_ns_2020", 2020 * 0.75e-3)
    close("freq_GHz_2020", 1.0 / (2020 * 0.75e-12) / 1e9)
    assert abs(2020 * d["t0_ps"] * 1e-3 - 1.51) < 0.02


def test_linear_law_coefficients():
    lam = 5.3e-9
    a = A_NM * 1e-9
    close("kF_linear_coef", lam * lam / (8 * a * a))
    # Omega_G for the linear law equals L/(16 pi R) (Sec. IV.B)
    L, R = 20e-9, 100e-9
    kF = col.kF_linear(PY, a, L, R)
    Om = col.Omega_dimensionless(kF, PY, a, L, Q=1)
    close("OmegaG_linear", -Om / (L / R))
    assert abs(-Om - L / (16 * math.pi * R)) < 1e-15


def test_thiele_forms_agree():
    a, L = 2e-9, 10e-9
    kF = 1e-4
    d = dimensionless(PY, A_NM, L * 1e9)
    om = col.omega_thiele(kF, PY, L, Q=1)
    Om1 = om * d["t0_ps"] * 1e-12
    Om2 = col.Omega_dimensionless(kF, PY, a, L, Q=1)
    Om3 = col.Omega_from_kt(col.kt_from_kF(kF, PY, a, L), Q=1)
    assert abs(Om1 / Om2 - 1) < 1e-12 and abs(Om3 / Om2 - 1) < 1e-12
    assert Om2 < 0   # positive gyrovector: clockwise (Sec. IV)


def test_rms_radius_predictions():
    kT = KB * 300.0
    for name, kF_units in (("rrms_nm_kF029", 0.29), ("rrms_nm_kF0080", 0.080)):
        kF = kF_units * PY.A / (A_NM * 1e-9)
        close(name, col.r_rms(kT, kF) * 1e9)


def test_gyrotropic_mass():
    close("mG_kg_R100", col.gyro_mass_linear(PY, 100e-9, A_NM * 1e-9))
    # m_G = G^2/k_F with the linear law reproduces the closed form (thickness cancels)
    a, R = A_NM * 1e-9, 100e-9
    for L in (5e-9, 10e-9, 20e-9):
        kF = col.kF_linear(PY, a, L, R)
        assert abs(col.gyro_mass(PY, L, kF) / col.gyro_mass_linear(PY, R, a) - 1) < 1e-12


def test_boltzmann_radial_density():
    kT, kF = 2.0, 0.5
    rmax = math.sqrt(kT / kF)
    p = lambda r: col.p_radial(r, kT, kF)
    assert abs(p(rmax) - math.exp(-0.5) / rmax) < 1e-12
    assert p(rmax) > p(0.99 * rmax) and p(rmax) > p(1.01 * rmax)
    from scipy.integrate import quad
    norm = quad(p, 0, math.inf)[0]
    r2 = quad(lambda r: r * r * p(r), 0, math.inf)[0]
    assert abs(norm - 1) < 1e-9 and abs(r2 - 2 * kT / kF) < 1e-8
