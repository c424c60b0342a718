"""Oracle pins: thin-film Green's kernels (Sec. II.B) against identities, limits
and quadrature that do not reuse the kernel formulas."""
import math

import numpy as np
import pytest
import torch
from scipy.integrate import quad

from oracle.greens import kernels, kzz_unsimplified, self_factors

ELLS = (1.0, 2.5, 5.0, 10.0)


def grid(n=9):
    d = torch.arange(-n, n + 1, dtype=torch.float64)
    v, u = torch.meshgrid(d, d, indexing="ij")
    return u, v


@pytest.mark.parametrize("ell", ELLS)
def test_trace_vanishes_off_origin_and_is_minus_one_at_origin(ell):
    # Away from the source the z-averaged potential is harmonic, so the trace
    # of the kernel vanishes; at the origin N_x + N_y + N_z = 1 (Sec. II.B).
    u, v = grid()
    kxx, kyy, kxy, kzz = kernels(u, v, ell)
    tr = kxx + kyy + kzz
    off = (u != 0) | (v != 0)
    assert float(tr[off].abs().max()) < 1e-15
    c = (u == 0) & (v == 0)
    assert abs(float(tr[c]) + 1.0) < 1e-15


@pytest.mark.parametrize("ell", ELLS)
def test_symmetries_and_sign(ell):
    u, v = grid()
    kxx, kyy, kxy, kzz = kernels(u, v, ell)
    kxx_t, kyy_t, kxy_t, _ = kernels(v, u, ell)
    assert torch.allclose(kyy, kxx_t, rtol=0, atol=1e-17)      # K_yy = K_xx with x,y swapped
    assert torch.allclose(kxy, kxy_t, rtol=0, atol=1e-17)      # K_xy symmetric under swap
    km = kernels(-u, -v, ell)
    for a, b in zip((kxx, kyy, kxy, kzz), km):
        assert torch.equal(a, b)                              # K(-r) = K(r)
    assert bool((kzz < 0).all())                              # G_zz always negative
    # K_xy odd in each coordinate separately
    assert torch.allclose(kernels(-u, v, ell)[2], -kxy, rtol=0, atol=1e-17)


@pytest.mark.parametrize("ell", ELLS)
def test_cancellation_free_kzz_equals_printed_form(ell):
    u, v = grid(6)
    off = (u != 0) | (v != 0)
    a = kernels(u, v, ell)[3][off]
    b = kzz_unsimplified(u, v, ell)[off]
    assert float(((a - b) / b).abs().max()) < 1e-12


@pytest.mark.parametrize("ell", (1.0, 2.5, 5.0))
def test_dipole_far_field(ell):
    # Far from the source the kernels become those of a point dipole of
    # moment ell (cell area 1 times thickness): H = ell (3 (m.r) r/r^2 - m)/(4 pi r^3).
    for (u, v) in ((400.0, 300.0), (-350.0, 120.0), (0.0, 500.0)):
        U, V = torch.tensor([u]), torch.tensor([v])
        kxx, kyy, kxy, kzz = (float(t) for t in kernels(U, V, ell))
        r = math.hypot(u, v)
        pre = ell / (4 * math.pi * r ** 3)
        ref = (pre * (3 * u * u / r ** 2 - 1), pre * (3 * v * v / r ** 2 - 1),
               pre * 3 * u * v / r ** 2, -pre)
        for got, want in zip((kxx, kyy, kxy, kzz), ref):
            assert abs(got - want) < 1e-3 * pre


def test_self_terms_closed_forms_and_limits():
    for ell in ELLS:
        nx, nz = self_factors(ell)
        assert abs(2 * nx + nz - 1) < 1e-15
        # -N_z is the integral of G_zz = (1/(2 pi l))(1/s - 1/r) over the
        # circle of area a^2 (radius 1/sqrt(pi)), done by quadrature.
        ro = 1 / math.sqrt(math.pi)
        integrand = lambda r: (1 / (2 * math.pi * ell)) * (1 / math.sqrt(r * r + ell * ell) - 1 / r) * 2 * math.pi * r
        val = quad(integrand, 0, ro, limit=200)[0]
        assert abs(val + nz) < 1e-10
    # long cells: N_x -> 1/2, N_z -> 0; flat cells: N_z -> 1
    nx, nz = self_factors(1e4)
    assert abs(nx - 0.5) < 1e-4 and nz < 1e-4
    nx, nz = self_factors(1e-4)
    assert abs(nz - 1) < 1e-3
    # the transverse self term enters with a negative sign (demagnetising)
    kxx0 = kernels(torch.tensor([0.0]), torch.tensor([0.0]), 5.0)[0]
    assert float(kxx0) < 0


def test_plane_integral_of_gzz_is_minus_one():
    # Thin-film limit: a uniform out-of-plane m in an infinite film feels
    # H_z = -M_z; the continuum kernel integrates to -1 over the plane.
    for ell in (1.0, 5.0):
        val = quad(lambda r: (1 / ell) * (r / math.sqrt(r * r + ell * ell) - 1), 0, np.inf, limit=400)[0]
        assert abs(val + 1) < 1e-8
