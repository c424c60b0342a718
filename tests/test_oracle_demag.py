"""Oracle pins: the FFT demagnetisation path against the direct real-space sum
(brute force), self-adjointness and the thin-film limit (Sec. II.B)."""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
from oracle import Disk
from oracle.demag import demag_direct, demag_fft


def field(D, seed):
    return torch.from_numpy(li.random_unit_field(D, seed))


@pytest.mark.parametrize("R,L,P", [(1, 5, None), (2, 2, None), (5, 10, None), (12, 10, None),
                                   (15, 5, None), (12, 10, 23), (12, 10, 48), (9, 20, 18)])
def test_fft_equals_direct_sum(R, L, P):
    d = Disk(R, L, 2.0, P=P)
    m = field(d.D, 11 + d.D)
    Hd = demag_direct(m, d)
    Hf = demag_fft(m, d)
    assert float((Hd - Hf).abs().max()) <= 1e-12 * float(Hd.abs().max())


def test_wraparound_is_detected():
    # With P < 2D-1 the circular convolution picks up image cells; the
    # direct sum exposes it (the geometry refuses such P for normal use).
    d = Disk(12, 10, 2.0)
    m = field(d.D, 3)
    d.P = 2 * d.D - 4
    Hw = demag_fft(m, d)
    Hd = demag_direct(m, d)
    assert float((Hw - Hd).abs().max()) > 1e-4


def test_rejects_small_padding():
    with pytest.raises(ValueError):
        Disk(12, 10, 2.0, P=22)


def test_self_adjoint():
    d = Disk(14, 7, 2.0)
    u, v = field(d.D, 1), field(d.D, 2)
    lhs = float((u * demag_fft(v, d)).sum())
    rhs = float((demag_fft(u, d) * v).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_values_outside_mask_are_ignored():
    d = Disk(10, 5, 2.0)
    m = field(d.D, 4)
    junk = m.clone()
    junk[:, ~d.mask] = 7.0
    assert torch.equal(demag_fft(m, d), demag_fft(junk, d))
    assert float(demag_fft(m, d)[:, ~d.mask].abs().max()) == 0.0


def test_uniform_out_of_plane_demagnetises_and_tends_to_thin_film_limit():
    # uniform m_z: H_z < 0 everywhere; at the centre of a wide disk it
    # approaches the continuum value (1/l)(sqrt(R^2+l^2) - R - l) -> -1.
    for ell, Rc in ((2.5, 60), (5.0, 80)):
        d = Disk(Rc * 2.0, ell * 2.0, 2.0)
        m = torch.zeros(3, d.D, d.D, dtype=torch.float64)
        m[2] = 1.0
        H = demag_fft(m, d)
        assert bool((H[2][d.mask] < 0).all())
        assert float(H[0].abs().max()) < 1e-12 and float(H[1].abs().max()) < 1e-12
        c = d.D // 2
        hz0 = float(H[2, c - 1:c + 1, c - 1:c + 1].mean())
        cont = (math.sqrt(Rc * Rc + ell * ell) - Rc - ell) / ell
        assert abs(hz0 - cont) < 0.1 / ell
        assert hz0 < -0.85


def test_uniform_in_plane_field_is_small_and_antiparallel():
    d = Disk(60, 5, 2.0)
    m = torch.zeros(3, d.D, d.D, dtype=torch.float64)
    m[0] = 1.0
    H = demag_fft(m, d)
    hx = H[0][d.mask]
    assert float(hx.mean()) < 0 and float(hx.mean()) > -0.1   # thin disk: in-plane N small
    assert float(H[2].abs().max()) < 1e-12
