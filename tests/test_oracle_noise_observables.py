"""Oracle pins: Philox4x32-10 against the known-answer vectors published with
the Random123 library, the Box-Muller normals, energy decompositions and the
vortex core position (Sec. IV)."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

import llg_inputs as li
from oracle import Disk, Params
from oracle.observables import (energy, energy_from_exchange_field, mean_m, plaquette_windings,
                                vortex_core_position)
from oracle.philox import gaussian_field, philox4x32_10, uniforms24

C_PY = 0.14298555
LAM_NM = 5.28906


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, want):
    # the philox4x32 (10 rounds) known-answer vectors of the Random123 distribution
    got = philox4x32_10([np.uint64(c) for c in ctr], [np.uint64(k) for k in key])
    assert [int(g) for g in got] == list(want)


def test_uniforms_exact_and_open():
    x = np.array([0, 2**32 - 1, 2**8, 2**31, 0xFF], dtype=np.uint64)
    u = uniforms24(x)
    assert u[0] == 0.5 * 2**-24 and u[1] == 1 - 0.5 * 2**-24 and 0 < u.min() and u.max() < 1
    assert u[2] == 1.5 * 2**-24 and u[4] == u[0]          # bit 8 is the lowest kept
    assert u[3] == 0.5 + 0.5 * 2**-24
    assert np.all(u * 2**25 == np.round(u * 2**25))       # multiples of 2^-25: exact in FP32


def test_normals_are_standard_and_independent():
    w = gaussian_field(12072192, 5, np.arange(64), 32)      # [64, 3, 32, 32]
    flat = w.reshape(-1)
    assert abs(flat.mean()) < 0.01 and abs(flat.std() - 1) < 0.01
    assert stats.kstest(flat[:50000], "norm").pvalue > 1e-3
    cxy = np.corrcoef(w[:, 0].ravel(), w[:, 1].ravel())[0, 1]
    cxz = np.corrcoef(w[:, 0].ravel(), w[:, 2].ravel())[0, 1]
    assert abs(cxy) < 0.02 and abs(cxz) < 0.02
    # the two rows of a pair share a block but not its normals
    ce = np.corrcoef(w[:, :, 0::2].ravel(), w[:, :, 1::2].ravel())[0, 1]
    assert abs(ce) < 0.02
    for c in range(3):
        assert abs(w[:, c].mean()) < 0.02 and abs(w[:, c].std() - 1) < 0.02
    # an odd box keeps its last row
    w7 = gaussian_field(3, 2, 0, 7)
    assert w7.shape == (3, 7, 7) and np.all(np.isfinite(w7)) and np.abs(w7[:, 6]).sum() > 0
    # different steps / replicas give unrelated noise
    a = gaussian_field(1, 0, 0, 16).ravel()
    b = gaussian_field(1, 1, 0, 16).ravel()
    c = gaussian_field(1, 0, 1, 16).ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.1 and abs(np.corrcoef(a, c)[0, 1]) < 0.1


def test_energy_forms_agree_and_parts_sum():
    d = Disk(10, 5, 2.0)
    prm = Params(c=C_PY, hext=(0.2, -0.1, 0.3))
    m = torch.from_numpy(li.random_unit_field(d.D, 3))
    e, ex, dm, ext = energy(m, d, prm)
    assert abs(e - (ex + dm + ext)) < 1e-12
    assert abs(e - energy_from_exchange_field(m, d, prm)) < 1e-11


def test_uniform_state_energy_counts_bonds():
    d = Disk(12, 4, 2.0)
    m = torch.zeros(3, d.D, d.D, dtype=torch.float64)
    m[0] = 1.0
    M = d.mask
    bonds = int((M[:, :-1] & M[:, 1:]).sum() + (M[:-1, :] & M[1:, :]).sum())
    e, ex, dm, ext = energy(m, d, Params(c=C_PY))
    assert ex == -bonds and ext == 0.0 and dm > 0   # in-plane demag energy is positive


def test_mean_m():
    d = Disk(8, 4, 2.0)
    m = torch.from_numpy(li.random_unit_field(d.D, 1))
    got = mean_m(m, d)
    for c in range(3):
        assert abs(got[c] - float(m[c][d.mask].sum()) / d.n_cells) < 1e-15


@pytest.mark.parametrize("x0,y0", [(3.3, -1.7), (-5.2, 4.4), (0.2, 0.1), (7.6, 2.8)])
def test_core_position_of_displaced_vortex(x0, y0):
    # r_v within one cell of the vortex centre, r_c within one cell of r_v (Sec. IV)
    d = Disk(40, 10, 2.0)
    m = torch.from_numpy(li.vortex_ansatz(d.D, x0, y0, core_width=2.5))
    xc, yc, xv, yv, n = vortex_core_position(m, d, LAM_NM)
    assert n == 1
    a = d.a_nm
    assert math.hypot(xv / a - x0, yv / a - y0) < 1.0
    assert math.hypot(xc - xv, yc - yv) < a
    assert math.hypot(xc / a - x0, yc / a - y0) < 0.35


def test_core_position_rotates_with_the_state():
    d = Disk(30, 10, 2.0)
    m = torch.from_numpy(li.vortex_ansatz(d.D, 4.2, 1.3))
    r0 = vortex_core_position(m, d, LAM_NM)
    # rotate the state by +90 degrees about the disk centre: positions (x, y) -> (-y, x),
    # vectors likewise; on the grid this is a rot90 of the arrays.
    mr = m.transpose(1, 2).flip(2)                  # new[iy, ix] = old[D-1-ix, iy]
    mr = torch.stack([-mr[1], mr[0], mr[2]])
    r1 = vortex_core_position(mr, d, LAM_NM)
    assert abs(r1[0] + r0[1]) < 1e-9 and abs(r1[1] - r0[0]) < 1e-9


def test_windings_of_vortex_antivortex_and_uniform():
    d = Disk(20, 5, 2.0)
    m = torch.from_numpy(li.vortex_ansatz(d.D, 1.3, -2.2, q=1))
    w = plaquette_windings(m, d)
    assert int((w == 1).sum()) == 1 and int((w == -1).sum()) == 0
    m = torch.from_numpy(li.vortex_ansatz(d.D, 1.3, -2.2, q=-1))
    w = plaquette_windings(m, d)
    assert int((w == -1).sum()) == 1 and int((w == 1).sum()) == 0
    m = torch.zeros(3, d.D, d.D, dtype=torch.float64); m[0] = 1
    assert int(plaquette_windings(m, d).abs().sum()) == 0
    xc, yc, xv, yv, n = vortex_core_position(torch.from_numpy(li.vortex_ansatz(d.D, 1.3, -2.2, q=-1)), d, LAM_NM)
    assert n == 0 and math.isnan(xv)
