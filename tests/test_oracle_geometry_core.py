"""Oracle pins for the disk mask (cell count N_c) and for core_centroid, the
differentiable core-position function behind every trajectory-gradient test.

N_c: the rule "cell centre inside or on the circle of radius R" (Sec. II.A)
fixes the count.  It is pinned by an independent row-by-row count with the
integer square root (no floating point) and by the values that rule gives
for the four single-disk sizes of the benchmark workloads: D = 30 (R = 30 nm),
D = 80 (R = 80 nm), D = 100 (R = 100 nm) and D = 250 (R = 250 nm).

core_centroid: with the plaquette r_v and the cutoff set frozen from
vortex_core_position, it must reproduce that function's r_c (Sec. IV), also
in the fallback without a +1 plaquette; and on states whose m_z^2 weights
are hand-placed it must give the weighted mean the definition fixes.
"""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
from oracle import Disk
from oracle.observables import core_centroid, vortex_core_position

LAM = 5.28906


def count_by_rows(D: int) -> int:
    """Cells whose centre (x, y) = (i - (D-1)/2, j - (D-1)/2) has x^2 + y^2 <= (D/2)^2,
    counted row by row in integers: with X = 2x, Y = 2y (integers of the parity of
    D - 1), the condition reads X^2 + Y^2 <= D^2."""
    total = 0
    for j in range(D):
        Y = 2 * j - (D - 1)
        rem = D * D - Y * Y
        if rem < 0:
            continue
        xmax = math.isqrt(rem)                  # |X| <= xmax, X of the parity of D - 1
        # X = 2 i - (D - 1) runs over i = 0 .. D-1; count i with |2i - (D-1)| <= xmax
        lo = max(0, -((xmax - (D - 1)) // 2))         # ceil((D - 1 - xmax) / 2)
        hi = min(D - 1, (D - 1 + xmax) // 2)
        total += max(0, hi - lo + 1)
    return total


@pytest.mark.parametrize("R,D,Nc", [(30.0, 30, 716), (80.0, 80, 5024), (100.0, 100, 7860), (250.0, 250, 49080)])
def test_cell_count_of_workload_disks(R, D, Nc):
    d = Disk(R, 10.0, 2.0)
    assert d.D == D
    assert d.n_cells == Nc
    assert count_by_rows(D) == Nc


@pytest.mark.parametrize("D", list(range(1, 40)) + [57, 64, 99, 120, 128, 201, 256])
def test_cell_count_matches_integer_row_count(D):
    d = Disk(D * 1.0, 5.0, 2.0)
    assert d.n_cells == count_by_rows(D)
    # four-fold symmetry of the mask about the disk centre
    M = d.mask
    assert torch.equal(M, M.flip(0)) and torch.equal(M, M.flip(1)) and torch.equal(M, M.t())
    # Gauss circle bound: the count is within a perimeter's worth of cells of the area
    assert abs(d.n_cells - math.pi * D * D / 4.0) <= 2.0 * math.pi * D / 2.0 + 4.0


def _states(D):
    yield li.vortex_ansatz(D, 0.3, -0.2)
    yield li.vortex_ansatz(D, 4.7, 2.1)
    yield li.vortex_ansatz(D, -6.2, 3.3, core_width=3.5)
    yield li.smooth_random_field(D, 11)
    # uniform in-plane state with a weak out-of-plane bump: no +1 plaquette
    u = np.zeros((3, D, D))
    x, y = li.cell_centres(D)
    u[2] = 0.2 * np.exp(-((x - 2.0) ** 2 + (y + 1.0) ** 2) / 8.0)
    u[0] = np.sqrt(1.0 - u[2] ** 2)
    yield u


@pytest.mark.parametrize("R", [20.0, 31.0, 40.0])
def test_core_centroid_equals_core_position_when_frozen(R):
    d = Disk(R, 10.0, 2.0)
    n_fallback = 0
    for s in _states(d.D):
        m = torch.tensor(s, dtype=torch.float64)
        xc, yc, xv, yv, n = vortex_core_position(m, d, LAM)
        rc = core_centroid(m, d, LAM, xv, yv, n > 0)
        assert abs(float(rc[0]) - xc) <= 1e-12 * max(1.0, abs(xc))
        assert abs(float(rc[1]) - yc) <= 1e-12 * max(1.0, abs(yc))
        n_fallback += n == 0
    assert n_fallback >= 1


def test_core_centroid_hand_placed_weights():
    d = Disk(20.0, 10.0, 2.0)          # D = 20, cell centres at half-integers
    D = d.D
    m = torch.zeros(3, D, D, dtype=torch.float64)
    m[0] = 1.0
    # one out-of-plane cell within the cutoff of r_v: r_c is that cell's centre
    j, i = 12, 9
    m[2, j, i] = 0.6
    m[0, j, i] = 0.8
    rc = core_centroid(m, d, LAM, 0.0, 0.0, True)
    assert abs(float(rc[0]) - (i - (D - 1) / 2) * 2.0) < 1e-12
    assert abs(float(rc[1]) - (j - (D - 1) / 2) * 2.0) < 1e-12
    # two cells with weights 1 : 4 -> r_c one fifth of the way from the heavier one
    m[2] = 0.0
    m[2, 10, 10] = 0.5       # weight 0.25, at (0.5, 0.5) a
    m[2, 10, 14] = 1.0       # weight 1.00, at (4.5, 0.5) a
    rc = core_centroid(m, d, LAM, 0.0, 0.0, True)
    assert abs(float(rc[0]) - 2.0 * (0.25 * 0.5 + 1.0 * 4.5) / 1.25) < 1e-12
    assert abs(float(rc[1]) - 2.0 * 0.5) < 1e-12
    # cells beyond the cutoff (4 lambda_ex = 10.58 cells from r_v) carry no weight...
    m[2, 10, 19] = 1.0       # at (9.5, 0.5) a: 9.51 from (0, 0), inside
    m[2, 0, 10] = 1.0        # at (0.5, -9.5) a: 9.51 from (0, 0), inside
    rc_in = core_centroid(m, d, LAM, 0.0, 0.0, True)
    rc_far = core_centroid(m, d, LAM, -8.0 * 2.0, 0.0, True)   # r_v moved: (9.5 + 8)^2 > 10.58^2
    w_near = np.array([0.25, 1.0, 1.0, 1.0])
    xs = np.array([0.5, 4.5, 9.5, 0.5])
    assert abs(float(rc_in[0]) - 2.0 * (w_near * xs).sum() / w_near.sum()) < 1e-12
    # around (-8, 0) a only (0.5, 0.5) lies within 10.58 a; (4.5, 0.5) is 12.5 away, (0.5, -9.5) 12.8
    keep = [(0.25, 0.5, 0.5)]
    ws = sum(w for w, _, _ in keep)
    assert abs(float(rc_far[0]) - 2.0 * sum(w * x for w, x, _ in keep) / ws) < 1e-12
    # ...and the fallback (no vortex) weighs the whole disk
    rc_all = core_centroid(m, d, LAM, float("nan"), float("nan"), False)
    w_all = np.array([0.25, 1.0, 1.0, 1.0])
    ys = np.array([0.5, 0.5, 0.5, -9.5])
    assert abs(float(rc_all[1]) - 2.0 * (w_all * ys).sum() / w_all.sum()) < 1e-12
