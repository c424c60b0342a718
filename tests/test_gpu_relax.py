"""GPU constrained relaxation (llg_relax) against the float64 oracle."""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.observables import energy as o_energy, vortex_core_position as o_core
from oracle.relax import relax as o_relax

pytestmark = pytest.mark.gpu
C_PY = 0.14298555
LAM = 5.28906


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").reshape(-1).contiguous()


def start(D, X_nm, Y_nm=0.0):
    return li.vortex_ansatz(D, X_nm / 2.0 + 1e-3, Y_nm / 2.0 + 1e-3)


@pytest.mark.parametrize("R,L,X,cut", [(20.0, 10.0, 3.0, 0.0), (30.0, 10.0, 4.0, 0.0), (31.0, 12.0, -2.5, 0.0),
                                       (30.0, 10.0, 4.0, 4 * LAM), (41.0, 8.0, 5.0, 4 * LAM)])
def test_relax_matches_oracle(R, L, X, cut):
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.build(R, L)
    D = disk.D[0]
    od = oracle.Disk(R, L)
    m0 = start(D, X)
    m = dev(m0)
    p = LLGParams(c=C_PY)
    out = disk.relax(m, [(X, 0.0)], p, tol=2e-6, cutoff_nm=cut).cpu()[0]
    disk.check()
    assert float(out[3]) < 2e-6 and abs(float(out[4])) < 2e-6
    mo, lam, it, res, C = o_relax(torch.tensor(m0), od, oracle.Params(c=C_PY), (X, 0.0), tol=1e-11,
                                  cutoff_nm=cut if cut > 0 else None)
    got = m.view(3, D, D).double().cpu()
    # a residual tol leaves the soft modes of the relaxed state uncertain by about
    # tol over the smallest stiffness; the energy is second order in that error
    assert float((got - mo).abs().max()) < 1e-3
    assert abs(float(out[0]) - float(lam[0])) <= 1e-2 * abs(float(lam[0])) + 1e-7
    e_gpu = disk.energy(m, p).cpu()[0, 0].item()
    e_ref = o_energy(mo, od, oracle.Params(c=C_PY))[0]
    assert abs(e_gpu - e_ref) <= 2e-7 * abs(e_ref)
    xc, yc, *_ = o_core(got, od, LAM)
    assert abs(xc - X) < 0.3


def test_batched_relaxations_equal_single_disks():
    # one launch relaxes the same disk at several positions
    from paper_1207_2192_amd import Disk, LLGParams
    Xs = [2.0, 4.0, 6.0]
    batch = Disk.batch([30.0] * 3, [10.0] * 3)
    D = batch.D[0]
    m = batch.pack([dev(start(D, X)) for X in Xs])
    p = LLGParams(c=C_PY)
    out = batch.relax(m, [(X, 0.0) for X in Xs], p, tol=2e-6).cpu()
    batch.check()
    E = batch.energy(m, p).cpu()[:, 0]
    single = Disk.build(30.0, 10.0)
    for k, X in enumerate(Xs):
        ms = dev(start(D, X))
        o1 = single.relax(ms, [(X, 0.0)], p, tol=2e-6).cpu()[0]
        # float64 partial sums are grouped by the launch plan, so agreement is to rounding
        assert abs(float(o1[0]) - float(out[k, 0])) <= 1e-6 * abs(float(out[k, 0]))
        assert float((ms - batch.unpack(m, k).reshape(-1)).abs().max()) < 1e-5
        assert abs(float(single.energy(ms, p).cpu()[0, 0]) - float(E[k])) <= 1e-8 * abs(float(E[k]))
    assert E[0] < E[1] < E[2]          # U grows with the displacement
