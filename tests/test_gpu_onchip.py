"""Spectra on chip (llg_set_on_chip): disks of FFT size 64 and 128 stepped by
one workgroup each with their row/column spectra in LDS.

Parity against the float64 oracle at the tolerances of test_gpu_parity.py
(fields and right-hand sides 1e-5 norm-wise, states after a few steps 2e-6
absolute), and bitwise equality with the same steps taken with the spectra in
global memory: the on-chip path changes where the spectra live, not how any
value is computed, so every state must come out bit for bit the same.  Also
the graph, the entry point without allocation, the adjoint and relaxation
kernels (which keep the spectra in global memory) on a handle whose plan
puts disks on chip, the autotuner's on-chip candidates and the error path."""
import ctypes

import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.demag import demag_fft
from oracle.dynamics import heun_step as o_heun, llg_rhs as o_rhs, rk4_step as o_rk4
from oracle.observables import energy as o_energy

pytestmark = pytest.mark.gpu
C_PY = 0.14298555


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").reshape(-1).contiguous()


def rel(got, ref):
    return float((got - ref).abs().max() / ref.abs().max())


# ragged batch: P = 64, 128, 128, 64, 256, 64 (odd and even D)
RS = [30.0, 61.0, 40.0, 15.0, 100.0, 31.0]
LS = [10.0, 12.0, 4.0, 5.0, 20.0, 20.0]


def ragged():
    from paper_1207_2192_amd import Disk
    batch = Disk.batch(RS, LS)
    states = [li.vortex_ansatz(D, 1.3 + 0.5 * k, -0.7) for k, D in enumerate(batch.D)]
    m = batch.pack([dev(s) for s in states])
    return batch, states, m


@pytest.mark.parametrize("R,L,P", [(15.0, 5.0, 0), (30.0, 10.0, 0), (31.0, 20.0, 0), (40.0, 7.5, 0),
                                   (61.0, 12.0, 0), (64.0, 10.0, 0), (30.0, 10.0, 128)])
@pytest.mark.parametrize("pol", [0, 1, 2, 3])
def test_field_rhs_energy_on_chip_match_oracle(R, L, P, pol):
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.build(R, L, 2.0, P)
    ug = 1
    disk.tune(ug, None, pol)
    disk.set_on_chip(disk.P[0])
    assert disk.on_chip == disk.P[0] and disk.workgroups == [1]
    od = oracle.Disk(R, L, 2.0, P=P or None)
    D = disk.D[0]
    print(f"on-chip field R={R} D={D} P={disk.P[0]} ug={ug} pol={pol}", flush=True)
    m0 = li.random_unit_field(D, 40 + D)
    H = disk.demag_field(dev(m0)).view(3, D, D).double().cpu()
    disk.check()
    assert rel(H, demag_fft(torch.tensor(m0), od)) <= 1e-5
    p = LLGParams(alpha=0.1, c=C_PY, hext=(0.02, -0.01, 0.005))
    po = oracle.Params(alpha=0.1, c=C_PY, hext=(0.02, -0.01, 0.005))
    f = disk.rhs(dev(m0), p).view(3, D, D).double().cpu()
    assert rel(f, o_rhs(torch.tensor(m0), od, po)) <= 1e-5
    # energy parts (float64 sums of float32 fields) of the float32-rounded input
    e = disk.energy(dev(m0), p).cpu()[0]
    eo = o_energy(torch.tensor(m0, dtype=torch.float32).double(), od, po)
    for k in range(4):
        assert abs(float(e[k]) - eo[k]) <= 1e-6 * abs(eo[0]) + 1e-12, k


def test_ragged_batch_on_chip_matches_oracle_and_global_spectra():
    from paper_1207_2192_amd import LLGParams
    batch, states, m0 = ragged()
    ps = [LLGParams(alpha=0.02 * (k + 1), c=C_PY, dtau=0.04) for k in range(batch.n)]
    ref = m0.clone()
    batch.rk4_step(ref, 4, ps)
    for max_p in (64, 128):
        batch.set_on_chip(max_p)
        assert [w for w, P in zip(batch.workgroups, batch.P) if P <= max_p] == [1] * sum(P <= max_p for P in batch.P)
        m = m0.clone()
        batch.rk4_step(m, 4, ps)
        batch.check()
        assert torch.equal(m, ref), max_p
    for k, (R, L) in enumerate(zip(RS, LS)):
        od = oracle.Disk(R, L)
        o = o_rk4(torch.tensor(states[k]), od, oracle.Params(alpha=0.02 * (k + 1), c=C_PY, dtau=0.04), 4)
        assert float((batch.unpack(ref, k).double().cpu() - o).abs().max()) <= 2e-6, k
    batch.set_on_chip(0)
    assert batch.on_chip == 0


@pytest.mark.parametrize("fd", [False, True])
def test_heun_on_chip_matches_oracle_and_global_spectra(fd):
    from paper_1207_2192_amd import LLGParams
    batch, states, m0 = ragged()
    ps = [LLGParams(alpha=0.1, c=C_PY, temp=0.0319, dtau=0.0266, renorm=True, fd_factor=fd)] * batch.n
    ref = m0.clone()
    batch.heun_step(ref, 6, ps, seed=91, step0=300, replica=3)
    batch.set_on_chip(128)
    m = m0.clone()
    batch.heun_step(m, 6, ps, seed=91, step0=300, replica=3)
    batch.check()
    assert torch.equal(m, ref)
    po = oracle.Params(alpha=0.1, c=C_PY, temp=0.0319, dtau=0.0266, renorm=True, fd_factor=fd)
    for k in (0, 1, 3):   # P = 64, 128, 64: disk k takes replica 3 + k
        od = oracle.Disk(RS[k], LS[k])
        o = o_heun(torch.tensor(states[k]), od, po, seed=91, step0=300, replica=3 + k, nsteps=6)
        assert float((batch.unpack(m, k).double().cpu() - o).abs().max()) <= 5e-6, k


def test_series_on_chip_equals_global_spectra():
    from paper_1207_2192_amd import LLGParams
    batch, _, m0 = ragged()
    ps = [LLGParams(alpha=0.05, c=C_PY, dtau=0.04, hext=(0.01, 0.0, 0.0))] * batch.n
    a, b = m0.clone(), m0.clone()
    batch.tune(1, [1] * batch.n, 0)       # the same workgroup per disk in both runs
    sa = batch.rk4_series(a, 12, ps, 3)
    batch.set_on_chip(128)
    sb = batch.rk4_series(b, 12, ps, 3)
    batch.check()
    assert torch.equal(a, b)
    small = [k for k, P in enumerate(batch.P) if P <= 128]
    # one workgroup per disk in both plans: the float64 sums run in the same order
    assert torch.equal(sa[:, small], sb[:, small])
    assert float((sa - sb).abs().max()) <= 1e-12 * float(sa.abs().max())


def test_graph_and_noalloc_on_chip():
    from paper_1207_2192_amd import LLGParams, _lib
    batch, _, m0 = ragged()
    batch.set_on_chip(128)
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04)] * batch.n
    mg, me = m0.clone(), m0.clone()
    g = batch.graph("rk4", mg, 9, p)
    for rep in range(3):
        g.launch()
        x = torch.randn(1 << 18, device="cuda")
        float((x * x).sum())
        batch.rk4_step(me, 9, p)
        torch.cuda.synchronize()
        batch.check()
        assert torch.equal(mg, me), rep
    g.close()
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    got = m0.clone()
    assert lib.llg_noalloc_bytes(batch._h) <= 32 << 20
    rc = lib.llg_rk4_step_noalloc(batch._h, ctypes.c_void_p(got.data_ptr()), 9, batch._params(p), stream)
    assert rc == 0, lib.llg_last_error()
    ref = m0.clone()
    batch.rk4_step(ref, 9, p)
    torch.cuda.synchronize()
    batch.check()
    assert torch.equal(got, ref)


def test_adjoint_and_relaxation_on_a_plan_with_disks_on_chip():
    # those kernels keep the spectra in global memory; with one workgroup per
    # disk in both plans (the same float64 reduction order) every result agrees
    # bit for bit
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.batch([30.0, 61.0], [10.0, 12.0])
    m0 = disk.pack([dev(li.smooth_random_field(D, 8 + D)) for D in disk.D])
    yb0 = disk.pack([dev(li.random_unit_field(D, 2 + D)) for D in disk.D])
    p = [LLGParams(alpha=0.07, c=C_PY, dtau=0.05)] * disk.n
    n = 3

    def vjp():
        m = m0.clone()
        rec = torch.empty(8 * n * disk.state_size, dtype=torch.float32, device="cuda")
        disk.rk4_record(m, n, p, rec)
        yb = yb0.clone()
        pg = torch.zeros(2 * disk.n, dtype=torch.float64, device="cuda")
        disk.rk4_vjp(rec, n, yb, pg, p)
        disk.check()
        return m, yb, pg

    disk.tune(1, [1, 1], 0)
    m_a, yb_a, pg_a = vjp()
    disk.set_on_chip(128)
    assert disk.workgroups == [1, 1]
    m_b, yb_b, pg_b = vjp()
    assert torch.equal(m_a, m_b)
    assert torch.equal(yb_a, yb_b)
    assert torch.equal(pg_a, pg_b)
    # relaxation towards a displaced core: the same result on both plans
    X = [(4.0, -2.0), (6.0, 3.0)]
    pr = [LLGParams(alpha=0.0, c=C_PY)] * disk.n
    r_b = m0.clone()
    out_b = disk.relax(r_b, X, pr, max_sweeps=300)
    disk.set_on_chip(0)
    disk.tune(1, [1, 1], 0)
    r_a = m0.clone()
    out_a = disk.relax(r_a, X, pr, max_sweeps=300)
    disk.check()
    assert torch.equal(r_a, r_b)
    assert torch.equal(out_a, out_b)


def test_autotune_may_choose_on_chip_and_keeps_parity():
    from paper_1207_2192_amd import Disk, LLGParams
    disk = Disk.batch([30.0] * 8, [10.0] * 8)
    od = oracle.Disk(30.0, 10.0)
    D = disk.D[0]
    s0 = li.vortex_ansatz(D, 2.0, 1.0)
    m0 = disk.pack([dev(s0)] * disk.n)
    p = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04)] * disk.n
    us = disk.autotune(m0, p, "rk4", probe_steps=30)
    print("autotuned", us, "us/step, on chip:", disk.on_chip, disk.launch_shape(), flush=True)
    assert us > 0 and disk.on_chip in (0, 64)
    m = m0.clone()
    disk.rk4_step(m, 5, p)
    disk.check()
    ref = o_rk4(torch.tensor(s0), od, oracle.Params(alpha=0.02, c=C_PY, dtau=0.04), 5)
    for k in range(disk.n):
        assert float((disk.unpack(m, k).double().cpu() - ref).abs().max()) <= 5e-6


def test_bad_on_chip_requests_keep_the_plan():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd._lib import LLGError
    disk = Disk.build(61.0, 12.0)
    with pytest.raises(LLGError):
        disk.set_on_chip(96)
    with pytest.raises(LLGError):
        disk.set_on_chip(256)
    assert disk.on_chip == 0
    m0 = dev(li.vortex_ansatz(disk.D[0], 1.0, 2.0))
    p = LLGParams(alpha=0.05, c=C_PY, dtau=0.04)
    ref = m0.clone()
    disk.rk4_step(ref, 3, p)
    # on-chip instances have one group of three wavefronts per workgroup: with
    # four the request is refused and the previous plan stays in force
    disk.tune(4, None, 0)
    with pytest.raises(LLGError):
        disk.set_on_chip(128)
    assert disk.on_chip == 0 and disk.launch_shape()[0] == 4
    m = m0.clone()
    disk.rk4_step(m, 3, p)
    disk.check()
    assert torch.equal(m, ref)
    # and a wider re-plan while disks are on chip is refused too
    disk.tune(1, None, 0)
    disk.set_on_chip(128)
    with pytest.raises(LLGError):
        disk.tune(2, None, 0)
    assert disk.on_chip == 128 and disk.workgroups == [1]
    m = m0.clone()
    disk.rk4_step(m, 3, p)
    disk.check()
    assert torch.equal(m, ref)
