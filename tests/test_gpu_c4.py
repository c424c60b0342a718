"""The checkpointed RK4 adjoint workload as configured: Permalloy disk R = 80 nm,
L = 10 nm (D = 80, FFT 256), 50 segments of 100 RK4 steps, loss = sum over the
51 checkpoints of |r_c - target|^2 with the target spiral of the float64
oracle at alpha = 0.015 and a 5 % longer exchange length.

Expected values (tests/golden/c4_adjoint.json) are written by
tests/golden/make_c4_golden.py from the oracle alone: the primal core
trajectory, the loss, and central finite differences (h = 1e-4) of the loss in
alpha and in the exchange length, with the core sets frozen at the primal.
The initial-state gradient is checked against the oracle's autograd on a
shortened horizon of the same disk (the full-horizon autograd graph of the
float64 oracle does not fit in memory)."""
import json
import os

import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.dynamics import rk4_step as o_rk4
from oracle.observables import core_centroid, vortex_core_position as o_core

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    with open(os.path.join(HERE, "golden", "c4_adjoint.json")) as f:
        return json.load(f)


def start(D):
    return li.vortex_ansatz(D, 5.0, 0.01, core_width=2.5)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda").reshape(-1).contiguous()


def test_c4_forward_core_trajectory_matches_oracle():
    from paper_1207_2192_amd import Disk, LLGParams
    g = golden()
    disk = Disk.build(80.0, 10.0)
    assert disk.D[0] == 80 and disk.P[0] == 256 and disk.n_cells[0] == 5024
    m = dev(start(disk.D[0]))
    p = LLGParams(alpha=g["alpha"], c=g["c"], dtau=g["dtau"])
    lam = g["cutoff_lambda_ex_nm"]
    worst = 0.0
    for s in range(g["n_seg"] + 1):
        if s > 0:
            disk.rk4_step(m, g["seg_steps"], p)
        core = disk.vortex_core_position(m, lam).cpu()[0]
        ref = g["primal"][s]
        assert int(core[4]) == ref[4]
        assert abs(float(core[2]) - ref[2]) < 1e-9 and abs(float(core[3]) - ref[3]) < 1e-9   # same plaquette
        worst = max(worst, abs(float(core[0]) - ref[0]), abs(float(core[1]) - ref[1]))
    disk.check()
    # float32 state after 5000 steps: the core path stays within 1e-3 nm of the float64 one
    assert worst < 1e-3, worst


def test_c4_adjoint_gradients_match_oracle_finite_differences():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory, grad_exchange_length
    g = golden()
    disk = Disk.build(80.0, 10.0)
    D = disk.D[0]
    m0 = dev(start(D)).requires_grad_(True)
    al = torch.tensor(g["alpha"], dtype=torch.float64, requires_grad=True)
    c = torch.tensor(g["c"], dtype=torch.float64, requires_grad=True)
    base = LLGParams(alpha=g["alpha"], c=g["c"], dtau=g["dtau"])
    lam = g["cutoff_lambda_ex_nm"]
    rc = core_trajectory(m0, al, c, disk, base, g["n_seg"], g["seg_steps"], lam)
    target = torch.tensor(g["target"], dtype=torch.float64, device="cuda")
    loss = ((rc - target) ** 2).sum()
    loss.backward()
    disk.check()
    assert abs(float(loss.detach()) - g["loss"]) <= 1e-3 * g["loss"]
    ga = float(al.grad)
    gl = float(grad_exchange_length(c.grad, g["c"], g["lambda_ex_nm"]))
    assert abs(ga - g["dL_dalpha_fd"]) <= 1e-2 * abs(g["dL_dalpha_fd"]), (ga, g["dL_dalpha_fd"])
    assert abs(gl - g["dL_dlambda_fd"]) <= 1e-2 * abs(g["dL_dlambda_fd"]), (gl, g["dL_dlambda_fd"])
    assert torch.isfinite(m0.grad).all() and float(m0.grad.abs().max()) > 0


def test_c4_initial_state_gradient_matches_oracle_autograd_short_horizon():
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory
    g = golden()
    disk = Disk.build(80.0, 10.0)
    D = disk.D[0]
    od = oracle.Disk(80.0, 10.0)
    n_seg, seg = 2, 20
    lam = g["cutoff_lambda_ex_nm"]
    tgt = torch.tensor(g["target"][:n_seg + 1], dtype=torch.float64)
    m0 = dev(start(D))
    m0g = m0.clone().requires_grad_(True)
    al = torch.tensor(g["alpha"], dtype=torch.float64, requires_grad=True)
    c = torch.tensor(g["c"], dtype=torch.float64, requires_grad=True)
    base = LLGParams(alpha=g["alpha"], c=g["c"], dtau=g["dtau"])
    rc = core_trajectory(m0g, al, c, disk, base, n_seg, seg, lam)
    loss = ((rc - tgt.cuda()) ** 2).sum()
    loss.backward()
    disk.check()
    m32 = m0.view(3, D, D).double().cpu()
    prm = oracle.Params(alpha=g["alpha"], c=g["c"], dtau=g["dtau"])
    frozen, mo = [], m32.clone()
    for s in range(n_seg + 1):
        if s > 0:
            mo = o_rk4(mo, od, prm, seg)
        frozen.append(o_core(mo, od, lam))
    mr = m32.clone().requires_grad_(True)
    ao = torch.tensor(g["alpha"], dtype=torch.float64, requires_grad=True)
    co = torch.tensor(g["c"], dtype=torch.float64, requires_grad=True)
    x, Lo = mr, 0.0
    for s in range(n_seg + 1):
        if s > 0:
            x = o_rk4(x, od, oracle.Params(alpha=ao, c=co, dtau=g["dtau"]), seg)
        f = frozen[s]
        Lo = Lo + ((core_centroid(x, od, lam, f[2], f[3], f[4] > 0) - tgt[s]) ** 2).sum()
    gm, ga, gc = torch.autograd.grad(Lo, (mr, ao, co))
    assert abs(float(loss.detach()) - float(Lo)) <= 1e-4 * abs(float(Lo))
    got = m0g.grad.view(3, D, D).double().cpu()
    gm = od.apply_mask(gm)
    assert float((got - gm).abs().max()) <= 2e-3 * float(gm.abs().max())
    assert abs(float(al.grad) - float(ga)) <= 2e-3 * abs(float(ga))
    assert abs(float(c.grad) - float(gc)) <= 2e-3 * abs(float(gc))
