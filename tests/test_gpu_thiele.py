"""Thiele check on the gyrotropic disk (Permalloy R = 100 nm, L = 20 nm,
a = 2 nm): constrained relaxations at X = 0, 2, ..., 20 nm in one batched
launch (constraint over the cells within 4 lambda_ex of X) give U(X) and the
static stiffness (Sec. IV.B); the vortex relaxed at
X = 10 nm, released at alpha = 0 with RK4, circles at the rate
Omega(r) = -Q U'(r)/(2 pi r) the static fit predicts (Sec. IV, eqs. wG, OG).
The relaxed energies are checked against the float64 oracle's energy of the
same states."""
import math

import numpy as np
import pytest
import torch

import llg_inputs as li
import oracle
from oracle.observables import energy as o_energy
from oracle.relax import fit_kF, thiele_omega

pytestmark = pytest.mark.gpu
C_PY = 0.14298555
LAM = 5.28906


def test_static_stiffness_predicts_gyrotropic_rate():
    from paper_1207_2192_amd import Disk, LLGParams
    R, L, a = 100.0, 20.0, 2.0
    Xs = [0.0] + [2.0 * k for k in range(1, 11)]
    batch = Disk.batch([R] * len(Xs), [L] * len(Xs), a)
    D = batch.D[0]
    m = batch.pack([torch.tensor(li.vortex_ansatz(D, X / a + 1e-3, 1e-3), dtype=torch.float32, device="cuda")
                    .reshape(-1) for X in Xs])
    p = LLGParams(c=C_PY)
    # constraint over the core region (4 lambda_ex around X), as the core position is defined
    out = batch.relax(m, [(X, 0.0) for X in Xs], p, tol=2e-6, max_sweeps=200000, cutoff_nm=4 * LAM).cpu()
    batch.check()
    assert float(out[:, 3].max()) < 2e-6, out[:, 2:4]
    U = batch.energy(m, p).cpu()[:, 0].double().numpy()
    core = batch.vortex_core_position(m, LAM).cpu().double().numpy()
    r = np.hypot(core[:, 0], core[:, 1]) / a
    print("\nX (nm):", Xs, "\nr_c (nm):", np.round(r * a, 3), "\nU - U0:", U - U[0], "\nrelax:", out[:, :6].numpy())
    # the relaxed energies agree with the float64 oracle's energy of the same states
    od = oracle.Disk(R, L, a)
    for k in (0, 5, 10):
        mk = batch.unpack(m, k).view(3, D, D).double().cpu()
        assert abs(o_energy(mk, od, oracle.Params(c=C_PY))[0] - U[k]) <= 2e-7 * abs(U[k])
    assert np.all(np.diff(U) > 0)                 # U grows with the displacement
    kt, k4 = fit_kF(r[1:], U[1:] - U[0])
    law = L / (8.0 * R)                           # loose linear law of Sec. IV.B in simulation units
    # free gyration from the state relaxed at X = 10 nm
    single = Disk.build(R, L, a)
    m5 = batch.unpack(m, 5).clone().contiguous()
    dyn = LLGParams(alpha=0.0, c=C_PY, dtau=0.04)
    pos = []
    for _ in range(60):
        single.rk4_step(m5, 500, dyn)
        c = single.vortex_core_position(m5, LAM).cpu()[0]
        pos.append((float(c[0]), float(c[1])))
    single.check()
    pos = np.array(pos)
    t = (np.arange(60) + 1) * 500 * 0.04
    ang = np.unwrap(np.arctan2(pos[:, 1], pos[:, 0]))
    om = np.polyfit(t, ang, 1)[0]
    rr = float(np.hypot(pos[:, 0], pos[:, 1]).mean() / a)
    pred = thiele_omega(kt, k4, rr, Q=1)
    print(f"\nkt = {kt:.5f} (L/8R = {law:.5f}), k4 = {k4:.3e}; orbit radius {rr * a:.2f} nm; "
          f"Omega dynamic {om:.5f}, static prediction {pred:.5f} (ratio {om / pred:.3f}) per t0")
    assert 0.7 < kt / law < 1.3
    assert om < 0 and pred < 0                    # clockwise for a positive gyrovector
    assert abs(om / pred - 1) < 0.15
    assert abs(ang[-1] - ang[0]) > math.pi        # more than half an orbit was followed
