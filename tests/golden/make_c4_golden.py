"""Write c4_adjoint.json: the float64 oracle's reference values for the
checkpointed RK4 adjoint workload (Permalloy disk R = 80 nm, L = 10 nm,
a = 2 nm; 50 segments of 100 RK4 steps, dtau = 0.04; start: the vortex
ansatz at X = (10 nm, 0) with a Gaussian core of width 5 nm, polarity +1).

Calls only the oracle (and the seeded input generator).  Stored:
* target:  core positions r_c (nm) at the 51 checkpoints of the oracle run at
           alpha = 0.015 with the exchange length 5 % longer (c / 1.05^2) -
           the target spiral of the trajectory loss;
* primal:  the same for the run at alpha = 0.01 and the nominal exchange
           length, with the plaquette r_v and the vortex flag of every
           checkpoint (the frozen core sets of the loss);
* loss:    L = sum over checkpoints of |r_c - target|^2 at the primal, with
           r_c the m_z^2-weighted centroid over the frozen sets;
* fd:      central finite differences (h = 1e-4) of that loss in alpha and
           in the exchange length lambda_ex (nm), the sets held frozen.
The core-position cutoff is 4 lambda_ex of the nominal exchange length in
every evaluation (one fixed observable for the whole loss).

    python tests/golden/make_c4_golden.py      (about 6 minutes on 8 cores)
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import torch  # noqa: E402

import llg_inputs as li  # noqa: E402
import oracle  # noqa: E402
from oracle.dynamics import rk4_step  # noqa: E402
from oracle.observables import core_centroid, vortex_core_position  # noqa: E402

R_NM, L_NM, A_NM = 80.0, 10.0, 2.0
N_SEG, SEG = 50, 100
DTAU = 0.04
ALPHA0, ALPHA_T = 0.01, 0.015
H = 1e-4


def nominal():
    mat = oracle.Material()
    lam_nm = oracle.units.exchange_length(mat) * 1e9
    return lam_nm


def start_state(D):
    return torch.tensor(li.vortex_ansatz(D, 10.0 / A_NM, 0.01, core_width=5.0 / A_NM), dtype=torch.float64)


def run(disk, m0, alpha, lam_nm, lam_cut_nm, frozen=None):
    """Checkpoint core positions: full vortex_core_position, or the centroid over frozen sets."""
    prm = oracle.Params(alpha=alpha, c=(A_NM / lam_nm) ** 2, dtau=DTAU)
    m = m0.clone()
    out = []
    for s in range(N_SEG + 1):
        if s > 0:
            m = rk4_step(m, disk, prm, SEG)
        if frozen is None:
            out.append(vortex_core_position(m, disk, lam_cut_nm))
        else:
            f = frozen[s]
            rc = core_centroid(m, disk, lam_cut_nm, f[2], f[3], f[4] > 0)
            out.append((float(rc[0]), float(rc[1])))
    return out


def main():
    t0 = time.time()
    disk = oracle.Disk(R_NM, L_NM, A_NM)
    lam = nominal()
    m0 = start_state(disk.D)
    target = run(disk, m0, ALPHA_T, 1.05 * lam, lam)
    print(f"target done {time.time() - t0:.0f} s", flush=True)
    primal = run(disk, m0, ALPHA0, lam, lam)
    print(f"primal done {time.time() - t0:.0f} s", flush=True)
    tgt = [(t[0], t[1]) for t in target]

    def loss(rcs):
        return sum((x - tx) ** 2 + (y - ty) ** 2 for (x, y), (tx, ty) in zip(rcs, tgt))

    L0 = loss([(p[0], p[1]) for p in primal])
    Lap = loss(run(disk, m0, ALPHA0 + H, lam, lam, primal))
    Lam = loss(run(disk, m0, ALPHA0 - H, lam, lam, primal))
    print(f"alpha fd done {time.time() - t0:.0f} s", flush=True)
    Llp = loss(run(disk, m0, ALPHA0, lam + H, lam, primal))
    Llm = loss(run(disk, m0, ALPHA0, lam - H, lam, primal))
    print(f"lambda fd done {time.time() - t0:.0f} s", flush=True)
    rec = {
        "workload": "Permalloy R=80 nm L=10 nm a=2 nm (D=80, P=256), RK4 dtau=0.04, 50 x 100 steps, "
                    "start: vortex ansatz X=(10 nm, 0), core width 5 nm, polarity +1",
        "lambda_ex_nm": lam, "c": (A_NM / lam) ** 2, "alpha": ALPHA0,
        "target_alpha": ALPHA_T, "target_lambda_factor": 1.05, "cutoff_lambda_ex_nm": lam,
        "n_seg": N_SEG, "seg_steps": SEG, "dtau": DTAU,
        "target": [[t[0], t[1]] for t in target],
        "primal": [[p[0], p[1], p[2], p[3], int(p[4])] for p in primal],
        "loss": L0,
        "fd_h": H,
        "dL_dalpha_fd": (Lap - Lam) / (2 * H),
        "dL_dlambda_fd": (Llp - Llm) / (2 * H),
        "generator": "tests/golden/make_c4_golden.py (float64 oracle only)",
    }
    with open(os.path.join(HERE, "c4_adjoint.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("loss", "dL_dalpha_fd", "dL_dlambda_fd")}), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
