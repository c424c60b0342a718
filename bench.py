"""Benchmark: LLG cell-steps/s including the FFT demagnetisation field, one MI355X.

Default workload: a Permalloy disk R = 100 nm, L = 20 nm on a = 2 nm cells
(100 x 100 box, 7860 disk cells, FFT size 256), RK4 at T = 0 with alpha = 0 and
dtau = 0.04, started from a vortex displaced to X = (10 nm, 0).  One step is a
full RK4 step (four field evaluations, each with the zero-padded FFT demag).

Prints one JSON line with the roofline of the persistent kernel and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
C_PY = 0.14298555          # a^2/lambda_ex^2, Permalloy, a = 2 nm
KERNEL_SOURCES = ["paper_1207_2192_amd/csrc/llg_kernels.hpp", "paper_1207_2192_amd/csrc/fft_lds.hpp",
                  "paper_1207_2192_amd/csrc/llg_device.hpp", "paper_1207_2192_amd/csrc/kernels_rk4.hip",
                  "paper_1207_2192_amd/csrc/kernels_heun.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_stage(D: int, P: int) -> int:
    """Algorithmic HBM bytes of one field evaluation + stage update (three-pass model):
    row spectra 3 x H x D complex float32 written and read by each of the two
    phases (4 x 24 D H), the kernel quarter spectra once (16 H^2), the stage
    state, RK accumulator and next state (60 D^2)."""
    H = P // 2 + 1
    return 96 * D * H + 16 * H * H + 60 * D * D


def traffic_record(workload: str):
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def cpu_baseline(R, L, dtau, m0_np, budget_s=15.0):
    """The FP64 oracle on the host cores: RK4 steps of the same disk for ~budget_s."""
    import torch
    import oracle
    from oracle.dynamics import rk4_step
    d = oracle.Disk(R, L, 2.0)
    prm = oracle.Params(alpha=0.0, c=C_PY, dtau=dtau)
    m = torch.tensor(m0_np)
    rk4_step(m, d, prm, 1)                       # warm the FFT plans and the kernel spectra
    t = time.perf_counter()
    rk4_step(m, d, prm, 2)
    per = (time.perf_counter() - t) / 2
    n = max(2, int(budget_s / per))
    t = time.perf_counter()
    rk4_step(m, d, prm, n)
    dt = time.perf_counter() - t
    return dict(value=d.n_cells * n / dt, unit="cell-steps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{n} RK4 steps of the same disk (float64 torch CPU FFT path), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--chunk", type=int, default=5000, help="steps per launch")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--wg", type=int, default=0, help="workgroups for the disk (0 = library choice)")
    ap.add_argument("--ug", type=int, default=0, help="wavefront groups per workgroup (0 = library choice)")
    ap.add_argument("--radix", type=int, default=0, help="transform policy for --ug/--wg (0..3: bit 0 radix 8, bit 1 lane-group columns)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch plan")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--plain", action="store_true", help="loop over single-disk handles instead of one batch")
    ap.add_argument("--sample-every", type=int, default=100,
                    help="steps between observable samples (core position + energy) in the timed region; 0 = none")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent disks shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import llg_inputs as li
    from paper_1207_2192_amd import Disk, LLGParams, params_from_si

    torch.cuda.set_device(0)
    a = 2.0
    PY = li.PERMALLOY
    if args.workload == "c4":
        return adjoint_bench(args)
    if args.workload == "c2":
        Rs, Ls = [100.0], [20.0]
        starts = [(10.0, 0.0)]
        prms = [LLGParams(alpha=0.0, c=C_PY, dtau=0.04)]
        integrator = "rk4"
        desc = ("RK4 T=0 gyrotropic disk: Permalloy R=100 nm L=20 nm a=2 nm, 100x100 box (7860 cells), "
                "FFT 256x256, alpha=0, dtau=0.04, vortex displaced to X=(10 nm,0)")
    elif args.workload == "c3":
        ens = li.ragged_ensemble(256)
        Rs, Ls = [e.R_nm for e in ens], [e.L_nm for e in ens]
        starts = [(e.x0_nm, e.y0_nm) for e in ens]
        prms = [LLGParams(alpha=0.02, c=C_PY, dtau=0.04) for _ in ens]
        integrator = "rk4"
        desc = ("ragged ensemble of 256 Permalloy disks, R in {30..120} nm, L/R in [0.05,0.3], a=2 nm, "
                "RK4 T=0 alpha=0.02 dtau=0.04, vortex offsets 2-15 nm")
    else:  # c5: thermal replicas
        nrep = 64
        Rs, Ls = [250.0] * nrep, [20.0] * nrep
        starts = [(0.0, 0.0)] * nrep
        p0, _ = params_from_si(PY["A"], PY["Ms"], PY["gamma"], a, 20.0, 0.02, 300.0, 0.1)
        p0.renorm = True
        prms = [p0] * nrep
        integrator = "heun"
        desc = ("64 thermal replicas of a Permalloy disk R=250 nm L=20 nm a=2 nm (250x250 box, FFT 512x512), "
                "Heun T=300 K alpha=0.1 dt=0.02 ps, independent Philox streams")
    disk = Disk.batch(Rs, Ls, a) if len(Rs) > 1 else Disk.build(Rs[0], Ls[0], a)
    if args.wg or args.ug:
        disk.tune(args.ug or disk.launch_shape()[0], [args.wg] * disk.n if args.wg else None, args.radix)
    Nc = sum(disk.n_cells)
    states = []
    for k in range(disk.n):
        x0, y0 = starts[k]
        # centred start: nudge off the exact grid symmetry point
        states.append(li.vortex_ansatz(disk.D[k], x0 / a + 0.01, y0 / a + 0.013))
    m = torch.tensor(np.concatenate([s.reshape(-1) for s in states]), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    tuned_us = None
    if not (args.wg or args.ug or args.no_autotune):
        tuned_us = disk.autotune(m, prms, integrator, probe_steps=300 if disk.n == 1 else 40)
        print(f"# autotune: {tuned_us:.2f} us/step with plan {disk.launch_shape()}", file=sys.stderr, flush=True)
    step_counter = [0]

    plain = None
    if args.plain and disk.n > 1:
        plain = [Disk.build(Rs[k], Ls[k], a) for k in range(disk.n)]

    eprm = [LLGParams(c=p.c) for p in prms]
    lam_nm = a / math.sqrt(C_PY)
    samples = []
    kernel_events = []

    def run(nsteps, timed=False):
        """nsteps of the integrator; in the timed region, observables every --sample-every
        steps (their kernels are part of the timed work) and events around each launch."""
        launches = 0
        left = nsteps
        chunk = min(args.chunk, args.sample_every) if (timed and args.sample_every) else args.chunk
        while left > 0:
            k = min(chunk, left)
            if timed:
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                ev[0].record(stream)
            if plain is not None:
                for j, dj in enumerate(plain):
                    mj = m[disk.offsets[j]:disk.offsets[j] + 3 * disk.D[j] ** 2]
                    if integrator == "rk4":
                        dj.rk4_step(mj, k, prms[j])
                    else:
                        dj.heun_step(mj, k, prms[j], seed=20120827, step0=step_counter[0], replica=j)
                    launches += 1
            else:
                if integrator == "rk4":
                    disk.rk4_step(m, k, prms)
                else:
                    disk.heun_step(m, k, prms, seed=20120827, step0=step_counter[0], replica=0)
                launches += 1
            if timed:
                ev[1].record(stream)
                kernel_events.append(ev)
                if args.sample_every:
                    if plain is not None:
                        for j, dj in enumerate(plain):
                            mj = m[disk.offsets[j]:disk.offsets[j] + 3 * disk.D[j] ** 2]
                            samples.append((dj.vortex_core_position(mj, lam_nm), dj.energy(mj, eprm[j:j + 1])))
                    else:
                        samples.append((disk.vortex_core_position(m, lam_nm), disk.energy(m, eprm)))
            step_counter[0] += k
            left -= k
        return launches

    e0 = disk.energy(m, eprm)[:, 0].cpu()
    if args.warmup:
        run(args.warmup)
    torch.cuda.synchronize()
    disk.check()
    print(f"# warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    launches = run(args.steps, timed=True)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    disk.check()
    gpu_s = start.elapsed_time(stop) / 1e3
    e1 = disk.energy(m, eprm)[:, 0].cpu()
    drift = float(((e1 - e0).abs() / e0.abs()).max())
    print(f"# timed {args.steps} steps in {gpu_s:.3f} s (wall {wall:.3f} s), max energy change {drift:.2e}",
          file=sys.stderr, flush=True)

    if args.copy_probe_mib:
        x = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    stages = 4 if integrator == "rk4" else 2
    value = Nc * args.steps / gpu_s
    b_step = sum(bytes_per_stage(disk.D[k], disk.P[k]) for k in range(disk.n)) * stages
    b_launch = b_step * args.steps / launches
    # duration of the integrator launches alone (the observables between them excluded)
    kernel_s = sum(e0.elapsed_time(e1) for e0, e1 in kernel_events) / 1e3
    t_launch = kernel_s / launches
    achieved = b_launch / t_launch / 1e9
    tr = traffic_record(f"{args.workload}_{integrator}")
    traffic = None if tr is None else tr["bytes_per_step"] * args.steps / launches
    out = {
        "metric": f"LLG cell-steps/s incl. FFT demag ({integrator.upper()})",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "disks": disk.n, "cells": Nc,
                   "D": sorted(set(disk.D)), "P": sorted(set(disk.P)), "launches": launches,
                   "path": "plain per-disk loop" if plain is not None else "batched persistent launch",
                   "workgroups": disk.launch_shape()[1], "threads_per_workgroup": disk.launch_shape()[2],
                   "radix_policy": disk.launch_shape()[3], "autotuned": tuned_us is not None,
                   "observables_every": args.sample_every, "observable_samples": len(samples),
                   "integrator_share_of_time": kernel_s / gpu_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "llg_persistent", "bytes_per_cell_step": b_step / Nc},
    }
    if not args.no_cpu and args.workload == "c2":
        out["cpu_baseline"] = cpu_baseline(Rs[0], Ls[0], prms[0].dtau, states[0], args.cpu_budget)
    print(json.dumps(out), flush=True)


def adjoint_bench(args):
    """Adjoint of a 5000-step RK4 trajectory on R=80 nm, L=10 nm (checkpoint every
    100 steps): time(backward incl. recompute) / time(forward)."""
    import numpy as np
    import torch

    import llg_inputs as li
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory
    R, L, a = 80.0, 10.0, 2.0
    disk = Disk.build(R, L, a)
    D = disk.D[0]
    n_seg, seg = 50, 100
    lam = 5.28906
    m0 = torch.tensor(li.vortex_ansatz(D, 10.0 / a, 0.01), dtype=torch.float32, device="cuda").reshape(-1)
    base = LLGParams(alpha=0.01, c=C_PY, dtau=0.04)
    k = torch.arange(n_seg + 1, dtype=torch.float64, device="cuda")
    target = torch.stack([10.0 * torch.exp(-0.01 * k) * torch.cos(0.2 * k),
                          10.0 * torch.exp(-0.01 * k) * torch.sin(0.2 * k)], 1)
    times = []
    for rep in range(2):
        m0g = m0.clone().requires_grad_(True)
        al = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        c = torch.tensor(C_PY, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = core_trajectory(m0g, al, c, disk, base, n_seg, seg, lam)
        loss = ((rc - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        disk.check()
        times.append((t1 - t0, t2 - t1))
        print(f"# rep {rep}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s, loss {float(loss):.4f}, "
              f"dL/dalpha {float(al.grad):.4e}, dL/dc {float(c.grad):.4e}", file=sys.stderr, flush=True)
    fwd, bwd = times[-1]
    Nc = disk.n_cells[0]
    steps = n_seg * seg
    out = {
        "metric": "adjoint/forward time ratio (RK4 trajectory, checkpointed)",
        "value": bwd / fwd, "unit": "ratio", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": fwd / steps * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "adjoint of 5000 RK4 steps, Permalloy R=80 nm L=10 nm a=2 nm (80x80, FFT 256), "
                               "checkpoint every 100 steps, loss on the core trajectory",
                   "forward_s": fwd, "backward_s": bwd, "forward_cell_steps_per_s": Nc * steps / fwd},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
