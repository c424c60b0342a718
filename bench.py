"""Benchmark: LLG cell-steps/s including the FFT demagnetisation field, one MI355X.

Default (headline) workload: 64 thermal replicas of a Permalloy disk R = 250 nm,
L = 20 nm on a = 2 nm cells (250 x 250 box, 49080 disk cells, FFT size 512),
Heun at T = 300 K, alpha = 0.1, dt = 0.02 ps, independent Philox streams, all
replicas in one batched persistent launch.  A step is one Heun step of every
replica (two field evaluations, each with the zero-padded FFT demag).

The same JSON line carries
* roofline: the persistent kernel's algorithmic bytes per launch over its
  average launch time (HIP events on the launch stream), against 8 TB/s;
* cpu_baseline: the float64 CPU oracle on one replica of the same disk for a
  bounded number of steps (scaled to the same cell-steps/s unit);
* batched_vs_plain: the 256-disk ragged ensemble (R in {30..120} nm, L/R in
  [0.05, 0.3], RK4) as one batched launch and as a loop over one handle per
  disk, both timed here over the same number of steps;
* adjoint_forward: the checkpointed adjoint of 5000 RK4 steps of the
  R = 80 nm, L = 10 nm disk (checkpoint every 100 steps, loss on the core
  trajectory against the oracle's target spiral): backward / forward time.
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
METRIC = "LLG cell-steps/s incl. FFT demag, batched vs plain; adjoint/forward time ratio"
KERNEL_SOURCES = ["paper_1207_2192_amd/csrc/llg_kernels.hpp", "paper_1207_2192_amd/csrc/fft_lds.hpp",
                  "paper_1207_2192_amd/csrc/llg_device.hpp", "paper_1207_2192_amd/csrc/kernels_rk4.hip",
                  "paper_1207_2192_amd/csrc/kernels_heun.hip", "paper_1207_2192_amd/csrc/kernels_rk4_series.hip",
                  "paper_1207_2192_amd/csrc/kernels_heun_series.hip"]
SEED = 20120827


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
    """Measured HBM bytes per step from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- workloads
def workload(name):
    """(R list, L list, start offsets nm, params list, integrator, description)."""
    import llg_inputs as li
    from paper_1207_2192_amd import LLGParams, params_from_si
    a = 2.0
    PY = li.PERMALLOY
    if name == "c2":
        return ([100.0], [20.0], [(10.0, 0.0)], [LLGParams(alpha=0.0, c=C_PY, dtau=0.04)], "rk4",
                "RK4 T=0 gyrotropic disk: Permalloy R=100 nm L=20 nm a=2 nm, 100x100 box (7860 cells), "
                "FFT 256x256, alpha=0, dtau=0.04, vortex displaced to X=(10 nm,0)")
    if name == "c3":
        ens = li.ragged_ensemble(256)
        return ([e.R_nm for e in ens], [e.L_nm for e in ens], [(e.x0_nm, e.y0_nm) for e in ens],
                [LLGParams(alpha=0.02, c=C_PY, dtau=0.04) for _ in ens], "rk4",
                "ragged ensemble of 256 Permalloy disks, R in {30..120} nm, L/R in [0.05,0.3], a=2 nm, "
                "RK4 T=0 alpha=0.02 dtau=0.04, vortex offsets 2-15 nm")
    nrep = 64
    p0, _ = params_from_si(PY["A"], PY["Ms"], PY["gamma"], a, 20.0, 0.02, 300.0, 0.1)
    p0.renorm = True
    return ([250.0] * nrep, [20.0] * nrep, [(0.0, 0.0)] * nrep, [p0] * nrep, "heun",
            "64 thermal replicas of a Permalloy disk R=250 nm L=20 nm a=2 nm (250x250 box, 49080 cells, "
            "FFT 512x512), Heun T=300 K alpha=0.1 dt=0.02 ps (dtau=0.0266), renormalised, "
            "independent Philox streams per replica and cell, vortex starting centred")


def start_states(D_list, starts, a=2.0):
    import numpy as np
    import llg_inputs as li
    # centred starts are nudged off the exact grid symmetry point
    return [li.vortex_ansatz(D, x0 / a + 0.01, y0 / a + 0.013) for D, (x0, y0) in zip(D_list, starts)]


def step_call(disk, m, k, prms, integrator, step0, replica0=0, series_every=0):
    """k integrator steps; with series_every > 0 the launch also records the float64
    <m> and energy of the state at the start of every series_every-th step."""
    if series_every:
        if integrator == "rk4":
            return disk.rk4_series(m, k, prms, series_every)
        return disk.heun_series(m, k, prms, series_every, seed=SEED, step0=step0, replica=replica0)
    if integrator == "rk4":
        disk.rk4_step(m, k, prms)
    else:
        disk.heun_step(m, k, prms, seed=SEED, step0=step0, replica=replica0)
    return None


# ---------------------------------------------------------------- CPU oracle
def cpu_baseline(R, L, prm, integrator, m0_np, budget_s):
    """The float64 oracle on the host cores for about budget_s: steps of one disk
    (one replica for the thermal ensemble), in cell-steps/s."""
    import torch
    import oracle
    from oracle.dynamics import heun_step, rk4_step
    d = oracle.Disk(R, L, 2.0)
    op = oracle.Params(alpha=prm.alpha, c=prm.c, dtau=prm.dtau, temp=prm.temp, renorm=prm.renorm)
    m = torch.tensor(m0_np)

    def run(x, n, s0):
        if integrator == "rk4":
            return rk4_step(x, d, op, n)
        return heun_step(x, d, op, seed=SEED, step0=s0, replica=0, nsteps=n)

    m = run(m, 1, 0)                          # warm the FFT plans and the kernel spectra
    t = time.perf_counter()
    m = run(m, 2, 1)
    per = (time.perf_counter() - t) / 2
    n = max(2, int(budget_s / per))
    t = time.perf_counter()
    run(m, n, 3)
    dt = time.perf_counter() - t
    what = "RK4 steps of the same disk" if integrator == "rk4" else "Heun steps of one replica of the same disk"
    return dict(value=d.n_cells * n / dt, unit="cell-steps/s", cores=torch.get_num_threads(),
                host_cores=os.cpu_count(), kind="oracle",
                sample=f"{n} {what} (float64 torch CPU FFT path, {torch.get_num_threads()} threads), {dt:.1f} s; "
                       f"cell-steps/s of that sample")


# ---------------------------------------------------------------- batched vs plain (ragged ensemble)
def batched_vs_plain(steps, warmup):
    import numpy as np
    import torch
    from paper_1207_2192_amd import Disk
    Rs, Ls, starts, prms, integrator, desc = workload("c3")
    batch = Disk.batch(Rs, Ls, 2.0)
    states = start_states(batch.D, starts)
    m0 = torch.tensor(np.concatenate([s.reshape(-1) for s in states]), dtype=torch.float32, device="cuda")
    m = m0.clone()
    tuned = batch.autotune(m, prms, integrator, probe_steps=40)
    plain = [Disk.build(Rs[k], Ls[k], 2.0) for k in range(batch.n)]
    stream = torch.cuda.current_stream()
    Nc = sum(batch.n_cells)

    def timed(fn):
        fn(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    def run_batch(k):
        if k:
            batch.rk4_step(m, k, prms)

    mp = m0.clone()

    def run_plain(k):
        if not k:
            return
        for j, dj in enumerate(plain):
            dj.rk4_step(mp[batch.offsets[j]:batch.offsets[j] + 3 * batch.D[j] ** 2], k, prms[j])

    # untimed spin-up on a scratch copy after the host-side set-up of the plain handles
    scratch = m0.clone()
    batch.rk4_step(scratch, max(1, int(30e3 / max(tuned, 1.0))), prms)
    del scratch
    tb = timed(run_batch)
    tp = timed(run_plain)
    batch.check()
    for dj in plain:
        dj.check()
    # the two paths take the same steps: their states agree to float rounding
    diff = float((m - mp).abs().max())
    out = {"workload": desc, "disks": batch.n, "cells": Nc, "steps": steps,
           "batched_cell_steps_per_s": Nc * steps / tb, "plain_cell_steps_per_s": Nc * steps / tp,
           "ratio": tp / tb, "batched_us_per_step": tb / steps * 1e6, "plain_us_per_step": tp / steps * 1e6,
           "batched_plan": list(batch.launch_shape()), "autotuned_us_per_step": tuned,
           "max_state_difference": diff}
    for dj in plain:
        dj.close()
    batch.close()
    return out


# ---------------------------------------------------------------- adjoint / forward
def adjoint_forward(reps=2):
    """Checkpointed adjoint of 5000 RK4 steps of the R = 80 nm, L = 10 nm disk
    against the oracle's target spiral (tests/golden/c4_adjoint.json)."""
    import torch
    import llg_inputs as li
    from paper_1207_2192_amd import Disk, LLGParams
    from paper_1207_2192_amd.adjoint import core_trajectory, grad_exchange_length
    with open(os.path.join(ROOT, "tests", "golden", "c4_adjoint.json")) as f:
        g = json.load(f)
    a = 2.0
    disk = Disk.build(80.0, 10.0, a)
    D = disk.D[0]
    lam, c0, al0 = g["lambda_ex_nm"], g["c"], g["alpha"]
    n_seg, seg = g["n_seg"], g["seg_steps"]
    m0 = torch.tensor(li.vortex_ansatz(D, 10.0 / a, 0.01, core_width=5.0 / a), dtype=torch.float32,
                      device="cuda").reshape(-1).contiguous()
    base = LLGParams(alpha=al0, c=c0, dtau=g["dtau"])
    target = torch.tensor(g["target"], dtype=torch.float64, device="cuda")
    times = []
    for rep in range(reps):
        m0g = m0.clone().requires_grad_(True)
        al = torch.tensor(al0, dtype=torch.float64, requires_grad=True)
        c = torch.tensor(c0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = core_trajectory(m0g, al, c, disk, base, n_seg, seg, g["cutoff_lambda_ex_nm"])
        loss = ((rc - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        disk.check()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    dl = float(grad_exchange_length(c.grad, c0, lam))
    out = {"workload": "adjoint of 5000 RK4 steps, Permalloy R=80 nm L=10 nm a=2 nm (80x80, FFT 256), "
                       "checkpoint every 100 steps, loss = sum |r_c - target|^2 over 51 checkpoints, target "
                       "spiral from the float64 oracle at alpha=0.015 and lambda_ex x 1.05",
           "forward_s": fwd, "backward_s": bwd, "ratio": bwd / fwd,
           "forward_cell_steps_per_s": disk.n_cells[0] * n_seg * seg / fwd,
           "loss": float(loss), "loss_oracle": g["loss"],
           "dL_dalpha": float(al.grad), "dL_dalpha_oracle_fd": g["dL_dalpha_fd"],
           "dL_dlambda_ex": dl, "dL_dlambda_ex_oracle_fd": g["dL_dlambda_fd"]}
    disk.close()
    return out


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=5000, help="steps per launch")
    ap.add_argument("--workload", default="c5", choices=["c2", "c3", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched-vs-plain and adjoint legs")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--wg", type=int, default=0, help="workgroups per disk (0 = library choice)")
    ap.add_argument("--ug", type=int, default=0, help="wavefront groups per workgroup (0 = library choice)")
    ap.add_argument("--radix", type=int, default=0, help="transform policy for --ug/--wg (0..3)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch plan")
    ap.add_argument("--plain", action="store_true", help="loop over single-disk handles instead of one batch")
    ap.add_argument("--sample-every", type=int, default=100,
                    help="steps between observable samples (core position + energy) in the timed region; 0 = none")
    ap.add_argument("--series-energy", action="store_true",
                    help="sample the energy from the integrator's own float64 series instead of llg_energy "
                         "(an extra field evaluation)")
    ap.add_argument("--spinup-ms", type=float, default=30.0,
                    help="untimed integrator work on a scratch copy of the state right before the warmup "
                         "(brings the GPU clocks up after the host-side set-up)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent disks shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1207_2192_amd import Disk, LLGParams

    torch.cuda.set_device(0)
    a = 2.0
    Rs, Ls, starts, prms, integrator, desc = workload(args.workload)
    disk = Disk.batch(Rs, Ls, a) if len(Rs) > 1 else Disk.build(Rs[0], Ls[0], a)
    if args.wg or args.ug:
        disk.tune(args.ug or disk.launch_shape()[0], [args.wg] * disk.n if args.wg else None, args.radix)
    Nc = sum(disk.n_cells)
    states = start_states(disk.D, starts, a)
    m = torch.tensor(np.concatenate([s.reshape(-1) for s in states]), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    tuned_us = None
    if not (args.wg or args.ug or args.no_autotune):
        tuned_us = disk.autotune(m, prms, integrator, probe_steps=300 if disk.n == 1 else 40)
        log(f"autotune: {tuned_us:.2f} us/step with plan {disk.launch_shape()}")
    step_counter = [0]
    last_k = [0]               # steps of the last timed launch

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
            # in the timed region the energy and <m> of every launch's start state come
            # from the integrator's own series (unless --separate-energy)
            ser_every = k if (timed and args.sample_every and args.series_energy) else 0
            if plain is not None:
                for j, dj in enumerate(plain):
                    mj = m[disk.offsets[j]:disk.offsets[j] + 3 * disk.D[j] ** 2]
                    step_call(dj, mj, k, prms[j], integrator, step_counter[0], j)
                    launches += 1
            else:
                ser = step_call(disk, m, k, prms, integrator, step_counter[0], series_every=ser_every)
                launches += 1
                last_k[0] = k
            if timed:
                ev[1].record(stream)
                kernel_events.append(ev)
                if args.sample_every:
                    if plain is not None:
                        for j, dj in enumerate(plain):
                            mj = m[disk.offsets[j]:disk.offsets[j] + 3 * disk.D[j] ** 2]
                            samples.append((dj.vortex_core_position(mj, lam_nm), dj.energy(mj, eprm[j:j + 1])))
                    elif args.series_energy:
                        samples.append((disk.vortex_core_position(m, lam_nm), ser))
                    else:
                        samples.append((disk.vortex_core_position(m, lam_nm), disk.energy(m, eprm)))
            step_counter[0] += k
            left -= k
        return launches

    e0 = disk.energy(m, eprm)[:, 0].cpu()
    # untimed spin-up on a scratch copy (the state itself is untouched), then the warmup steps
    spin = 0
    if args.spinup_ms > 0 and plain is None:
        per_us = tuned_us if tuned_us else 300.0
        spin = max(1, int(math.ceil(args.spinup_ms * 1e3 / per_us)))
        scratch = m.clone()
        step_call(disk, scratch, spin, prms, integrator, 10 ** 9)
        del scratch
    if args.warmup:
        run(args.warmup)
    torch.cuda.synchronize()
    disk.check()
    log(f"warmup {args.warmup} steps done")

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if plain is None:
        disk.timing(True)   # the library's events right around each cooperative launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    launches = run(args.steps, timed=True)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    disk.check()
    gpu_s = start.elapsed_time(stop) / 1e3
    lib_ms = disk.last_launch_ms(integrator) if plain is None else None
    e1 = disk.energy(m, eprm)[:, 0].cpu()
    drift = float(((e1 - e0).abs() / e0.abs()).max())
    log(f"timed {args.steps} steps in {gpu_s:.4f} s (wall {wall:.4f} s), max relative energy change {drift:.2e}")

    if args.copy_probe_mib:
        x = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    stages = 4 if integrator == "rk4" else 2
    value = Nc * args.steps / gpu_s
    b_step = sum(bytes_per_stage(disk.D[k], disk.P[k]) for k in range(disk.n)) * stages
    b_launch = b_step * args.steps / launches
    # duration of the integrator launches alone (the observables between them excluded):
    # stream events around each launch call (they also bracket the barrier reset) ...
    kernel_s = sum(x0.elapsed_time(x1) for x0, x1 in kernel_events) / 1e3
    t_launch = kernel_s / launches
    # ... and the library's events right around the cooperative kernel of the last
    # timed launch, the duration a kernel trace reports; achieved uses the latter
    if lib_ms is not None:
        t_kernel = lib_ms / 1e3
        achieved = b_step * last_k[0] / t_kernel / 1e9
    else:
        t_kernel = t_launch
        achieved = b_launch / t_launch / 1e9
    tr = traffic_record(f"{args.workload}_{integrator}")
    traffic = None if tr is None else tr["bytes_per_step"] * args.steps / launches
    shape = disk.launch_shape()
    out = {
        "metric": METRIC,
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
        "config": {"workload": desc, "integrator": integrator, "disks": disk.n, "cells": Nc,
                   "D": sorted(set(disk.D)), "P": sorted(set(disk.P)), "launches": launches,
                   "path": "plain per-disk loop" if plain is not None else "batched persistent launch",
                   "workgroups": shape[1], "threads_per_workgroup": shape[2],
                   "radix_policy": shape[3], "autotuned": tuned_us is not None,
                   "observables_every": args.sample_every, "observable_samples": len(samples),
                   "energy_from": "integrator float64 series" if args.series_energy else "llg_energy",
                   "spinup_steps_on_scratch_copy": spin,
                   "integrator_share_of_time": kernel_s / gpu_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "llg_persistent", "kernel_us_per_launch": t_kernel * 1e6,
                     "steps_per_launch": last_k[0] if lib_ms is not None else args.steps / launches,
                     "launch_us_stream_events": t_launch * 1e6,
                     "bytes_per_launch": b_launch, "bytes_per_cell_step": b_step / Nc},
    }
    if plain is not None:
        for dj in plain:
            dj.close()
    disk.close()
    if not args.no_extras and args.workload == "c5":
        t = time.perf_counter()
        out["batched_vs_plain"] = batched_vs_plain(args.steps, args.warmup)
        log(f"batched vs plain leg: ratio {out['batched_vs_plain']['ratio']:.1f} "
            f"({time.perf_counter() - t:.1f} s)")
        t = time.perf_counter()
        out["adjoint_forward"] = adjoint_forward()
        log(f"adjoint leg: ratio {out['adjoint_forward']['ratio']:.2f} ({time.perf_counter() - t:.1f} s)")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(Rs[0], Ls[0], prms[0], integrator, states[0], args.cpu_budget)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
