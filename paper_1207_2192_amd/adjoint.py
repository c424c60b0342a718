"""Hand-written adjoint of RK4 and Heun trajectories as a torch.autograd.Function.

`CoreTrajectory.apply(m0, alpha, c, disk, params, n_seg, seg_steps, lambda_ex_nm, noise)`
integrates n_seg * seg_steps RK4 steps (noise = None) or Heun steps (noise =
(seed, step0, replica); segment s uses the step indices step0 + s*seg_steps ...)
on the GPU and returns the vortex core position r_c (nm, float64) at the
n_seg + 1 checkpoints t = 0, seg_steps, ...  Checkpoints of the state are kept
every seg_steps steps.  The backward pass recomputes each segment once with the
stage record (llg_rk4_record / llg_heun_record) and runs the reverse sweep
(llg_rk4_vjp / llg_heun_vjp, the noise replayed from its counter); the
cotangent of each sampled core position enters through llg_core_position_vjp.
Gradients come out for m0, alpha and c = a^2/lambda_ex^2;
`grad_exchange_length` converts d/dc into d/d lambda_ex.  All arithmetic runs
in lib_llgdisk; torch provides buffers and the stream.
"""
from __future__ import annotations

from dataclasses import replace

import torch

from .api import Disk, LLGParams


class CoreTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, alpha, c, disk: Disk, params: LLGParams, n_seg: int, seg_steps: int,
                lambda_ex_nm: float, noise=None):
        if disk.n != 1:
            raise ValueError("CoreTrajectory steps one disk")
        if noise is None and params.renorm:
            raise ValueError("the RK4 adjoint covers RK4 without renormalisation")
        prm = replace(params, alpha=float(alpha), c=float(c))
        m = m0.detach().clone().contiguous()
        ckpts = [m.clone()]
        cores = [disk.vortex_core_position(m, lambda_ex_nm)]
        for s in range(n_seg):
            if noise is None:
                disk.rk4_step(m, seg_steps, prm)
            else:
                seed, step0, rep = noise
                disk.heun_step(m, seg_steps, prm, seed=seed, step0=step0 + s * seg_steps, replica=rep)
            ckpts.append(m.clone())
            cores.append(disk.vortex_core_position(m, lambda_ex_nm))
        ctx.noise = noise
        ctx.disk, ctx.prm, ctx.n_seg, ctx.seg = disk, prm, n_seg, seg_steps
        ctx.lam, ctx.ckpts, ctx.cores = lambda_ex_nm, ckpts, cores
        ctx.alpha_like, ctx.c_like = alpha, c
        return torch.stack([cr[0, :2] for cr in cores])

    @staticmethod
    def backward(ctx, grad_rc):
        disk, prm, seg = ctx.disk, ctx.prm, ctx.seg
        grad_rc = grad_rc.to(torch.float64).contiguous()
        ybar = torch.zeros_like(ctx.ckpts[0])
        pgrad = torch.zeros(2, dtype=torch.float64, device=ybar.device)
        per_step = 8 if ctx.noise is None else 4
        rec = torch.empty(per_step * seg * disk.state_size, dtype=torch.float32, device=ybar.device)
        disk.core_position_vjp(ctx.ckpts[-1], ctx.lam, ctx.cores[-1], grad_rc[-1], ybar)
        for s in reversed(range(ctx.n_seg)):
            m = ctx.ckpts[s].clone()
            if ctx.noise is None:
                disk.rk4_record(m, seg, prm, rec)
                disk.rk4_vjp(rec, seg, ybar, pgrad, prm)
            else:
                seed, step0, rep = ctx.noise
                kw = dict(seed=seed, step0=step0 + s * seg, replica=rep)
                disk.heun_record(m, seg, prm, rec, **kw)
                disk.heun_vjp(rec, seg, ybar, pgrad, prm, **kw)
            disk.core_position_vjp(ctx.ckpts[s], ctx.lam, ctx.cores[s], grad_rc[s], ybar)
        ga = pgrad[0].to(dtype=torch.as_tensor(ctx.alpha_like).dtype)
        gc = pgrad[1].to(dtype=torch.as_tensor(ctx.c_like).dtype)
        if isinstance(ctx.alpha_like, torch.Tensor):
            ga = ga.to(ctx.alpha_like.device)
        if isinstance(ctx.c_like, torch.Tensor):
            gc = gc.to(ctx.c_like.device)
        return ybar, ga, gc, None, None, None, None, None, None


def core_trajectory(m0, alpha, c, disk, params, n_seg, seg_steps, lambda_ex_nm, noise=None):
    """noise = None: RK4; noise = (seed, step0, replica): Heun with that Philox stream."""
    return CoreTrajectory.apply(m0, alpha, c, disk, params, n_seg, seg_steps, lambda_ex_nm, noise)


def grad_exchange_length(grad_c, c, lambda_ex_nm):
    """d/d lambda_ex from d/dc with c = (a/lambda_ex)^2: dc/dlambda = -2c/lambda."""
    return grad_c * (-2.0 * c / lambda_ex_nm)
