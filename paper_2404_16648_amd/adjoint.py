"""Discrete adjoint of the SSP-RK3 integration behind a torch.autograd.Function.

Forward: n SSP-RK3 steps with dg_rk_stage, keeping the state every
``ckpt_every`` steps.  Backward: for each segment in reverse, recompute its
steps once from the checkpoint (keeping the three stage inputs of every step)
and run the transposed stages with dg_rk_stage_adjoint.  All arithmetic runs in
the HIP library; this module only orders calls and holds buffers.
"""
from __future__ import annotations

import torch

from . import dg


def rk3_step_adjoint(mesh, phys, dt, q0, q1, q2, lam3, stream=None):
    """dJ/dq_n from dJ/dq_{n+1} = lam3 and the stage inputs q0 = q_n, q1, q2.

    lam2 = 2/3 (lam3 + dt A(q2)^T lam3), lam1 = 1/4 (lam2 + dt A(q1)^T lam2),
    dJ/dq_n = 1/3 lam3 + 3/4 lam2 + lam1 + dt A(q0)^T lam1."""
    lam2 = torch.empty_like(lam3)
    lam1 = torch.empty_like(lam3)
    out = torch.empty_like(lam3)
    dg.dg_rk_stage_adjoint(mesh, phys, 0.0, None, 0.0, None, 2.0 / 3.0, dt, q2, lam3, lam2, stream)
    dg.dg_rk_stage_adjoint(mesh, phys, 0.0, None, 0.0, None, 0.25, dt, q1, lam2, lam1, stream)
    dg.dg_rk_stage_adjoint(mesh, phys, 1.0 / 3.0, lam3, 0.75, lam2, 1.0, dt, q0, lam1, out, stream)
    return out


def _step_keep_stages(mesh, phys, dt, q):
    """One SSP-RK3 step from q; returns (q_next, (q0, q1, q2))."""
    q1 = torch.empty_like(q)
    q2 = torch.empty_like(q)
    qn = torch.empty_like(q)
    dg.dg_rk_stage(mesh, phys, 0.0, 1.0, dt, q, q, q1)
    dg.dg_rk_stage(mesh, phys, 0.75, 0.25, dt, q, q1, q2)
    dg.dg_rk_stage(mesh, phys, 1.0 / 3.0, 2.0 / 3.0, dt, q, q2, qn)
    return qn, (q, q1, q2)


class SSPRK3Integrate(torch.autograd.Function):
    """q_T = Phi_dt^n(q_0) with a hand-written discrete adjoint and checkpointed
    recomputation; use via :func:`integrate`."""

    @staticmethod
    def forward(ctx, q0, mesh, phys, dt, nsteps, ckpt_every):
        q = q0.detach().contiguous()
        ckpts = {0: q.clone()}
        for n in range(nsteps):
            q, _ = _step_keep_stages(mesh, phys, dt, q)
            if (n + 1) % ckpt_every == 0 and n + 1 < nsteps:
                ckpts[n + 1] = q.clone()
        ctx.mesh, ctx.phys, ctx.dt, ctx.nsteps, ctx.ckpt_every = mesh, phys, dt, nsteps, ckpt_every
        ctx.ckpts = ckpts
        return q

    @staticmethod
    def backward(ctx, grad_qT):
        mesh, phys, dt = ctx.mesh, ctx.phys, ctx.dt
        lam = grad_qT.detach().contiguous().clone()
        for start in sorted(ctx.ckpts, reverse=True):
            end = min(start + ctx.ckpt_every, ctx.nsteps)
            q = ctx.ckpts[start]
            stages = []
            for _ in range(start, end):
                q, st = _step_keep_stages(mesh, phys, dt, q)
                stages.append(st)
            for q0, q1, q2 in reversed(stages):
                lam = rk3_step_adjoint(mesh, phys, dt, q0, q1, q2, lam)
        ctx.ckpts = None
        return lam, None, None, None, None, None


def integrate(q0, mesh, phys, dt, nsteps, ckpt_every=10):
    """Differentiable n-step SSP-RK3 integration on a fixed mesh."""
    return SSPRK3Integrate.apply(q0, mesh, phys, dt, nsteps, ckpt_every)
