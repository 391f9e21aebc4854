"""Discrete adjoint of the SSP-RK3 integration behind torch.autograd.Functions.

Forward: n SSP-RK3 steps with dg_rk_stage, keeping the state every
``ckpt_every`` steps.  Backward: for each segment in reverse, recompute its
steps once from the checkpoint (keeping the three stage inputs of every step)
and run the transposed stages with dg_rk_stage_adjoint.  Through an adaptation
cycle the gradient flows back through the transposes of the conservative
transfers (section 3.3; on a shell, of section 3.4's transfer) along the
recorded mesh sequence.  All arithmetic runs in the HIP library; this module
only orders calls and holds buffers.
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


class Transfer(torch.autograd.Function):
    """q_to = P q_from for the refine or coarsen transfer src -> dst (a linear
    map); the backward applies P^T with the library's transposed transfer."""

    @staticmethod
    def forward(ctx, q, src, dst, refine):
        out = torch.empty(5, dst.K, dst.Np, dtype=torch.float64, device=q.device)
        (dg.dg_refine_project if refine else dg.dg_coarsen_project)(src, dst, q.detach().contiguous(), out)
        ctx.src, ctx.dst, ctx.refine = src, dst, refine
        return out

    @staticmethod
    def backward(ctx, g):
        src, dst = ctx.src, ctx.dst
        out = torch.empty(5, src.K, src.Np, dtype=torch.float64, device=g.device)
        adj = dg.dg_refine_project_adjoint if ctx.refine else dg.dg_coarsen_project_adjoint
        adj(src, dst, g.detach().contiguous(), out)
        return out, None, None, None


class ShellTransfer(torch.autograd.Function):
    """q_to = T(q_from) for the transfer of a shell's refine or coarsen pass
    (dg_sphere_adapt_project: affine for a coarsening, nonlinear through the
    refinement's scale factor); the backward applies the transpose of its
    derivative at q_from with dg_sphere_adapt_project_adjoint."""

    @staticmethod
    def forward(ctx, q, src, dst, phys):
        qd = q.detach().contiguous()
        out = torch.empty(5, dst.K, dst.Np, dtype=torch.float64, device=q.device)
        s = dg.dg_sphere_adapt_project(src, dst, phys, qd, out)
        ctx.save_for_backward(qd, out)
        ctx.src, ctx.dst, ctx.phys, ctx.s = src, dst, phys, s
        return out

    @staticmethod
    def backward(ctx, g):
        qd, out = ctx.saved_tensors
        gin = torch.empty(5, ctx.src.K, ctx.src.Np, dtype=torch.float64, device=g.device)
        dg.dg_sphere_adapt_project_adjoint(ctx.src, ctx.dst, ctx.phys, qd, out, ctx.s, g.detach().contiguous(), gin)
        return gin, None, None, None


class AdaptPlan:
    """Mesh sequence of an adaptive run: (mesh_c, mesh_r) of every cycle, as
    :func:`dg.adapt_meshes` returns them.  The flags are piecewise constant in
    the state, so derivatives are taken along a fixed sequence: a plan recorded
    by one run is replayed by the next (gradient, finite differences)."""

    def __init__(self, cycles=None):
        self.cycles = list(cycles or [])


def integrate_adaptive(q0, mesh, phys, dt, nsteps, adapt_every, kind=None, thr=None, plan=None,
                       ckpt_every=10):
    """Differentiable SSP-RK3 integration with an adaptation cycle after every
    ``adapt_every`` steps (none after the last step).  Without a plan, each cycle
    comes from the indicator (kind, thr) of the current state and is recorded;
    with a plan, its meshes are replayed.  Returns (q_T, mesh_T, plan)."""
    record = plan is None
    plan = AdaptPlan() if record else plan
    q, m, n, cyc = q0, mesh, 0, 0
    while n < nsteps:
        seg = min(adapt_every, nsteps - n)
        q = integrate(q, m, phys, dt, seg, min(ckpt_every, seg))
        n += seg
        if n >= nsteps:
            break
        if record:
            mc, mr = dg.adapt_meshes(m, phys, q.detach(), kind, thr)
            plan.cycles.append((mc, mr))
        else:
            mc, mr = plan.cycles[cyc]
        if mc is not m:
            q = ShellTransfer.apply(q, m, mc, phys) if m.shell else Transfer.apply(q, m, mc, False)
        if mr is not mc:
            q = ShellTransfer.apply(q, mc, mr, phys) if mc.shell else Transfer.apply(q, mc, mr, True)
        m, cyc = mr, cyc + 1
    return q, m, plan
