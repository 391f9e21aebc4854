"""The discrete adjoint on the cubed-sphere shell on the GPU (the transpose of the
curvilinear right-hand side of section 3.4, with the curved mortars of refined
shells; the adjoint itself is not in the paper): dg_rhs_adjoint and
dg_rk_stage_adjoint on uniform and refined shells against the oracle's
reverse-mode derivative of its own shell operator at N = 2..5, the dot-product
test against the oracle's forward-mode JVP, SSP-RK3 steps transposed against the
oracle, and the gradient of a forecast functional over 20 checkpointed SSP-RK3
steps on a shell refined once around a Gaussian theta vortex against central
differences; the transposed shell transfers of refine and coarsen passes against
the oracle's, and the gradient through two adaptation cycles of a shell (a
replayed sequence of passes) against the oracle and central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import adjoint as adj
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_direction, random_state
from tests.helpers import TOL_FP64, assert_fields, to_elem, to_nodes
from tests.test_gpu_parity import gpu

pytestmark = pytest.mark.gpu

PH = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
OPH = eu.Phys()


def _shell(N, n, nz, L=0, seed=0, fracs=()):
    lm = dg.dg_sphere_mesh_build(N, n, nz, max_level=L)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz, max_level=L))
    rng = np.random.default_rng(seed)
    for fr in fracs:
        fl = (rng.random(om.K) < fr).astype(np.int8)
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = sp.refine_pass(om, fl)
    assert np.array_equal(lm.tables()["leaf"], om.leaves.astype(np.int32))
    return lm, om


SHELLS = [
    dict(N=2, n=2, nz=2, L=0, seed=0, fracs=()),
    dict(N=3, n=2, nz=1, L=0, seed=0, fracs=()),
    dict(N=4, n=2, nz=1, L=0, seed=0, fracs=()),
    dict(N=5, n=1, nz=2, L=0, seed=0, fracs=()),
    dict(N=2, n=1, nz=2, L=2, seed=1, fracs=(0.4, 0.3)),
    dict(N=3, n=2, nz=1, L=2, seed=2, fracs=(0.4, 0.3)),
    dict(N=4, n=2, nz=1, L=1, seed=3, fracs=(0.4,)),
    dict(N=5, n=1, nz=1, L=1, seed=4, fracs=(0.4,)),
]


def _id(c):
    return f"N{c['N']}-L{c['L']}"


@pytest.mark.parametrize("case", SHELLS, ids=_id)
def test_shell_rhs_adjoint_against_oracle(case):
    N = case["N"]
    lm, om = _shell(**case)
    print(f"shell adjoint N={N} K={om.K} hanging={len(om.hang)}", flush=True)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 80 + N)) * 0.1 + to_nodes(sp.vortex_state(op, width=2.0e6))
    ln = torch.as_tensor(random_state(om.K, N, 90 + N))
    g = lm.field()
    dg.dg_rhs_adjoint(lm, PH, gpu(qn), gpu(ln), g)
    torch.cuda.synchronize()
    ref = eu.rhs_adjoint(op, to_elem(qn, N), to_elem(ln, N))
    assert_fields(g, to_nodes(ref), TOL_FP64, "shell rhs adjoint")


@pytest.mark.parametrize("case", [SHELLS[2], SHELLS[5]], ids=_id)
def test_shell_adjoint_dot_product_and_stage(case):
    """<lam, J v> (the oracle's forward-mode JVP) against <J^T lam, v> (the library),
    and the transposed stage a1 w1 + a2 w2 + b (y + dt J^T y) against the oracle"""
    N = case["N"]
    lm, om = _shell(**case)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 11)) * 0.1
    ln = torch.as_tensor(random_state(om.K, N, 12))
    vn = torch.as_tensor(random_state(om.K, N, 13))
    g = lm.field()
    dg.dg_rhs_adjoint(lm, PH, gpu(qn), gpu(ln), g)
    torch.cuda.synchronize()
    jv = to_nodes(eu.rhs_jvp(op, to_elem(qn, N), to_elem(vn, N)))
    lhs, rhs = float((ln * jv).sum()), float((g.cpu() * vn).sum())
    print("dot product", lhs, rhs, flush=True)
    assert abs(lhs - rhs) <= 1e-12 * (ln.abs() * jv.abs()).sum()
    w1, w2 = torch.as_tensor(random_state(om.K, N, 14)), torch.as_tensor(random_state(om.K, N, 15))
    out = lm.field()
    a1, a2, b, dt = 1.0 / 3.0, 0.75, 0.25, 3.0
    dg.dg_rk_stage_adjoint(lm, PH, a1, gpu(w1), a2, gpu(w2), b, dt, gpu(qn), gpu(ln), out)
    torch.cuda.synchronize()
    ref = a1 * w1 + a2 * w2 + b * (ln + dt * to_nodes(eu.rhs_adjoint(op, to_elem(qn, N), to_elem(ln, N))))
    assert_fields(out, ref, TOL_FP64, "shell stage adjoint")


def test_shell_reverse_steps_against_oracle():
    """three SSP-RK3 steps on a refined shell, reversed: the library's checkpointed
    gradient of <c, q_3> against the oracle's reverse steps"""
    N, dt, nsteps = 3, 2.0, 3
    lm, om = _shell(N=N, n=2, nz=1, L=1, seed=21, fracs=(0.3,))
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    q0n = to_nodes(sp.vortex_state(op, width=2.0e6)) + torch.as_tensor(random_state(om.K, N, 22)) * 0.01
    cn = torch.as_tensor(random_state(om.K, N, 23))
    x = gpu(q0n).requires_grad_(True)
    (g,) = torch.autograd.grad((gpu(cn) * adj.integrate(x, lm, PH, dt, nsteps, 2)).sum(), x)
    qs = [to_elem(q0n, N)]
    for _ in range(nsteps - 1):
        qs.append(eu.ssp_rk3_step(op, dt, qs[-1]))
    lam = to_elem(cn, N)
    for k in reversed(range(nsteps)):
        lam = eu.rk3_step_adjoint(op, dt, qs[k], lam)
    assert_fields(g, to_nodes(lam), TOL_FP64, "shell reverse steps")


def test_shell_vortex_gradient_20_steps():
    """A shell refined once around a Gaussian theta vortex (1 K; 2000 km wide on this
    coarse shell), N = 3, 20 SSP-RK3 steps of 2 s with checkpoints every 10, J the
    J W quadrature of theta'^2 over the cap within 3000 km of the vortex centre at
    the final time: dJ/dq0 from the checkpointed autograd.Function against central
    differences on 10 seeded directions (eps = 1e-4, relative gap <= 1e-7)."""
    N, dt, nsteps = 3, 2.0, 20
    lm = dg.dg_sphere_mesh_build(N, 3, 1, max_level=1)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=3, nz=1, max_level=1))
    op0 = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    q00 = sp.vortex_state(op0, width=2.0e6)
    eta = torch.empty(om.K, dtype=torch.float64, device="cuda")
    fl = dg.dg_indicator(lm, PH, gpu(to_nodes(q00)), dg.DG_IND_THETA, 0.3, eta=eta)
    fl = np.where(np.asarray(fl) > 0, 1, 0).astype(np.int8)
    assert fl.sum() > 0
    lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    om = sp.refine_pass(om, fl)
    assert np.array_equal(lm.tables()["leaf"], om.leaves.astype(np.int32)) and len(om.hang) > 0
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    print(f"vortex shell: K = {om.K}, hanging faces {len(om.hang)}", flush=True)
    qo = sp.vortex_state(op, width=2.0e6)
    cosang = op.geo.rhat[0]
    cap = (6.371e6 * torch.arccos(torch.clamp(cosang, -1.0, 1.0)) <= 3.0e6).double()
    wm = gpu(to_nodes((sp.quad_weights(op) * cap)[None])[0])
    rb = gpu(to_nodes(op.bg[0][None])[0])
    tb = gpu(to_nodes(op.bg[1][None])[0])

    def J(q):
        thp = (tb + q[4]) / (rb + q[0]) - tb / rb
        return (wm * thp * thp).sum()

    q0 = gpu(to_nodes(qo))
    x = q0.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(J(adj.integrate(x, lm, PH, dt, nsteps, 10)), x)

    def Jonly(y):
        with torch.no_grad():
            return float(J(adj.integrate(y, lm, PH, dt, nsteps, nsteps)))

    worst = 0.0
    for k in range(1, 11):
        d = gpu(torch.as_tensor(random_direction(om.K, N, 100 + k)))
        ad = float((g * d).sum())
        eps = 1e-4
        fd = (Jonly(q0 + eps * d) - Jonly(q0 - eps * d)) / (2 * eps)
        gap = abs(fd - ad) / max(abs(fd), abs(ad))
        worst = max(worst, gap)
        assert gap <= 1e-7, (k, fd, ad)
    print("vortex shell: worst FD relative gap over 10 directions at eps = 1e-4", worst, flush=True)


@pytest.mark.parametrize("N", [3, 4])
def test_shell_transfer_adjoint_against_oracle(N):
    """dg_sphere_adapt_project_adjoint for a refine pass (the scale factor's
    derivative included) and for the coarsen pass that undoes it, against the
    oracle's reverse-mode derivative of its own transfer"""
    lm, om = _shell(N=N, n=2, nz=1, L=2, seed=41, fracs=(0.3,))
    fl = (np.random.default_rng(42).random(om.K) < 0.3).astype(np.int8)
    lm2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    om2 = sp.refine_pass(om, fl)
    assert np.array_equal(lm2.tables()["leaf"], om2.leaves.astype(np.int32))
    o1, o2 = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL), sp.SphereOperator(om2, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 43)) * 0.1 + to_nodes(sp.acoustic_state(o1))
    q2 = lm2.field()
    s = dg.dg_sphere_adapt_project(lm, lm2, PH, gpu(qn), q2)
    gb = torch.as_tensor(random_state(om2.K, N, 44))
    g = lm.field()
    dg.dg_sphere_adapt_project_adjoint(lm, lm2, PH, gpu(qn), q2, s, gpu(gb), g)
    ref = to_nodes(sp.adapt_project_adjoint(o1, o2, to_elem(qn, N), to_elem(gb, N)))
    # rho' carries the scale factor's derivative (dot / M) (w_p - s sum_a I_a^T w_a),
    # a difference of two terms that agree to 1e-4..1e-5 (the children's weights
    # interpolate back to nearly the parent's), so both sides' rounding is relative
    # to those terms: its bound adds their magnitude |dot / M| |w_p|.  The other
    # fields are held to the plain bound.
    q2o, s_o = sp.adapt_project(o1, o2, to_elem(qn, N))
    ch = [e for e in range(om2.K) if 0 <= om2.xfer_kind[e] < 8]
    par = sorted({int(om2.xfer_src[e]) for e in ch})
    JW1, JW2 = sp.quad_weights(o1), sp.quad_weights(o2)
    q1e = to_elem(qn, N)
    M = float((JW1[par] * (o1.bg[0][par] + q1e[0][par])).sum())
    B2 = torch.stack([o2.bg[0], 0 * o2.bg[0], 0 * o2.bg[0], 0 * o2.bg[0], o2.bg[1]])
    dot = float((to_elem(gb, N)[:, ch] * (q2o[:, ch] + B2[:, ch])).sum())
    cancel = abs(dot / M) * float(torch.linalg.vector_norm(JW1[par]))
    err0 = float(torch.linalg.vector_norm(g[0].cpu() - ref[0]))
    print(f"refine pass transfer adjoint rho': {err0 / float(torch.linalg.vector_norm(ref[0])):.2e} of the field, "
          f"{err0 / (float(torch.linalg.vector_norm(ref[0])) + cancel):.2e} of field + cancelling terms", flush=True)
    assert err0 <= TOL_FP64 * (float(torch.linalg.vector_norm(ref[0])) + cancel)
    assert_fields(torch.cat([ref[:1], g[1:].cpu()]), ref, TOL_FP64, "refine pass transfer adjoint (U, Theta')")
    back = -np.ones(om2.K, dtype=np.int8)
    lm3 = dg.dg_mesh_build(prev=lm2, flags=back, pass_=dg.DG_PASS_COARSEN)
    om3 = sp.coarsen_pass(om2, back)
    o3 = sp.SphereOperator(om3, OPH, sp.BG_ISOTHERMAL)
    gb3 = torch.as_tensor(random_state(om3.K, N, 45))
    g2 = lm2.field()
    dg.dg_sphere_adapt_project_adjoint(lm2, lm3, PH, None, None, 1.0, gpu(gb3), g2)
    ref3 = sp.adapt_project_adjoint(o2, o3, to_elem(q2.cpu(), N), to_elem(gb3, N))
    assert_fields(g2, to_nodes(ref3), TOL_FP64, "coarsen pass transfer adjoint")


def test_shell_gradient_through_adaptation():
    """J(q_T) through 6 SSP-RK3 steps with two adaptation cycles on a shell (a
    replayed sequence of coarsen and refine passes): the library's gradient against
    the oracle's reverse-mode derivative of its own steps and transfers, and against
    central differences on seeded directions along the same sequence"""
    N, dt, nsteps, every = 3, 2.0, 6, 2
    lm, om = _shell(N=N, n=2, nz=1, L=1, seed=51, fracs=(0.4,))
    rng = np.random.default_rng(52)
    cycles, ocycles = [], []
    m, o = lm, om
    for _ in range(2):
        flc = np.where(o.leaves[:, 1] == 1, -1, 0).astype(np.int8)
        mc = dg.dg_mesh_build(prev=m, flags=flc, pass_=dg.DG_PASS_COARSEN)
        oc = sp.coarsen_pass(o, flc)
        assert mc.info.n_coarsened > 0
        flr = (rng.random(oc.K) < 0.4).astype(np.int8)
        mr = dg.dg_mesh_build(prev=mc, flags=flr, pass_=dg.DG_PASS_REFINE)
        orr = sp.refine_pass(oc, flr)
        assert mr.info.n_refined > 0 and np.array_equal(mr.tables()["leaf"], orr.leaves.astype(np.int32))
        cycles.append((mc, mr))
        ocycles.append((oc, orr))
        m, o = mr, orr
    plan = adj.AdaptPlan(cycles)
    opT = sp.SphereOperator(ocycles[-1][1], OPH, sp.BG_ISOTHERMAL)
    cap = (6.371e6 * torch.arccos(torch.clamp(opT.geo.rhat[0], -1.0, 1.0)) <= 4.0e6).double()
    wq = sp.quad_weights(opT) * cap
    rbo, tbo = opT.bg[0], opT.bg[1]
    wm, rb, tb = (gpu(to_nodes(x[None])[0]) for x in (wq, rbo, tbo))

    def J(q):
        thp = (tb + q[4]) / (rb + q[0]) - tb / rb
        return (wm * thp * thp).sum()

    op0 = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    q0o = sp.vortex_state(op0, width=2.0e6) + 0.01 * to_elem(torch.as_tensor(random_state(om.K, N, 53)), N)
    q0 = gpu(to_nodes(q0o))
    x = q0.clone().requires_grad_(True)
    qT, mT, _ = adj.integrate_adaptive(x, lm, PH, dt, nsteps, every, plan=plan, ckpt_every=2)
    assert mT is plan.cycles[-1][1]
    (g,) = torch.autograd.grad(J(qT), x)
    xo = q0o.clone().requires_grad_(True)
    qo, o, cyc = xo, om, 0
    for n in range(nsteps):
        qo = eu.ssp_rk3_step(sp.SphereOperator(o, OPH, sp.BG_ISOTHERMAL), dt, qo)
        if (n + 1) % every == 0 and n + 1 < nsteps:
            oc, orr = ocycles[cyc]
            o_from = sp.SphereOperator(o, OPH, sp.BG_ISOTHERMAL)
            o_c = sp.SphereOperator(oc, OPH, sp.BG_ISOTHERMAL)
            qo = sp.adapt_project(o_from, o_c, qo)[0]
            qo = sp.adapt_project(o_c, sp.SphereOperator(orr, OPH, sp.BG_ISOTHERMAL), qo)[0]
            o, cyc = orr, cyc + 1
    thp = (tbo + qo[4]) / (rbo + qo[0]) - tbo / rbo
    (go,) = torch.autograd.grad((wq * thp * thp).sum(), xo)
    assert_fields(g, to_nodes(go), TOL_FP64, "shell adaptive gradient vs oracle")

    def Jonly(y):
        with torch.no_grad():
            return float(J(adj.integrate_adaptive(y, lm, PH, dt, nsteps, every, plan=plan)[0]))

    for k in range(1, 4):
        d = gpu(torch.as_tensor(random_direction(om.K, N, 60 + k)))
        eps = 1e-4
        fd = (Jonly(q0 + eps * d) - Jonly(q0 - eps * d)) / (2 * eps)
        ad = float((g * d).sum())
        print("shell adaptive direction", k, "fd", fd, "adjoint", ad, flush=True)
        assert abs(fd - ad) <= 1e-7 * max(abs(fd), abs(ad)), (k, fd, ad)
