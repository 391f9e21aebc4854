"""GPU parity of the discrete adjoint: dg_rhs_adjoint and dg_rk_stage_adjoint
against the oracle's reverse-mode derivative of its own RHS, the dot-product
test against the oracle's forward-mode JVP, the checkpointed autograd.Function
gradient against central finite differences, the transposed transfers against
the oracle's, and the gradient through adaptation cycles (replayed mesh
sequence) against the oracle and central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from paper_2404_16648_amd import adjoint as adj
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_direction, random_state
from tests.helpers import (TOL_FP64, assert_fields, oracle_desc, oracle_phys, phys_for, random_refinements,
                           tables_equal, to_elem, to_nodes)

pytestmark = pytest.mark.gpu

DEV = "cuda"
BOX = ((0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))


def both_meshes(N, nroot, L, periodic=(0, 0, 0), flag_seq=()):
    lm = dg.dg_mesh_build(N, nroot, L, *BOX, periodic)
    od = oracle_desc(N, nroot, L, *BOX, periodic)
    om = fo.build(od, None)
    for fl in flag_seq:
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = fo.build(od, om, fl, fo.PASS_REFINE)
    assert tables_equal(lm.tables(), om)
    return lm, om


def gpu(t):
    return t.to(DEV).contiguous()


def check(a_gpu, b_oracle, tol=TOL_FP64, what=""):
    """Every component within tol in relative L2 (the adjoint weights are random:
    no component vanishes)."""
    assert_fields(a_gpu, to_nodes(b_oracle), tol, what)


CASES = [
    dict(N=2, nroot=(2, 2, 2), periodic=(0, 0, 0), seed=31),
    dict(N=3, nroot=(2, 3, 2), periodic=(1, 0, 1), seed=32),
    dict(N=4, nroot=(2, 2, 2), periodic=(1, 1, 1), seed=33),
    dict(N=5, nroot=(2, 1, 2), periodic=(0, 1, 0), seed=34),
    dict(N=6, nroot=(1, 2, 2), periodic=(0, 0, 1), seed=39),
    dict(N=7, nroot=(2, 2, 2), periodic=(0, 0, 0), seed=35),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c['N']}")
def test_rhs_adjoint_random_amr(case):
    N = case["N"]
    od = oracle_desc(N, case["nroot"], 2, *BOX, case["periodic"])
    lm, om = both_meshes(N, case["nroot"], 2, case["periodic"], random_refinements(od, 2, case["seed"]))
    ph = phys_for(case["periodic"])
    op = eu.Operator(om, oracle_phys(ph))
    qn = torch.as_tensor(random_state(om.K, N, case["seed"]))
    ln = torch.as_tensor(random_state(om.K, N, case["seed"] + 100, (1.0, 1.0, 1.0, 1.0, 1.0)))
    out = lm.field()
    dg.dg_rhs_adjoint(lm, ph, gpu(qn), gpu(ln), out)
    torch.cuda.synchronize()
    want = eu.rhs_adjoint(op, to_elem(qn, N), to_elem(ln, N))
    check(out, want, what=f"adjoint N={N}")
    # dot-product test against the oracle's forward-mode derivative
    v = torch.as_tensor(random_direction(om.K, N, case["seed"] + 200))
    jv = eu.rhs_jvp(op, to_elem(qn, N), to_elem(v, N))
    a = float((to_elem(ln, N) * jv).sum())
    b = float((out.cpu() * v).sum())
    assert abs(a - b) <= 1e-11 * max(abs(a), abs(b)), (a, b)


def test_rhs_adjoint_zero_wind_bubble():
    """The bubble state has u = 0 everywhere and equal wave speeds on both sides
    of every face: the non-smooth points of |u.n| and of the max."""
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(4, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 36))
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q = eu.bubble_state(op)
    ln = torch.as_tensor(random_state(om.K, 4, 37, (1.0, 1.0, 1.0, 1.0, 1.0)))
    out = lm.field()
    dg.dg_rhs_adjoint(lm, ph, gpu(to_nodes(q)), gpu(ln), out)
    check(out, eu.rhs_adjoint(op, q, to_elem(ln, 4)), what="adjoint at rest")


@pytest.mark.parametrize("N", [3, 6, 7])
def test_rk_stage_adjoint_combination(N):
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    seed = {3: 41, 6: 44, 7: 46}[N]  # refinements that leave hanging faces
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, seed))
    assert lm.info.n_hang > 0
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q, y, w1, w2 = (torch.as_tensor(random_state(om.K, N, s + N)) for s in (40, 41, 42, 43))
    dt = 0.01
    out = lm.field()
    dg.dg_rk_stage_adjoint(lm, ph, 1 / 3, gpu(w1), 0.75, gpu(w2), 0.5, dt, gpu(q), gpu(y), out)
    E = lambda t: to_elem(t, N)
    want = E(w1) / 3 + 0.75 * E(w2) + 0.5 * (E(y) + dt * eu.rhs_adjoint(op, E(q), E(y)))
    check(out, want, what=f"stage adjoint N={N}")
    with pytest.raises(dg.DGError):
        yy = gpu(y)
        dg.dg_rk_stage_adjoint(lm, ph, 0.0, None, 0.0, None, 1.0, dt, gpu(q), yy, yy)


def test_rk3_step_adjoint_matches_oracle():
    od = oracle_desc(3, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(3, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, 44))
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q0 = eu.bubble_state(op) + to_elem(torch.as_tensor(random_state(om.K, 3, 45)), 3) * 0.1
    lam3 = to_elem(torch.as_tensor(random_state(om.K, 3, 46, (1.0,) * 5)), 3)
    dt = 0.01
    want = eu.rk3_step_adjoint(op, dt, q0, lam3)
    g0 = gpu(to_nodes(q0))
    _, (s0, s1, s2) = adj._step_keep_stages(lm, ph, dt, g0)
    got = adj.rk3_step_adjoint(lm, ph, dt, s0, s1, s2, gpu(to_nodes(lam3)))
    check(got, want, what="rk3 step adjoint")


def _functional_weights(op, box):
    """J_e W_n 1_box, rho_bar and Theta_bar at the nodes (node layout, on the GPU)."""
    X, Y, Z = eu.node_xyz(op.mesh)
    (x0, x1), (y0, y1), (z0, z1) = box
    mask = ((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1) & (Z >= z0) & (Z <= z1)).double()
    wm = gpu(to_nodes((eu.quad_weights(op) * mask)[None])[0])
    rb = gpu(to_nodes(op.bg[0][None])[0])
    tb = gpu(to_nodes(op.bg[1][None])[0])
    return wm, rb, tb


def _functional_parts(om, ph, box):
    """Test-side functional J(q) = sum J_e W_n 1_box theta'^2 (torch on the GPU)."""
    op = eu.Operator(om, oracle_phys(ph))
    wm, rb, tb = _functional_weights(op, box)

    def J(q):
        thp = (tb + q[4]) / (rb + q[0]) - tb / rb
        return (wm * thp * thp).sum()

    return J, op


def test_integrate_gradient_fd_and_checkpoints():
    """Adjoint configuration in miniature: bubble on a uniform mesh, N = 4,
    J = integral of theta'^2 over a 200 m box, gradient w.r.t. the initial state
    by the checkpointed adjoint; central differences (eps = 1e-6) on seeded
    directions; checkpoint spacing does not change the gradient."""
    lm, om = both_meshes(4, (4, 4, 4), 0)
    ph = dg.PhysParams()
    box = ((400.0, 600.0), (400.0, 600.0), (250.0, 450.0))
    J, op = _functional_parts(om, ph, box)
    q0 = gpu(to_nodes(eu.bubble_state(op)))
    dt, nsteps = 0.02, 6

    def grad(ck):
        x = q0.clone().requires_grad_(True)
        Jv = J(adj.integrate(x, lm, ph, dt, nsteps, ck))
        (g,) = torch.autograd.grad(Jv, x)
        return g

    g = grad(2)
    assert torch.equal(g, grad(6)) and torch.equal(g, grad(4))

    def Jonly(x):
        with torch.no_grad():
            return float(J(adj.integrate(x, lm, ph, dt, nsteps, nsteps)))

    eps = 1e-6
    for k in range(1, 4):
        d = gpu(torch.as_tensor(random_direction(om.K, 4, k)))
        fd = (Jonly(q0 + eps * d) - Jonly(q0 - eps * d)) / (2 * eps)
        ad = float((g * d).sum())
        print("direction", k, "fd", fd, "adjoint", ad, flush=True)
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (k, fd, ad)


@pytest.mark.parametrize("N,seed", [(2, 60), (4, 61), (7, 62)], ids=lambda x: str(x))
def test_transfer_adjoints_random_amr(N, seed):
    """dg_refine_project_adjoint / dg_coarsen_project_adjoint against the oracle's
    transposes, and <P x, y> = <x, P^T y> with the library's own forward transfers."""
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, seed))
    rng = np.random.default_rng(seed)
    fl_r = (rng.random(om.K) < 0.4).astype(np.int8)
    lr = dg.dg_mesh_build(prev=lm, flags=fl_r, pass_=dg.DG_PASS_REFINE)
    orr = fo.build(od, om, fl_r, fo.PASS_REFINE)
    fl_c = np.where(orr.levels() == 2, -1, np.where(orr.levels() == 1, -1, 0)).astype(np.int8)
    lc = dg.dg_mesh_build(prev=lr, flags=fl_c, pass_=dg.DG_PASS_COARSEN)
    oc = fo.build(od, orr, fl_c, fo.PASS_COARSEN)
    assert tables_equal(lr.tables(), orr) and tables_equal(lc.tables(), oc)
    assert lr.info.n_refined > 0 and lc.info.n_coarsened > 0
    for name, fwd, tr_adj, src, dst, ot, oadj, Kf in (
            ("refine", dg.dg_refine_project, dg.dg_refine_project_adjoint, lm, lr, orr, eu.refine_project_adjoint,
             om.K),
            ("coarsen", dg.dg_coarsen_project, dg.dg_coarsen_project_adjoint, lr, lc, oc, eu.coarsen_project_adjoint,
             orr.K)):
        y = torch.as_tensor(random_state(dst.K, N, seed + 1, (1.0,) * 5))
        x = torch.as_tensor(random_state(src.K, N, seed + 2, (1.0,) * 5))
        g = src.field()
        tr_adj(src, dst, gpu(y), g)
        check(g, oadj(ot, to_elem(y, N), Kf), what=f"{name} transpose N={N}")
        px = dst.field()
        fwd(src, dst, gpu(x), px)
        torch.cuda.synchronize()
        a = float((px.cpu() * y).sum())
        b = float((x * g.cpu()).sum())
        assert abs(a - b) <= 1e-13 * max(abs(a), abs(b)), (name, a, b)


def _plan_meshes(N, seed):
    """A fixed mesh sequence with real changes: an AMR start, then two cycles, each
    coarsening every family of level-1 leaves and refining random leaves; library
    meshes and the oracle's, tables equal."""
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, seed))
    rng = np.random.default_rng(seed)
    cycles, ocycles = [], []
    m, o = lm, om
    for _ in range(2):
        flc = np.where(o.levels() == 1, -1, 0).astype(np.int8)
        mc = dg.dg_mesh_build(prev=m, flags=flc, pass_=dg.DG_PASS_COARSEN)
        oc = fo.build(od, o, flc, fo.PASS_COARSEN)
        assert mc.info.n_coarsened > 0
        flr = (rng.random(oc.K) < 0.3).astype(np.int8)
        mr = dg.dg_mesh_build(prev=mc, flags=flr, pass_=dg.DG_PASS_REFINE)
        orr = fo.build(od, oc, flr, fo.PASS_REFINE)
        assert mr.info.n_refined > 0 and tables_equal(mc.tables(), oc) and tables_equal(mr.tables(), orr)
        cycles.append((mc, mr))
        ocycles.append((oc, orr))
        m, o = mr, orr
    return lm, om, adj.AdaptPlan(cycles), ocycles


def test_integrate_adaptive_gradient_through_transfers():
    """Gradient of J(q_T) through 6 SSP-RK3 steps with two adaptation cycles (a
    replayed mesh sequence that coarsens and refines): against the oracle's
    reverse-mode derivative of its own steps and transfers, and against central
    differences on seeded directions along the same sequence."""
    N, dt, nsteps, every = 3, 0.02, 6, 2
    lm, om, plan, ocycles = _plan_meshes(N, 63)
    ph = dg.PhysParams()
    om_T = ocycles[-1][1]
    box = ((300.0, 700.0), (300.0, 700.0), (200.0, 600.0))
    J, opT = _functional_parts(om_T, ph, box)
    op0 = eu.Operator(om, oracle_phys(ph))
    q0o = eu.bubble_state(op0) + 0.1 * to_elem(torch.as_tensor(random_state(om.K, N, 64)), N)
    q0 = gpu(to_nodes(q0o))
    x = q0.clone().requires_grad_(True)
    qT, mT, _ = adj.integrate_adaptive(x, lm, ph, dt, nsteps, every, plan=plan, ckpt_every=2)
    assert mT is plan.cycles[-1][1]
    (g,) = torch.autograd.grad(J(qT), x)
    # the oracle: the same steps and transfers, differentiated in reverse mode
    xo = q0o.clone().requires_grad_(True)
    qo, o, cyc = xo, om, 0
    for n in range(nsteps):
        qo = eu.ssp_rk3_step(eu.Operator(o, oracle_phys(ph)), dt, qo)
        if (n + 1) % every == 0 and n + 1 < nsteps:
            oc, orr = ocycles[cyc]
            qo = eu.refine_project(orr, eu.coarsen_project(oc, qo))
            o, cyc = orr, cyc + 1
    wm, rb, tb = (to_elem(t.cpu()[None], N)[0] for t in _functional_weights(opT, box))
    thp = (tb + qo[4]) / (rb + qo[0]) - tb / rb
    (go,) = torch.autograd.grad((wm * thp * thp).sum(), xo)
    check(g, go, what="adaptive gradient vs oracle")

    def Jonly(y):
        with torch.no_grad():
            return float(J(adj.integrate_adaptive(y, lm, ph, dt, nsteps, every, plan=plan)[0]))

    eps = 1e-6
    for k in range(1, 4):
        d = gpu(torch.as_tensor(random_direction(om.K, N, k)))
        fd = (Jonly(q0 + eps * d) - Jonly(q0 - eps * d)) / (2 * eps)
        ad = float((g * d).sum())
        print("adaptive direction", k, "fd", fd, "adjoint", ad, flush=True)
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (k, fd, ad)
