"""GPU parity of the discrete adjoint: dg_rhs_adjoint and dg_rk_stage_adjoint
against the oracle's reverse-mode derivative of its own RHS, the dot-product
test against the oracle's forward-mode JVP, and the checkpointed
autograd.Function gradient against central finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from paper_2404_16648_amd import adjoint as adj
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_direction, random_state
from tests.helpers import (TOL_FP64, field_errors, oracle_desc, oracle_phys, random_refinements, rel_l2,
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
    b = to_nodes(b_oracle)
    err = field_errors(a_gpu, b)
    print(what, "fields", ["%.2e" % x for x in err], "components", ["%.2e" % x for x in rel_l2(a_gpu, b)],
          flush=True)
    assert max(err) <= tol, (what, err)


CASES = [
    dict(N=2, nroot=(2, 2, 2), periodic=(0, 0, 0), seed=31),
    dict(N=3, nroot=(2, 3, 2), periodic=(1, 0, 1), seed=32),
    dict(N=4, nroot=(2, 2, 2), periodic=(1, 1, 1), seed=33),
    dict(N=5, nroot=(2, 1, 2), periodic=(0, 1, 0), seed=34),
    dict(N=7, nroot=(2, 2, 2), periodic=(0, 0, 0), seed=35),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c['N']}")
def test_rhs_adjoint_random_amr(case):
    N = case["N"]
    od = oracle_desc(N, case["nroot"], 2, *BOX, case["periodic"])
    lm, om = both_meshes(N, case["nroot"], 2, case["periodic"], random_refinements(od, 2, case["seed"]))
    ph = dg.PhysParams()
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


def test_rk_stage_adjoint_combination():
    od = oracle_desc(3, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(3, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, 38))
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q, y, w1, w2 = (torch.as_tensor(random_state(om.K, 3, s)) for s in (40, 41, 42, 43))
    dt = 0.01
    out = lm.field()
    dg.dg_rk_stage_adjoint(lm, ph, 1 / 3, gpu(w1), 0.75, gpu(w2), 0.5, dt, gpu(q), gpu(y), out)
    E = lambda t: to_elem(t, 3)
    want = E(w1) / 3 + 0.75 * E(w2) + 0.5 * (E(y) + dt * eu.rhs_adjoint(op, E(q), E(y)))
    check(out, want, what="stage adjoint")
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


def _functional_parts(om, ph, box):
    """Test-side functional J(q) = sum J_e W_n 1_box theta'^2 (torch on the GPU)."""
    op = eu.Operator(om, oracle_phys(ph))
    X, Y, Z = eu.node_xyz(om)
    (x0, x1), (y0, y1), (z0, z1) = box
    mask = ((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1) & (Z >= z0) & (Z <= z1)).double()
    wm = gpu(to_nodes((eu.quad_weights(op) * mask)[None])[0])
    rb = gpu(to_nodes(op.bg[0][None])[0])
    tb = gpu(to_nodes(op.bg[1][None])[0])

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
