"""GPU parity: the HIP library through the C ABI against the oracle, element by
element on the same seeded inputs (float64, per-variable relative L2 <= 1e-12,
integer tables bit-exact).  Run on an MI355X: ``pytest -m gpu``."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import (TOL_FP64, assert_fields, oracle_desc, oracle_phys, phys_for, random_refinements,
                           tables_equal, to_elem, to_nodes)

pytestmark = pytest.mark.gpu

DEV = "cuda"
BOX = ((0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))


def both_meshes(N, nroot, L, periodic=(0, 0, 0), lo=BOX[0], hi=BOX[1], flag_seq=()):
    lm = dg.dg_mesh_build(N, nroot, L, lo, hi, periodic)
    od = oracle_desc(N, nroot, L, lo, hi, periodic)
    om = fo.build(od, None)
    for fl in flag_seq:
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = fo.build(od, om, fl, fo.PASS_REFINE)
    assert tables_equal(lm.tables(), om)
    return lm, om


def gpu(t):
    return t.to(DEV).contiguous()


def check(a_gpu, b_oracle, tol=TOL_FP64, what="", vector_momentum=False):
    """Every component within tol in relative L2 (bubble states: rho', momentum as
    one vector field and Theta')."""
    assert_fields(a_gpu, to_nodes(b_oracle), tol, what, vector_momentum)


def test_bell_initial_state_matches_oracle():
    lm, om = both_meshes(4, (4, 4, 4), 2)
    ph = dg.PhysParams()
    q = lm.field()
    dg.dg_init_bell(lm, ph, q, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
    op = eu.Operator(om, oracle_phys(ph))
    check(q, eu.bubble_state(op), what="bubble IC", vector_momentum=True)


def test_rhs_config1_bubble():
    """Uniform 4x4x4, N = 4, walls, warm bubble: first RHS."""
    lm, om = both_meshes(4, (4, 4, 4), 2)
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q0 = eu.bubble_state(op)
    R = lm.field()
    dg.dg_rhs(lm, ph, gpu(to_nodes(q0)), R)
    torch.cuda.synchronize()
    Ro = op.rhs(q0)
    check(R, Ro, what="C1 rhs", vector_momentum=True)
    # structural zeros (Theta' = 0, U = 0, rho' continuous): only rho*w is non-zero
    for v in (0, 1, 2, 4):
        assert torch.count_nonzero(R[v]) == 0


AMR_CASES = [
    dict(N=2, nroot=(2, 2, 2), L=2, periodic=(0, 0, 0), seed=1),
    dict(N=3, nroot=(2, 3, 2), L=2, periodic=(1, 0, 1), seed=2),
    dict(N=4, nroot=(2, 2, 2), L=2, periodic=(1, 1, 1), seed=3),
    dict(N=5, nroot=(2, 1, 2), L=2, periodic=(0, 1, 0), seed=4),
    dict(N=6, nroot=(1, 2, 2), L=2, periodic=(0, 0, 1), seed=5),
    dict(N=7, nroot=(2, 2, 2), L=2, periodic=(0, 0, 0), seed=6),
]


@pytest.mark.parametrize("case", AMR_CASES, ids=lambda c: f"N{c['N']}")
def test_rhs_random_state_amr(case):
    od = oracle_desc(case["N"], case["nroot"], case["L"], *BOX, case["periodic"])
    seq = random_refinements(od, 2, case["seed"])
    lm, om = both_meshes(case["N"], case["nroot"], case["L"], case["periodic"], flag_seq=seq)
    assert lm.info.n_hang > 0
    ph = phys_for(case["periodic"])
    op = eu.Operator(om, oracle_phys(ph))
    qn = torch.as_tensor(random_state(om.K, om.N, case["seed"]))
    q = to_elem(qn, om.N)
    R = lm.field()
    dg.dg_rhs(lm, ph, gpu(qn), R)
    torch.cuda.synchronize()
    check(R, op.rhs(q), what=f"rhs N={case['N']}")


@pytest.mark.parametrize("N", [4, 7])
def test_rhs_large_theta_perturbation(N):
    """Theta' up to ~+-25% of Thetabar: P' leaves the short binomial series and takes
    the kernels' wide-range path (log-halving), checked against the oracle's
    expm1/log1p form, on faces, mortars and volume, with a periodic wrap along x
    and walls along z (gravity on: the background varies with z)."""
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (1, 0, 0))
    seq = random_refinements(od, 2, 31 + N)
    lm, om = both_meshes(N, (2, 2, 2), 2, (1, 0, 0), flag_seq=seq)
    assert lm.info.n_hang > 0
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    qn = torch.as_tensor(random_state(om.K, N, 40 + N, scales=(1e-3, 0.1, 0.1, 0.1, 30.0)))
    x = qn[4] / to_nodes(op.bg[1][None])[0]
    assert float(x.abs().max()) > 0.1  # far outside the series range 2^-7
    R = lm.field()
    dg.dg_rhs(lm, ph, gpu(qn), R)
    out = lm.field()
    dg.dg_rk_stage(lm, ph, 0.75, 0.25, 0.001, gpu(qn), gpu(qn), out)
    torch.cuda.synchronize()
    q = to_elem(qn, N)
    check(R, op.rhs(q), what=f"rhs wide P' N={N}")
    check(out, eu.rk_stage(op, 0.75, 0.25, 0.001, q, q), what=f"stage wide P' N={N}")


@pytest.mark.parametrize("case", AMR_CASES, ids=lambda c: f"N{c['N']}")
def test_rk_stage_random_state_amr(case):
    """A Shu-Osher stage with q0 distinct from the stage input (the update reads q0),
    at every order: the low orders gather the tile and traces into LDS, N = 6, 7
    load straight into registers."""
    od = oracle_desc(case["N"], case["nroot"], case["L"], *BOX, case["periodic"])
    seq = random_refinements(od, 2, case["seed"] + 100)
    lm, om = both_meshes(case["N"], case["nroot"], case["L"], case["periodic"], flag_seq=seq)
    ph = phys_for(case["periodic"])
    op = eu.Operator(om, oracle_phys(ph))
    N = om.N
    q0 = torch.as_tensor(random_state(om.K, N, case["seed"] + 200))
    qs = torch.as_tensor(random_state(om.K, N, case["seed"] + 300))
    out = lm.field()
    dg.dg_rk_stage(lm, ph, 0.75, 0.25, 0.002, gpu(q0), gpu(qs), out)
    torch.cuda.synchronize()
    check(out, eu.rk_stage(op, 0.75, 0.25, 0.002, to_elem(q0, N), to_elem(qs, N)), what=f"stage N={N}")


def test_hydrostatic_rest_bitwise_zero_and_conservation():
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    seq = random_refinements(od, 2, 11)
    lm, om = both_meshes(4, (2, 2, 2), 2, flag_seq=seq)
    ph = dg.PhysParams()
    z = lm.field()
    R = lm.field()
    R.fill_(1.0)
    dg.dg_rhs(lm, ph, z, R)
    q1 = lm.field()
    dg.dg_rk_stage(lm, ph, 0.0, 1.0, 0.05, z, z, q1)
    torch.cuda.synchronize()
    assert torch.count_nonzero(R) == 0 and torch.count_nonzero(q1) == 0
    # discrete conservation of rho' and Theta' with walls and mortars
    op = eu.Operator(om, oracle_phys(ph))
    JW = to_nodes(eu.quad_weights(op)[None])[0]
    qn = torch.as_tensor(random_state(om.K, om.N, 12))
    dg.dg_rhs(lm, ph, gpu(qn), R)
    Rc = R.cpu()
    for v in (0, 4):
        tot = math.fsum((JW * Rc[v]).reshape(-1).tolist())
        scale = float((JW * Rc[v].abs()).sum())
        assert abs(tot) < 1e-13 * scale, (v, tot, scale)


def test_free_stream_gpu():
    od = oracle_desc(3, (2, 2, 2), 2, *BOX, (1, 1, 1))
    seq = random_refinements(od, 2, 13)
    lm, om = both_meshes(3, (2, 2, 2), 2, (1, 1, 1), flag_seq=seq)
    ph = dg.PhysParams(g=0.0, background=dg.DG_BG_CONSTANT, rho0=1.2, Theta0=360.0)
    q = lm.field()
    q[1], q[2], q[3] = 12.0, -7.0, 3.0
    R = lm.field()
    dg.dg_rhs(lm, ph, q, R)
    torch.cuda.synchronize()
    assert float(R.abs().max()) < 1e-13 * 1e5 / 250.0 * 10


def test_rk_stages_and_aliasing():
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    seq = random_refinements(od, 1, 14)
    lm, om = both_meshes(4, (2, 2, 2), 2, flag_seq=seq)
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q0 = torch.as_tensor(random_state(om.K, 4, 15))
    qs = torch.as_tensor(random_state(om.K, 4, 16))
    dt = 0.05
    for a, b in eu.SSP_RK3:
        out = lm.field()
        dg.dg_rk_stage(lm, ph, a, b, dt, gpu(q0), gpu(qs), out)
        want = eu.rk_stage(op, a, b, dt, to_elem(q0, 4), to_elem(qs, 4))
        check(out, want, what=f"stage a={a:.3f}")
    # qout aliasing q0 is allowed
    buf = gpu(q0)
    dg.dg_rk_stage(lm, ph, 1 / 3, 2 / 3, dt, buf, gpu(qs), buf)
    check(buf, eu.rk_stage(op, 1 / 3, 2 / 3, dt, to_elem(q0, 4), to_elem(qs, 4)), what="aliased")
    with pytest.raises(dg.DGError):
        x = gpu(qs)
        dg.dg_rk_stage(lm, ph, 0.0, 1.0, dt, x, x, x)


def test_config1_ten_steps():
    """Config 1: uniform 4^3, N = 4, bubble, dt = 0.05 s, 10 SSP-RK3 steps."""
    lm, om = both_meshes(4, (4, 4, 4), 2)
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    qo = eu.bubble_state(op)
    q = gpu(to_nodes(qo))
    q1, q2 = lm.field(), lm.field()
    for step in range(10):
        dg.ssp_rk3_step(lm, ph, 0.05, q, q1, q2)
        qo = eu.ssp_rk3_step(op, 0.05, qo)
        torch.cuda.synchronize()
        check(q, qo, what=f"C1 step {step + 1}", vector_momentum=True)


def test_refine_and_coarsen_projection():
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    seq = random_refinements(od, 1, 17)
    lm, om = both_meshes(4, (2, 2, 2), 2, flag_seq=seq)
    qn = torch.as_tensor(random_state(om.K, 4, 18))
    fl = (np.random.default_rng(19).random(om.K) < 0.4).astype(np.int8)
    lr = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    orr = fo.build(om.desc, om, fl, fo.PASS_REFINE)
    assert tables_equal(lr.tables(), orr)
    qr = lr.field()
    dg.dg_refine_project(lm, lr, gpu(qn), qr)
    check(qr, eu.refine_project(orr, to_elem(qn, 4)), what="refine")
    fl2 = -np.ones(orr.K, dtype=np.int8)
    lc = dg.dg_mesh_build(prev=lr, flags=fl2, pass_=dg.DG_PASS_COARSEN)
    oc = fo.build(om.desc, orr, fl2, fo.PASS_COARSEN)
    assert tables_equal(lc.tables(), oc)
    qc = lc.field()
    qrn = torch.as_tensor(random_state(orr.K, 4, 20))
    dg.dg_coarsen_project(lr, lc, gpu(qrn), qc)
    check(qc, eu.coarsen_project(oc, to_elem(qrn, 4)), what="coarsen")
    with pytest.raises(dg.DGError):
        dg.dg_coarsen_project(lm, lc, gpu(qn), lc.field())


def test_budgets_and_indicator():
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    seq = random_refinements(od, 2, 21)
    lm, om = both_meshes(4, (2, 2, 2), 2, flag_seq=seq)
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    q = eu.bubble_state(op) + to_elem(torch.as_tensor(random_state(om.K, 4, 22, (1e-4, 0.1, 0.1, 0.1, 1e-2))), 4)
    b = dg.dg_budgets(lm, ph, gpu(to_nodes(q)))
    bo = eu.budgets(op, q)
    for x, y in zip(b, bo):
        assert abs(x - y) <= 1e-12 * abs(y) + 1e-15, (b, bo)
    for kind, thr in ((dg.DG_IND_THETA, 0.1), (dg.DG_IND_GRAD_THETA, 1e-3)):
        eta = torch.zeros(lm.K, dtype=torch.float64, device=DEV)
        fl = dg.dg_indicator(lm, ph, gpu(to_nodes(q)), kind, thr, eta)
        eo = eu.indicator(op, q, kind)
        assert float((eta.cpu() - eo).abs().max()) <= 1e-12 * float(eo.abs().max())
        fo_ = eu.flags_from_indicator(om, eo.numpy(), thr)
        tie = np.abs(eo.numpy() - thr) <= 1e-9 * thr
        assert np.array_equal(fl[~tie], fo_[~tie])


def _adapt_initial_mesh(N, nroot, L, lo, hi, thr, bell):
    """Both sides: uniform -> (oracle IC, oracle flags) -> refine pass, to a fixed point."""
    ph = dg.PhysParams()
    lm, om = both_meshes(N, nroot, L, lo=lo, hi=hi)
    for _ in range(L):
        op = eu.Operator(om, oracle_phys(ph))
        q = bell(op)
        fl = eu.flags_from_indicator(om, eu.indicator(op, q).numpy(), thr)
        fl[fl < 0] = 0
        if not (fl > 0).any():
            break
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = fo.build(om.desc, om, fl, fo.PASS_REFINE)
        assert tables_equal(lm.tables(), om)
    return lm, om


def test_config2_full_size_rhs_and_step():
    """Config 2 mesh (8^3 base, N = 7, 2 levels where |theta'| > 0.1 K): full-size
    RHS and one SSP-RK3 step (dt = 0.001 s) against the oracle."""
    lm, om = _adapt_initial_mesh(7, (8, 8, 8), 2, *BOX, 0.1, eu.bubble_state)
    print("C2 leaves", om.K, "hanging faces", len(om.hang), flush=True)
    assert len(om.hang) > 0
    ph = dg.PhysParams()
    op = eu.Operator(om, oracle_phys(ph))
    qo = eu.bubble_state(op)
    q = gpu(to_nodes(qo))
    R = lm.field()
    dg.dg_rhs(lm, ph, q, R)
    check(R, op.rhs(qo), what="C2 rhs", vector_momentum=True)
    q1, q2 = lm.field(), lm.field()
    dg.ssp_rk3_step(lm, ph, 0.001, q, q1, q2)
    check(q, eu.ssp_rk3_step(op, 0.001, qo), what="C2 step", vector_momentum=True)


def test_unchanged_pass_clones_device_tables():
    """A pass that changes no leaf clones the previous mesh's device block (and its
    background when computed): the RHS on the clone equals the RHS on the source
    bitwise, with the cached background and after the physics changes it; the
    oracle agrees on both; a projection through such a pass copies the field."""
    od = oracle_desc(3, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(3, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 51))
    ph = dg.PhysParams()
    qn = torch.as_tensor(random_state(om.K, 3, 52))
    q = gpu(qn)
    R0 = lm.field()
    dg.dg_rhs(lm, ph, q, R0)  # computes and caches lm's background
    zero = np.zeros(om.K, np.int8)
    m2 = dg.dg_mesh_build(prev=lm, flags=zero, pass_=dg.DG_PASS_REFINE)
    assert tables_equal(m2.tables(), fo.build(od, om, zero, fo.PASS_REFINE)) and m2.info.n_refined == 0
    R2 = m2.field()
    dg.dg_rhs(m2, ph, q, R2)
    torch.cuda.synchronize()
    assert torch.equal(R0, R2)
    check(R2, eu.Operator(om, oracle_phys(ph)).rhs(to_elem(qn, 3)), what="rhs on the cloned mesh")
    # a clone of the clone, then another background (theta0) on it
    m3 = dg.dg_mesh_build(prev=m2, flags=zero, pass_=dg.DG_PASS_COARSEN)
    assert m3.info.n_coarsened == 0 and m3.K == om.K
    ph2 = dg.PhysParams(theta0=290.0)
    R3 = m3.field()
    dg.dg_rhs(m3, ph2, q, R3)
    check(R3, eu.Operator(om, oracle_phys(ph2)).rhs(to_elem(qn, 3)), what="rhs, other background, on the clone")
    # the projections through an unchanged pass copy the field
    qc = m3.field()
    dg.dg_coarsen_project(m2, m3, q, qc)
    torch.cuda.synchronize()
    assert torch.equal(qc, q)


def test_z_periodic_mesh_refuses_a_z_dependent_background():
    """A periodic z axis with gravity on the neutral background is refused (the
    hydrostatic profile cannot be periodic); with g = 0 the same mesh runs."""
    lm = dg.dg_mesh_build(3, (1, 1, 2), 0, *BOX, (0, 0, 1))
    q, R = lm.field(), lm.field()
    with pytest.raises(dg.DGError) as e:
        dg.dg_rhs(lm, dg.PhysParams(), q, R)
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError):
        dg.dg_rhs_adjoint(lm, dg.PhysParams(), q, q.clone(), R)
    dg.dg_rhs(lm, phys_for((0, 0, 1)), q, R)
    torch.cuda.synchronize()
    assert torch.count_nonzero(R) == 0


@pytest.mark.parametrize("N", [4, 7])
def test_isentropic_vortex_amr(N):
    """The isentropic vortex of section 4.1 (R = P0 = 1, gamma = 1.4, constant
    background, no gravity, periodic), extruded one root along z, on a mesh
    refined once around the vortex: Theta'/Thetabar reaches -0.5 (the kernels'
    wide-range P' path) and every variable moves.  RHS and a Shu-Osher stage
    (q0 = the vortex, stage input = the vortex translated by 0.1) against the
    oracle, every component to 1e-12."""
    n, L = 8, 12.0
    lo, hi = (-6.0, -6.0, 0.0), (6.0, 6.0, L / n)
    lm = dg.dg_mesh_build(N, (n, n, 1), 1, lo, hi, (1, 1, 1))
    od = oracle_desc(N, (n, n, 1), 1, lo, hi, (1, 1, 1))
    om = fo.build(od, None)
    lo_e, h_e = fo.elem_lo_h(om)
    c = lo_e + 0.5 * h_e
    fl = ((c[:, 0] ** 2 + c[:, 1] ** 2) < 9.0).astype(np.int8)
    lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    om = fo.build(od, om, fl, fo.PASS_REFINE)
    assert tables_equal(lm.tables(), om) and lm.info.n_hang > 0
    ph = dg.PhysParams(cp=3.5, cv=2.5, P0=1.0, g=0.0, background=dg.DG_BG_CONSTANT, rho0=1.0, Theta0=1.0)
    op = eu.Operator(om, oracle_phys(ph))
    X, Y, _ = eu.node_xyz(om)
    q0 = eu.isentropic_vortex(X, Y, 0.0, gamma=1.4)
    qs = eu.isentropic_vortex(X, Y, 0.1, gamma=1.4)
    assert float(q0[4].min()) < -0.45
    R = lm.field()
    dg.dg_rhs(lm, ph, gpu(to_nodes(q0)), R)
    out = lm.field()
    dg.dg_rk_stage(lm, ph, 0.75, 0.25, 0.01, gpu(to_nodes(q0)), gpu(to_nodes(qs)), out)
    torch.cuda.synchronize()
    Ro = op.rhs(q0)
    # rho w stays zero: the vortex has no w and does not depend on z
    check(R[[0, 1, 2, 4]], Ro[[0, 1, 2, 4]], what=f"vortex rhs N={N}")
    assert float(R[3].abs().max()) <= 1e-13 * float(R[1].abs().max())
    want = eu.rk_stage(op, 0.75, 0.25, 0.01, q0, qs)
    check(out[[0, 1, 2, 4]], want[[0, 1, 2, 4]], what=f"vortex stage N={N}")
    assert float(out[3].abs().max()) <= 1e-15
