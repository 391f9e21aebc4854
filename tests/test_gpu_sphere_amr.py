"""Refinement on the cubed-sphere shell on the GPU (section 3.1's forest on the
panels of section 3.4, section 3.3's mortars on curved hanging faces, section 3.4's
transfer, section 4.4's pressure-based regrid): dg_rhs and dg_rk_stage on refined
shells against the oracle at N = 2..5, the transfers of refine and coarsen passes
(fields and the scale factor), the P' indicator, SSP-RK3 steps with the mass kept
to round-off, and adaptation cycles that keep the total mass exactly."""
import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import TOL_FP64, assert_conserved_fields, assert_fields, to_elem, to_nodes
from tests.test_gpu_parity import gpu

pytestmark = pytest.mark.gpu

PH = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
OPH = eu.Phys()


def _refined_pair(N, n, nz, L, seed, fracs):
    lm = dg.dg_sphere_mesh_build(N, n, nz, max_level=L)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz, max_level=L))
    rng = np.random.default_rng(seed)
    for fr in fracs:
        fl = (rng.random(om.K) < fr).astype(np.int8)
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = sp.refine_pass(om, fl)
    assert np.array_equal(lm.tables()["leaf"], om.leaves.astype(np.int32))
    assert len(om.hang) > 0
    return lm, om


@pytest.mark.parametrize("N,n,nz,L,seed", [(2, 1, 2, 2, 1), (3, 2, 1, 2, 2), (4, 2, 1, 1, 3), (5, 1, 1, 1, 4)])
def test_refined_shell_rhs_and_stage(N, n, nz, L, seed):
    lm, om = _refined_pair(N, n, nz, L, seed, (0.4, 0.3)[:L])
    print(f"refined shell N={N} K={om.K} hanging={len(om.hang)}", flush=True)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn, q0n = torch.as_tensor(random_state(om.K, N, 30 + N)) * 0.1, torch.as_tensor(random_state(om.K, N, 40 + N)) * 0.1
    R, out = lm.field(), lm.field()
    dg.dg_rhs(lm, PH, gpu(qn), R)
    dg.dg_rk_stage(lm, PH, 0.75, 0.25, 2.0, gpu(q0n), gpu(qn), out)
    torch.cuda.synchronize()
    q = to_elem(qn, N)
    assert_fields(R, to_nodes(op.rhs(q)), TOL_FP64, "refined shell rhs")
    assert_fields(out, to_nodes(eu.rk_stage(op, 0.75, 0.25, 2.0, to_elem(q0n, N), q)), TOL_FP64, "refined shell stage")


@pytest.mark.parametrize("N", [3, 4])
def test_refined_shell_transfers(N):
    """a refine pass and the coarsen pass that undoes it, library against oracle"""
    lm, om = _refined_pair(N, 2, 1, 2, 7, (0.3,))
    fl = (np.random.default_rng(8).random(om.K) < 0.3).astype(np.int8)
    lm2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    om2 = sp.refine_pass(om, fl)
    o1, o2 = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL), sp.SphereOperator(om2, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 50 + N)) * 0.1 + to_nodes(sp.acoustic_state(o1))
    q2 = lm2.field()
    s = dg.dg_sphere_adapt_project(lm, lm2, PH, gpu(qn), q2)
    q2_ref, s_ref = sp.adapt_project(o1, o2, to_elem(qn, N))
    print("refine pass scale", s, s_ref, flush=True)
    assert abs(s - s_ref) <= 1e-15 * abs(s_ref)
    assert_fields(q2, to_nodes(q2_ref), TOL_FP64, "refine pass transfer")
    b1, b2 = dg.dg_budgets(lm, PH, gpu(qn)), dg.dg_budgets(lm2, PH, q2)
    assert abs(b2[1] - b1[1]) <= 1e-15 * b1[1]
    back = -np.ones(om2.K, dtype=np.int8)
    lm3 = dg.dg_mesh_build(prev=lm2, flags=back, pass_=dg.DG_PASS_COARSEN)
    om3 = sp.coarsen_pass(om2, back)
    assert np.array_equal(lm3.tables()["leaf"], om3.leaves.astype(np.int32))
    o3 = sp.SphereOperator(om3, OPH, sp.BG_ISOTHERMAL)
    q3 = lm3.field()
    s3 = dg.dg_sphere_adapt_project(lm2, lm3, PH, q2, q3)
    q3_ref, _ = sp.adapt_project(o2, o3, to_elem(q2.cpu(), N))
    assert s3 == 1.0
    assert_conserved_fields(q3, to_nodes(q3_ref), (to_nodes(o3.bg[0][None])[0], to_nodes(o3.bg[1][None])[0]), TOL_FP64,
                            "coarsen pass transfer")


def test_refined_shell_pressure_indicator():
    N = 4
    lm, om = _refined_pair(N, 2, 1, 2, 11, (0.3,))
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    q = to_nodes(sp.acoustic_state(op))
    eta = torch.empty(om.K, dtype=torch.float64, device="cuda")
    fl = dg.dg_indicator(lm, PH, gpu(q), dg.DG_IND_PPRIME, 20.0, eta=eta)
    ref = sp.indicator(op, to_elem(q, N), sp.IND_PPRIME)
    assert float((eta.cpu() - ref).abs().max()) <= 1e-12 * float(ref.max())
    want = sp.flags_from_indicator(om, ref.numpy(), 20.0)
    near = np.abs(ref.numpy() - 20.0) <= 1e-9 * 20.0
    assert np.array_equal(np.asarray(fl)[~near], want[~near])
    assert (want > 0).any() and (want < 0).any()


def test_refined_shell_steps_and_cycles_keep_mass():
    """five SSP-RK3 steps of the acoustic state on a refined shell (library against
    oracle, mass change at round-off), then two adaptation cycles on P' (20 Pa):
    the total mass changes by round-off through the regrids"""
    N, dt = 3, 2.0
    ph, oph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, g=0.0), eu.Phys(g=0.0)
    lm, om = _refined_pair(N, 2, 1, 2, 12, (0.3,))
    op = sp.SphereOperator(om, oph, sp.BG_ISOTHERMAL)
    qo = sp.acoustic_state(op)
    q = gpu(to_nodes(qo))
    a, b = lm.field(), lm.field()
    b0 = dg.dg_budgets(lm, ph, q)
    for _ in range(5):
        dg.ssp_rk3_step(lm, ph, dt, q, a, b)
        qo = eu.ssp_rk3_step(op, dt, qo)
    torch.cuda.synchronize()
    b1 = dg.dg_budgets(lm, ph, q)
    assert abs(b1[1] - b0[1]) <= 1e-14 * b0[1]
    assert_fields(q, to_nodes(qo), TOL_FP64, "refined shell steps")
    m = lm
    for cycle in range(2):
        m2, q2 = dg.adapt_cycle(m, ph, q, dg.DG_IND_PPRIME, 20.0)
        bb = dg.dg_budgets(m2, ph, q2)
        print(f"cycle {cycle}: {m.K} -> {m2.K} leaves, mass change {(bb[1] - b0[1]) / b0[1]:.2e}", flush=True)
        assert abs(bb[1] - b0[1]) <= 1e-14 * b0[1]
        m, q = m2, q2
        for _ in range(3):
            a, b = m.field(), m.field()
            dg.ssp_rk3_step(m, ph, dt, q, a, b)
    b3 = dg.dg_budgets(m, ph, q)
    assert abs(b3[1] - b0[1]) <= 1e-14 * b0[1]
