"""The precision split on the cubed-sphere shell on the GPU: the stage's line
contractions in float32 (the contravariant flux minus its value at the element's
first node, D split into float32 high and low parts, float32 accumulation),
faces, curved mortars, metric terms and the update in float64; in the adjoint the
transposed contractions in float32 likewise.  Judged against the float64 oracle
at relative L2 <= 1e-5 for every component, on uniform and refined shells at
N = 2..5, over ten SSP-RK3 steps of a Gaussian theta vortex on a shell refined
around it, and for the checkpointed gradient through 20 steps against the
float64 gradient.  The float32 contractions break the exact
summation-by-parts cancellation of the volume term against the faces, so the
total mass drifts by a float32 rounding of the flux divergence (reported, and
bounded far below the field tolerance)."""
import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import assert_fields, field_errors, to_elem, to_nodes
from tests.test_gpu_parity import gpu
from tests.test_gpu_sphere_adjoint import SHELLS, _id, _shell

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5
MIXED = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, precision=dg.DG_MIXED)
OPH = eu.Phys()


@pytest.mark.parametrize("case", SHELLS, ids=_id)
def test_mixed_shell_rhs_and_stage(case):
    N = case["N"]
    lm, om = _shell(**case)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 40 + N)) * 0.1 + to_nodes(sp.vortex_state(op, width=2.0e6))
    q0n = torch.as_tensor(random_state(om.K, N, 50 + N)) * 0.1
    R, out = lm.field(), lm.field()
    dg.dg_rhs(lm, MIXED, gpu(qn), R)
    dg.dg_rk_stage(lm, MIXED, 0.75, 0.25, 2.0, gpu(q0n), gpu(qn), out)
    torch.cuda.synchronize()
    print(f"mixed shell N={N} K={om.K} hanging={len(om.hang)}", flush=True)
    q = to_elem(qn, N)
    assert_fields(R, to_nodes(op.rhs(q)), TOL_MIXED, "mixed shell rhs")
    assert_fields(out, to_nodes(eu.rk_stage(op, 0.75, 0.25, 2.0, to_elem(q0n, N), q)), TOL_MIXED, "mixed shell stage")


def test_mixed_shell_vortex_steps():
    """a 6 x 4 x 4 x 1 shell, N = 4, refined once where theta' > 0.3 K of a Gaussian
    vortex 2000 km wide; ten SSP-RK3 steps of 2 s in the split against the float64
    oracle, compared after every step (the vortex at rest: momentum as one vector)"""
    N, dt = 4, 2.0
    lm = dg.dg_sphere_mesh_build(N, 4, 1, max_level=1)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=4, nz=1, max_level=1))
    op0 = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    fl = dg.dg_indicator(lm, MIXED, gpu(to_nodes(sp.vortex_state(op0, width=2.0e6))), dg.DG_IND_THETA, 0.3)
    fl = np.where(np.asarray(fl) > 0, 1, 0).astype(np.int8)
    lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    om = sp.refine_pass(om, fl)
    assert np.array_equal(lm.tables()["leaf"], om.leaves.astype(np.int32)) and len(om.hang) > 0
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qo = sp.vortex_state(op, width=2.0e6)
    q = gpu(to_nodes(qo))
    a, b = lm.field(), lm.field()
    b0 = dg.dg_budgets(lm, MIXED, q)
    worst = [0.0, 0.0, 0.0]
    for step in range(10):
        dg.ssp_rk3_step(lm, MIXED, dt, q, a, b)
        qo = eu.ssp_rk3_step(op, dt, qo)
        torch.cuda.synchronize()
        err = field_errors(q, to_nodes(qo))
        worst = [max(w, e) for w, e in zip(worst, err)]
        assert max(err) <= TOL_MIXED, (step, err)
    b1 = dg.dg_budgets(lm, MIXED, q)
    print(f"mixed vortex shell K={om.K}: worst relative L2 over 10 steps (rho', momentum, Theta') "
          f"{['%.2e' % w for w in worst]}, mass change {(b1[1] - b0[1]) / b0[1]:.2e}", flush=True)
    assert abs(b1[1] - b0[1]) <= 1e-12 * b0[1]


@pytest.mark.parametrize("case", [SHELLS[1], SHELLS[2], SHELLS[5], SHELLS[7]], ids=_id)
def test_mixed_shell_adjoint(case):
    """dg_rhs_adjoint and dg_rk_stage_adjoint with the precision split (the transposed
    contractions in float32) against the float64 oracle's adjoint"""
    N = case["N"]
    lm, om = _shell(**case)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn = torch.as_tensor(random_state(om.K, N, 60 + N)) * 0.1 + to_nodes(sp.vortex_state(op, width=2.0e6))
    ln = torch.as_tensor(random_state(om.K, N, 61 + N))
    wn = torch.as_tensor(random_state(om.K, N, 62 + N))
    want = to_nodes(eu.rhs_adjoint(op, to_elem(qn, N), to_elem(ln, N)))
    g = lm.field()
    dg.dg_rhs_adjoint(lm, MIXED, gpu(qn), gpu(ln), g)
    assert_fields(g, want, TOL_MIXED, f"mixed shell adjoint N={N}")
    dt = 2.0
    dg.dg_rk_stage_adjoint(lm, MIXED, 0.5, gpu(wn), 0.0, None, 0.25, dt, gpu(qn), gpu(ln), g)
    assert_fields(g, 0.5 * wn + 0.25 * (ln + dt * want), TOL_MIXED, f"mixed shell stage adjoint N={N}")


def test_mixed_shell_gradient_through_steps():
    """the checkpointed gradient of a functional through 20 SSP-RK3 steps on a shell
    refined around the vortex, forward and adjoint with the precision split, against
    the float64 gradient (both from the library; the float64 path is pinned to the
    oracle and to central differences)"""
    from paper_2404_16648_amd import adjoint as adj
    N, dt = 3, 2.0
    lm, om = _shell(N=N, n=3, nz=1, L=1, seed=31, fracs=(0.3,))
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    q0 = gpu(to_nodes(sp.vortex_state(op, width=2.0e6)))
    wm = gpu(to_nodes(sp.quad_weights(op)[None])[0])
    fp64 = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)

    def grad(phys):
        x = q0.clone().requires_grad_(True)
        qT = adj.integrate(x, lm, phys, dt, 20, 10)
        (g,) = torch.autograd.grad((wm * qT[4] * qT[4]).sum() + (wm * qT[0] * qT[0]).sum(), x)
        return g

    g64, gmx = grad(fp64), grad(MIXED)
    err = field_errors(gmx, g64)
    print("mixed shell gradient vs float64", ["%.2e" % x for x in err], flush=True)
    assert max(err) <= TOL_MIXED
