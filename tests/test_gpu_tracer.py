"""The passive tracer on the GPU (section 2.1's C = rho c; section 4.2's tracer
loss of mortars against pointwise matching): dg_tracer_rhs and dg_tracer_stage
against the oracle's tracer operator on AMR meshes at every order with both
hanging-face schemes, the tracer with c = 1 against the library's own mass
equation, the tracer's budget through SSP-RK3 steps (mortars conserve it,
pointwise matching does not), and the conservative transfer of a tracer field
and of several fields at once (dg_project_fields) against the oracle's."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import TOL_FP64, oracle_desc, oracle_phys, phys_for, random_refinements, tables_equal, to_elem
from tests.test_gpu_parity import AMR_CASES, BOX, both_meshes, gpu

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = a.detach().double().cpu().reshape(-1), b.detach().double().cpu().reshape(-1)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _tracer_field(K, N, seed):
    return 1.0 + 0.2 * torch.as_tensor(np.random.default_rng(seed).standard_normal((K, (N + 1) ** 3)))


@pytest.mark.parametrize("scheme", ["mortar", "pointwise"])
@pytest.mark.parametrize("case", AMR_CASES, ids=lambda c: f"N{c['N']}")
def test_tracer_rhs_and_stage_amr(case, scheme):
    N = case["N"]
    od = oracle_desc(N, case["nroot"], case["L"], *BOX, case["periodic"])
    lm, om = both_meshes(N, case["nroot"], case["L"], case["periodic"],
                         flag_seq=random_refinements(od, 2, case["seed"]))
    assert lm.info.n_hang > 0
    ph = phys_for(case["periodic"])
    if scheme == "pointwise":
        ph = dataclasses.replace(ph, nonconforming=dg.DG_NC_POINTWISE)
    op = eu.Operator(om, oracle_phys(ph), nonconforming=scheme)
    qn = torch.as_tensor(random_state(om.K, N, case["seed"] + 7))
    cs = _tracer_field(om.K, N, case["seed"] + 8)
    c0 = _tracer_field(om.K, N, case["seed"] + 9)
    R = torch.empty_like(gpu(cs))
    dg.dg_tracer_rhs(lm, ph, gpu(qn), gpu(cs), R)
    out = torch.empty_like(R)
    dg.dg_tracer_stage(lm, ph, 0.75, 0.25, 0.002, gpu(qn), gpu(c0), gpu(cs), out)
    torch.cuda.synchronize()
    q = to_elem(qn, N)
    Ro = eu.tracer_rhs(op, q, cs.reshape(om.K, N + 1, N + 1, N + 1)).reshape(om.K, -1)
    So = eu.tracer_stage(op, 0.75, 0.25, 0.002, q, c0.reshape(Ro.shape[0], N + 1, N + 1, N + 1),
                         cs.reshape(om.K, N + 1, N + 1, N + 1)).reshape(om.K, -1)
    e1, e2 = rel(R, Ro), rel(out, So)
    print(f"tracer {scheme} N={N}: rhs {e1:.2e} stage {e2:.2e}", flush=True)
    assert e1 <= TOL_FP64 and e2 <= TOL_FP64


def test_tracer_with_c_one_is_the_mass_equation():
    """C = rho: the tracer right-hand side equals the library's own R_rho' (a
    background constant in z, so the mortars interpolate the full and the
    perturbation density alike)."""
    N = 4
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 91))
    ph = dg.PhysParams(g=0.0)
    q = gpu(torch.as_tensor(random_state(om.K, N, 92)))
    op = eu.Operator(om, oracle_phys(ph))
    rho = gpu(op.bg[0].reshape(om.K, -1)) + q[0]
    R = lm.field()
    dg.dg_rhs(lm, ph, q, R)
    Rc = torch.empty_like(rho)
    dg.dg_tracer_rhs(lm, ph, q, rho, Rc)
    torch.cuda.synchronize()
    assert rel(Rc, R[0]) <= 1e-12, rel(Rc, R[0])


def test_tracer_budget_mortar_against_pointwise():
    """10 SSP-RK3 steps of the AMR bubble with a tracer bell: the tracer integral
    changes at round-off with mortars, by far more with pointwise matching."""
    N = 4
    od = oracle_desc(N, (4, 4, 4), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (4, 4, 4), 2, flag_seq=random_refinements(od, 1, 93, p=0.3))
    gaps = {}
    for scheme in (dg.DG_NC_MORTAR, dg.DG_NC_POINTWISE):
        ph = dg.PhysParams(nonconforming=scheme)
        q = lm.field()
        dg.dg_init_bell(lm, ph, q, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
        q += 0.05 * gpu(torch.as_tensor(random_state(om.K, N, 94)))
        c = 1.0 + q[0].clone() * 0.0 + 0.5 * gpu(_tracer_field(om.K, N, 95) - 1.0)
        q1, q2, c1, c2 = lm.field(), lm.field(), torch.empty_like(c), torch.empty_like(c)
        m0 = dg.dg_tracer_mass(lm, c)
        for _ in range(10):
            dg.ssp_rk3_step_tracer(lm, ph, 0.01, q, q1, q2, c, c1, c2)
        m1 = dg.dg_tracer_mass(lm, c)
        gaps[scheme] = abs(m1 - m0) / abs(m0)
    print("tracer budget change over 10 steps: mortar", gaps[dg.DG_NC_MORTAR], "pointwise",
          gaps[dg.DG_NC_POINTWISE], flush=True)
    assert gaps[dg.DG_NC_MORTAR] < 1e-14
    assert gaps[dg.DG_NC_POINTWISE] > 1e3 * max(gaps[dg.DG_NC_MORTAR], 1e-16)


def test_tracer_steps_beside_the_euler_stages_are_bitwise_the_same():
    """ssp_rk3_step_tracer with the tracer stages on a side stream (beside the Euler
    stages) against the one-stream order: bitwise the same state and tracer after
    5 steps, the side-stream run starting on a mesh with no device tables yet"""
    N = 4
    od = oracle_desc(N, (4, 4, 4), 2, *BOX, (0, 0, 0))
    seq = random_refinements(od, 1, 93, p=0.3)
    runs = []
    for use_side in (False, True):
        lm, om = both_meshes(N, (4, 4, 4), 2, flag_seq=seq)
        ph = dg.PhysParams()
        q = lm.field()
        dg.dg_init_bell(lm, ph, q, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
        q += 0.05 * gpu(torch.as_tensor(random_state(om.K, N, 94)))
        c = 0.5 + 0.5 * gpu(_tracer_field(om.K, N, 95))
        q1, q2, c1, c2 = lm.field(), lm.field(), torch.empty_like(c), torch.empty_like(c)
        side = torch.cuda.Stream() if use_side else None
        for _ in range(5):
            dg.ssp_rk3_step_tracer(lm, ph, 0.01, q, q1, q2, c, c1, c2, side=side)
        torch.cuda.synchronize()
        runs.append((q.cpu(), c.cpu()))
    print("side-stream tracer steps: K", om.K, "hanging", len(om.hang), flush=True)
    assert len(om.hang) > 0
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])


def test_project_fields_against_oracle():
    N = 3
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 1, 96))
    fl = (np.random.default_rng(97).random(om.K) < 0.4).astype(np.int8)
    lr = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    orr = fo.build(od, om, fl, fo.PASS_REFINE)
    assert tables_equal(lr.tables(), orr)
    for nv in (1, 3):
        x = torch.as_tensor(np.random.default_rng(98 + nv).standard_normal((nv, om.K, (N + 1) ** 3)))
        y = torch.empty(nv, lr.K, lr.Np, dtype=torch.float64, device="cuda")
        src = gpu(x[0]) if nv == 1 else gpu(x)
        dst = y[0] if nv == 1 else y
        dg.dg_project_fields(lm, lr, src, dst)
        torch.cuda.synchronize()
        want = eu.refine_project(orr, to_elem(x, N)).reshape(nv, lr.K, -1)
        assert rel(y, want) <= TOL_FP64
    fl2 = -np.ones(orr.K, dtype=np.int8)
    lc = dg.dg_mesh_build(prev=lr, flags=fl2, pass_=dg.DG_PASS_COARSEN)
    oc = fo.build(od, orr, fl2, fo.PASS_COARSEN)
    x = torch.as_tensor(np.random.default_rng(99).standard_normal((orr.K, (N + 1) ** 3)))
    y = torch.empty(lc.K, lc.Np, dtype=torch.float64, device="cuda")
    dg.dg_project_fields(lr, lc, gpu(x), y)
    torch.cuda.synchronize()
    want = eu.coarsen_project(oc, to_elem(x[None], N)).reshape(lc.K, -1)
    assert rel(y, want) <= TOL_FP64
    # tracer mass is kept by both transfers
    c = gpu(x)
    assert abs(dg.dg_tracer_mass(lc, y) - dg.dg_tracer_mass(lr, c)) <= 1e-13 * float(c.abs().sum())
