"""GPU checks of the precision split: volume contractions in float32 (flux minus
an element-constant reference, D split into float32 high and low parts, float32
accumulation), everything else float64.  Judged against the float64 oracle at
relative L2 <= 1e-5 for every field; the conservation drift is reported."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import field_errors, oracle_desc, oracle_phys, random_refinements, rel_l2, tables_equal, \
    to_elem, to_nodes

pytestmark = pytest.mark.gpu

DEV = "cuda"
BOX = ((0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))
TOL_MIXED = 1e-5
MIXED = dg.PhysParams(precision=dg.DG_MIXED)


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


def check(a, b_oracle, what):
    b = to_nodes(b_oracle)
    err = field_errors(a, b)
    print(what, "fields", ["%.2e" % x for x in err], "components", ["%.2e" % x for x in rel_l2(a, b)], flush=True)
    assert max(err) <= TOL_MIXED, (what, err)
    return err


@pytest.mark.parametrize("N", [2, 4, 7])
def test_mixed_rhs_random_amr(N):
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 50 + N))
    op = eu.Operator(om, oracle_phys(MIXED))
    qn = torch.as_tensor(random_state(om.K, N, 60 + N))
    R = lm.field()
    dg.dg_rhs(lm, MIXED, gpu(qn), R)
    check(R, op.rhs(to_elem(qn, N)), f"mixed rhs random N={N}")


def test_mixed_rhs_and_steps_bubble():
    """Evolved bubble (smooth fields, the hard case for float32 cancellation),
    N = 4 on an AMR mesh: RHS, then 10 SSP-RK3 steps compared after each step."""
    od = oracle_desc(4, (4, 4, 4), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(4, (4, 4, 4), 2, flag_seq=random_refinements(od, 1, 70, p=0.2))
    op = eu.Operator(om, oracle_phys(MIXED))
    qo = eu.bubble_state(op)
    for _ in range(3):
        qo = eu.ssp_rk3_step(op, 0.02, qo)
    q = gpu(to_nodes(qo))
    R = lm.field()
    dg.dg_rhs(lm, MIXED, q, R)
    check(R, op.rhs(qo), "mixed rhs bubble")
    q1, q2 = lm.field(), lm.field()
    for s in range(10):
        dg.ssp_rk3_step(lm, MIXED, 0.02, q, q1, q2)
        qo = eu.ssp_rk3_step(op, 0.02, qo)
        check(q, qo, f"mixed step {s + 1}")
    # conservation drift of the float32 volume term (reported, not exact)
    JW = to_nodes(eu.quad_weights(op)[None])[0]
    dg.dg_rhs(lm, MIXED, q, R)
    Rc = R.cpu()
    for v in (0, 4):
        tot = math.fsum((JW * Rc[v]).reshape(-1).tolist())
        scale = float((JW * Rc[v].abs()).sum())
        print("mixed conservation drift", v, tot / scale, flush=True)
        assert abs(tot) <= 1e-5 * scale


def test_mixed_hydrostatic_rest_exact():
    od = oracle_desc(4, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, _ = both_meshes(4, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 71))
    z = lm.field()
    R = lm.field()
    R.fill_(1.0)
    dg.dg_rhs(lm, MIXED, z, R)
    torch.cuda.synchronize()
    assert torch.count_nonzero(R) == 0
