"""Degenerate meshes on the GPU against the oracle: one root periodic along every
axis (each face is conforming with the leaf itself), one root with walls all
round, and one root refined once and periodic (every wrap meets a sibling), at
every order."""
import pytest
import torch

from oracle import euler as eu
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import oracle_phys, phys_for, to_elem
from tests.test_gpu_parity import both_meshes, check, gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("shape", ["self_periodic", "walls", "refined_periodic"])
def test_single_root_meshes(N, shape):
    print(f"degenerate {shape} N={N}", flush=True)
    periodic = (0, 0, 0) if shape == "walls" else (1, 1, 1)
    seq = [torch.ones(1, dtype=torch.int8).numpy()] if shape == "refined_periodic" else []
    lm, om = both_meshes(N, (1, 1, 1), 1, periodic, flag_seq=seq)
    assert lm.K == (8 if seq else 1)
    ph = phys_for(periodic)
    op = eu.Operator(om, oracle_phys(ph))
    qn = torch.as_tensor(random_state(om.K, N, 40 + N))
    R = lm.field()
    dg.dg_rhs(lm, ph, gpu(qn), R)
    q0 = torch.as_tensor(random_state(om.K, N, 60 + N))
    out = lm.field()
    dg.dg_rk_stage(lm, ph, 1.0 / 3.0, 2.0 / 3.0, 0.01, gpu(q0), gpu(qn), out)
    torch.cuda.synchronize()
    check(R, op.rhs(to_elem(qn, N)), what=f"{shape} rhs N={N}")
    check(out, eu.rk_stage(op, 1.0 / 3.0, 2.0 / 3.0, 0.01, to_elem(q0, N), to_elem(qn, N)), what=f"{shape} stage N={N}")
