"""dg_budgets_noalloc (the allocation-free budgets: partial sums in a file-scope
device array) against dg_budgets (partial sums in the mesh's workspace) through
the C ABI: the same kernels in the same order, so the four budgets must agree
bitwise, on two calls in a row, the second on a smaller mesh; a mesh without
device tables is refused (making them would allocate)."""
import numpy as np
import pytest
import torch

from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state

pytestmark = pytest.mark.gpu

BOX = ((0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))


def _mesh_and_state(N, nroot, seed):
    m = dg.dg_mesh_build(N, nroot, 1, *BOX)
    fl = (np.random.default_rng(seed).random(m.K) < 0.35).astype(np.int8)
    m = dg.dg_mesh_build(prev=m, flags=fl, pass_=dg.DG_PASS_REFINE)
    q = torch.as_tensor(random_state(m.K, N, seed)).to("cuda")
    return m, q


def test_budgets_noalloc_matches_budgets():
    ph = dg.PhysParams()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    # the first mesh runs the reduction's full 1024 blocks, the second far fewer
    for N, nroot, seed in ((3, (8, 8, 8), 1), (4, (2, 2, 1), 2)):
        m, q = _mesh_and_state(N, nroot, seed)
        print(f"noalloc budgets: N={N} leaves={m.K}", flush=True)
        want = dg.dg_budgets(m, ph, q)       # makes the mesh's device tables
        dg.dg_budgets_noalloc(m, ph, q, out)
        torch.cuda.synchronize()
        got = out.cpu().tolist()
        assert got == list(want), (got, want)
    assert _mesh_and_state(4, (2, 2, 1), 2)[0].K < 1024 < _mesh_and_state(3, (8, 8, 8), 1)[0].K


def test_budgets_noalloc_refuses_a_mesh_without_device_tables():
    ph = dg.PhysParams()
    m = dg.dg_mesh_build(3, (2, 2, 2), 0, *BOX)
    q = m.field()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError):
        dg.dg_budgets_noalloc(m, ph, q, out)
