"""SSP-RK3 steps captured as a HIP graph and replayed, against the same steps
launched eagerly: every replay, with eager work and synchronisations of the
program's own between the replays, must give the eager result bitwise (an AMR
mesh, so the mortar pre-pass is in the graph too)."""
import pytest
import torch

from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import oracle_desc, random_refinements
from tests.test_gpu_parity import BOX, both_meshes, gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [4, 7])
def test_graph_replays_match_eager_steps(N):
    print(f"graph N={N}", flush=True)
    od = oracle_desc(N, (2, 2, 2), 2, *BOX, (0, 0, 0))
    lm, om = both_meshes(N, (2, 2, 2), 2, flag_seq=random_refinements(od, 2, 81))
    assert lm.info.n_hang > 0
    ph = dg.PhysParams()
    q = gpu(torch.as_tensor(random_state(lm.K, N, 82)) * 0.1)
    ref = q.clone()
    g = dg.GraphedSteps(lm, ph, 0.002, q.clone(), 3)
    r1, r2 = torch.empty_like(q), torch.empty_like(q)
    for rep in range(3):
        g.replay()
        for _ in range(3):  # the same steps, eager, between the replays
            dg.ssp_rk3_step(lm, ph, 0.002, ref, r1, r2)
        junk = torch.randn(1 << 16, device=q.device, dtype=torch.float64).sum()  # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(g.q, ref), rep
