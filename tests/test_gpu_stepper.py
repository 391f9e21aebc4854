"""The overlapped adaptive stepper (regrid decision on the host while the GPU
computes the next step on the current mesh) against the plain order of calls:
adaptation cycle, then the step.  Both run the same library calls on the same
inputs, so the states and meshes must agree bitwise, on cycles that change the
mesh and on cycles that do not."""
import pytest
import torch

from paper_2404_16648_amd import dg

pytestmark = pytest.mark.gpu


def _tables_equal(a, b):
    ta, tb = a.tables(), b.tables()
    return ta.keys() == tb.keys() and all((ta[k] == tb[k]).all() for k in ta)


@pytest.mark.parametrize("N,every,buffer,steps", [(3, 2, 0, 9), (4, 3, 1, 13)])
def test_stepper_matches_cycle_then_step(N, every, buffer, steps):
    print(f"stepper N={N} every={every} buffer={buffer} steps={steps}", flush=True)
    ph = dg.PhysParams()
    thr, dt = 0.1, 0.02
    # start one level below the adapted mesh, so the first cycle refines and later
    # cycles (the bubble barely moves) change nothing
    m0 = dg.dg_mesh_build(N, (4, 4, 4), 2, (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))
    q0 = m0.field()
    dg.dg_init_bell(m0, ph, q0, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))

    st = dg.AdaptiveStepper(m0, ph, q0.clone(), dt, every, dg.DG_IND_THETA, thr, buffer=buffer)
    for _ in range(steps):
        st.step()

    m, q = m0, q0.clone()
    for n in range(steps):
        if n > 0 and n % every == 0:
            m2, q = dg.adapt_cycle(m, ph, q, dg.DG_IND_THETA, thr, buffer=buffer)
            m2.prev = None
            m = m2
        q1, q2 = torch.empty_like(q), torch.empty_like(q)
        dg.ssp_rk3_step(m, ph, dt, q, q1, q2)
    torch.cuda.synchronize()
    assert m.K == st.mesh.K and _tables_equal(m, st.mesh)
    assert torch.equal(q, st.q)
    assert st.cycles == (steps - 1) // every and st.changed >= 1
    if buffer == 0:  # the speculative step is also kept at least once
        assert st.changed < st.cycles, (st.changed, st.cycles)


def test_stepper_on_its_own_stream():
    """The stepper on a stream of its own (not torch's current stream), with
    unrelated allocations and work on the current stream between its steps, gives
    the same state as the plain order of calls on the current stream; its buffers
    are allocated for its stream, so blocks it drops at a cycle that changes the
    mesh are not handed to the other stream's work while it still uses them."""
    N, every, steps = 3, 2, 9
    ph = dg.PhysParams()
    thr, dt = 0.1, 0.02
    m0 = dg.dg_mesh_build(N, (4, 4, 4), 2, (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0))
    q0 = m0.field()
    dg.dg_init_bell(m0, ph, q0, 2.0, (500.0, 500.0, 350.0), (250.0, 250.0, 250.0))
    side = torch.cuda.Stream()
    st = dg.AdaptiveStepper(m0, ph, q0.clone(), dt, every, dg.DG_IND_THETA, thr, stream=side)
    for _ in range(steps):
        st.step()
        junk = torch.empty(st.q.numel() * 3, dtype=torch.float64, device="cuda")
        junk.fill_(float("nan"))                 # would poison a block still in use by `side`
        del junk
    side.synchronize()
    m, q = m0, q0.clone()
    for n in range(steps):
        if n > 0 and n % every == 0:
            m2, q = dg.adapt_cycle(m, ph, q, dg.DG_IND_THETA, thr)
            m2.prev = None
            m = m2
        q1, q2 = torch.empty_like(q), torch.empty_like(q)
        dg.ssp_rk3_step(m, ph, dt, q, q1, q2)
    torch.cuda.synchronize()
    assert st.changed >= 1
    assert m.K == st.mesh.K and _tables_equal(m, st.mesh)
    assert torch.equal(q, st.q)
