"""The cubed-sphere shell on the GPU (section 3.4 spherical geometry, section 4.4
global tests): dg_rhs and dg_rk_stage on shell meshes against the oracle's
curvilinear operator at N = 2..5 with the isothermal background and radial
gravity, the node positions, SSP-RK3 steps of a Gaussian theta perturbation with
the mass budget held to round-off, and the calls the shell refuses."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import TOL_FP64, assert_fields, to_elem, to_nodes
from tests.test_gpu_parity import gpu

pytestmark = pytest.mark.gpu

PH = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
OPH = eu.Phys()


def _meshes(N, n, nz):
    lm = dg.dg_sphere_mesh_build(N, n, nz)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz))
    assert np.array_equal(dg.dg_sphere_faces(lm), om.nb.astype(np.int32))
    return lm, om


def _state(K, N, seed, scale=0.1):
    return torch.as_tensor(random_state(K, N, seed)) * scale


# element aspect ratios (horizontal over radial size) from 330 to 2000: the
# geometry of both sides is made in long double, so the thin shell's cancellation
# in the metric terms stays below the tolerance
@pytest.mark.parametrize("N,n,nz", [(2, 2, 2), (3, 4, 1), (4, 2, 1), (5, 1, 2), (4, 6, 2)])
def test_sphere_rhs_and_stage(N, n, nz):
    lm, om = _meshes(N, n, nz)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    qn, q0n = _state(om.K, N, 10 + N), _state(om.K, N, 20 + N)
    R, out = lm.field(), lm.field()
    dg.dg_rhs(lm, PH, gpu(qn), R)
    dg.dg_rk_stage(lm, PH, 0.75, 0.25, 2.0, gpu(q0n), gpu(qn), out)
    torch.cuda.synchronize()
    print(f"sphere N={N} n={n} nz={nz} K={om.K}", flush=True)
    q = to_elem(qn, N)
    assert_fields(R, to_nodes(op.rhs(q)), TOL_FP64, "sphere rhs")
    assert_fields(out, to_nodes(eu.rk_stage(op, 0.75, 0.25, 2.0, to_elem(q0n, N), q)), TOL_FP64, "sphere stage")


def test_sphere_node_positions():
    lm, om = _meshes(4, 2, 2)
    xyz = torch.empty(3, lm.K, lm.Np, dtype=torch.float64, device="cuda")
    dg.dg_node_coords(lm, xyz)
    torch.cuda.synchronize()
    geo = sp.SphereGeometry(om)
    for c in range(3):
        ref = geo.x[c].reshape(om.K, -1)
        err = float((xyz[c].cpu() - ref).abs().max())
        assert err <= 1e-15 * 6.4e6 * 4, (c, err)


def test_sphere_steps_conserve_mass():
    """five SSP-RK3 steps of a Gaussian theta perturbation (1 K, 500 km) in the
    isothermal shell: the library's budgets against the oracle's after the steps,
    and the mass change at round-off"""
    N, n, nz = 3, 3, 2
    lm, om = _meshes(N, n, nz)
    op = sp.SphereOperator(om, OPH, sp.BG_ISOTHERMAL)
    geo = op.geo
    rho_b, Th_b, _ = op.bg
    # theta' Gaussian about the point at longitude 0, latitude 0 (the +x axis)
    cosang = geo.rhat[0]
    dist = 6.371e6 * torch.arccos(torch.clamp(cosang, -1.0, 1.0))
    thp = torch.exp(-(dist / 5.0e5) ** 2)
    qo = torch.zeros(5, om.K, N + 1, N + 1, N + 1, dtype=torch.float64)
    qo[4] = rho_b * thp                       # Theta' = rhobar theta' with rho' = 0
    q = gpu(to_nodes(qo))
    q1, q2 = lm.field(), lm.field()
    b0 = dg.dg_budgets(lm, PH, q)
    dt = 5.0
    for _ in range(5):
        dg.ssp_rk3_step(lm, PH, dt, q, q1, q2)
        qo = eu.ssp_rk3_step(op, dt, qo)
    torch.cuda.synchronize()
    b1 = dg.dg_budgets(lm, PH, q)
    bo = sp.budgets(op, qo)
    print("sphere budgets", b0, b1, bo, flush=True)
    assert abs(b1[0] - b0[0]) <= 1e-13 * abs(b0[1])
    for i in range(4):
        assert abs(b1[i] - bo[i]) <= 1e-12 * max(abs(bo[i]), abs(bo[1]) * (i == 0)), (i, b1[i], bo[i])
    assert_fields(q, to_nodes(qo), TOL_FP64, "sphere steps", vector_momentum=True)


def test_sphere_refusals():
    lm, _ = _meshes(3, 1, 1)
    q, r = lm.field(), lm.field()
    with pytest.raises(dg.DGError) as e:
        dg.dg_rhs(lm, dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, mu=1.5), q, r)
    assert e.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as e:
        dg.dg_indicator(lm, PH, q, dg.DG_IND_GRAD_THETA, 0.1)
    assert e.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as e:
        dg.dg_rhs(lm, dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, nonconforming=dg.DG_NC_POINTWISE), q, r)
    assert e.value.code == dg.DG_EUNSUPPORTED
