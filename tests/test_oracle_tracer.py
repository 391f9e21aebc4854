"""Pins of the oracle's passive tracer (section 2.1's fourth equation,
dC/dt + div(C u) = 0 with C = rho c, advected by the Euler state's velocity):

  * with c = 1 (C = rho) and c = theta (C = Theta) the tracer right-hand side is
    the Euler operator's right-hand side of rho' and Theta' (pinned by
    test_oracle_physics.py), through walls, periodic wraps and hanging faces, with
    mortars and with pointwise matching (background constant in z, so that the
    full and the perturbation forms interpolate alike on mortars);
  * the mortars conserve the tracer's integral to round-off, pointwise matching
    does not (section 3.3's comparison, section 4.2's tracer loss);
  * a uniform free stream carries a constant tracer unchanged, and a smooth
    tracer profile in a uniform flow has R_C -> -u . grad C at the design rate on
    a mesh with hanging faces.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from tests.test_oracle_euler import amr_mesh, rand_q

F64 = torch.float64


@pytest.mark.parametrize("nc", ["mortar", "pointwise"])
@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 0, 1)])
def test_tracer_with_c_one_and_c_theta_is_mass_and_theta(nc, periodic):
    m = amr_mesh(3, periodic=periodic, seed=3)
    op = eu.Operator(m, eu.Phys(g=0.0), nonconforming=nc)
    q = rand_q(op, 5)
    R = op.rhs(q)
    for C, v in ((op.bg[0] + q[0], 0), (op.bg[1] + q[4], 4)):
        Rc = eu.tracer_rhs(op, q, C)
        assert float((Rc - R[v]).abs().max()) <= 1e-12 * float(R[v].abs().max()), (nc, v)


def test_tracer_conservation_mortar_not_pointwise():
    m = amr_mesh(3, periodic=(1, 0, 0), seed=7)
    C = None
    for nc in ("mortar", "pointwise"):
        op = eu.Operator(m, eu.Phys(), nonconforming=nc)
        q = rand_q(op, 8)
        if C is None:
            C = torch.as_tensor(np.random.default_rng(9).random(q[0].shape))
        Rc = eu.tracer_rhs(op, q, C)
        JW = eu.quad_weights(op)
        tot = math.fsum((JW * Rc).reshape(-1).tolist())
        scale = float((JW * Rc.abs()).sum())
        if nc == "mortar":
            assert abs(tot) < 1e-13 * scale, tot / scale
        else:
            assert abs(tot) > 1e-6 * scale, tot / scale


def test_tracer_free_stream_and_rest():
    m = amr_mesh(3, periodic=(1, 1, 1), seed=2)
    ph = eu.Phys(g=0.0, background=eu.BG_CONSTANT, rho0=1.2, Theta0=360.0)
    op = eu.Operator(m, ph)
    q = torch.zeros(5, m.K, 4, 4, 4, dtype=F64)
    C = torch.full_like(q[0], 0.7)
    # at rest: zero up to the rounding of the mortar interpolation of a constant
    # (lambda ~ 380 m/s, lift ~ 0.05 / m)
    assert float(eu.tracer_rhs(op, q, C).abs().max()) < 1e-13 * 0.7 * 380.0 * 0.05 * 10
    q[1], q[2], q[3] = 12.0, -7.0, 3.0
    assert float(eu.tracer_rhs(op, q, C).abs().max()) < 1e-13 * 0.7 * 12.0 / 250.0 * 10


def _advection_error(n, N):
    L = 1.0
    desc = fo.ForestDesc(N, n, n, n, 1, (0.0, 0.0, 0.0), (L, L, L), (1, 1, 1))
    m = fo.build(desc, None)
    lo, hh = fo.elem_lo_h(m)
    fl = np.all(lo + 0.5 * hh < L / 2, axis=1).astype(np.int8)   # one octant refined: hanging faces
    m = fo.build(desc, m, fl, fo.PASS_REFINE)
    ph = eu.Phys(cp=3.5, cv=2.5, P0=1.0, g=0.0, background=eu.BG_CONSTANT, rho0=1.0, Theta0=1.0)
    op = eu.Operator(m, ph)
    X, Y, Z = eu.node_xyz(m)
    u0 = (0.6, -0.3, 0.2)
    q = torch.zeros(5, *X.shape, dtype=F64)
    for d in range(3):
        q[1 + d] = u0[d]
    k = 2 * math.pi / L
    C = 1.0 + 0.5 * torch.sin(k * X) * torch.cos(k * Y + 0.4) * torch.sin(k * Z + 1.0)
    dC = (0.5 * k * torch.cos(k * X) * torch.cos(k * Y + 0.4) * torch.sin(k * Z + 1.0) * u0[0]
          - 0.5 * k * torch.sin(k * X) * torch.sin(k * Y + 0.4) * torch.sin(k * Z + 1.0) * u0[1]
          + 0.5 * k * torch.sin(k * X) * torch.cos(k * Y + 0.4) * torch.cos(k * Z + 1.0) * u0[2])
    return float((eu.tracer_rhs(op, q, C) + dC).abs().max()), len(m.hang)


def test_tracer_advection_design_order_with_hanging_faces():
    """R_C of a smooth tracer in a uniform flow (constant density, g = 0: the Euler
    state is a free stream) against -u . grad C, on meshes with one octant refined."""
    N = 4
    res = [_advection_error(n, N) for n in (2, 4, 8)]
    assert all(r[1] > 0 for r in res)
    rates = [math.log2(res[i][0] / res[i + 1][0]) for i in range(2)]
    assert rates[-1] > N - 0.5, (res, rates)
