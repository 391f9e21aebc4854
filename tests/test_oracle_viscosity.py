"""Pins of the oracle's artificial viscosity (section 4.3 runs the rising bubble
with mu = 1.5 m^2/s; the operator div(mu grad q') on every perturbation variable,
discretised by the two-pass central scheme, is a reading).

What the mathematics fixes, independently of the code:
  * exactness: for a continuous field of degree <= N per axis on every leaf whose
    normal derivative vanishes on the walls, every face jump is zero and the
    result is mu times the Laplacian at the nodes, through hanging faces (this
    pins the volume terms and the mortar interpolation I_a);
  * conservation: the integral of R over the domain vanishes for any state, with
    walls (no diffusive flux), periodic wraps and mortars (pins the balance of
    the lifted terms between the two sides of every face and R_a's weights);
  * energy: on a conforming mesh, with the lumped quadrature and summation by
    parts, sum J W q.R = -mu sum J W |sigma|^2 to round-off for any state (pins
    the lift scale, the central averages and the wall treatment of both
    passes); on a mesh with hanging faces the sum is <= 0 (the identity there
    holds only up to the difference between the exact mortar mass and the
    lumped face mass, a few parts in a thousand);
  * consistency on a smooth periodic field: L2 error rate >= N - 1.5 between
    the two finest meshes, uniform and with hanging faces, N = 3, 4, 5.

Planted mistakes at the end: each must make at least one of these pins fail.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import forest as fo
from tests.test_oracle_euler import amr_mesh, rand_q

F64 = torch.float64
MU = 1.5


def _phys(mu=MU):
    return eu.Phys(g=0.0, background=eu.BG_CONSTANT, rho0=1.0, Theta0=300.0, mu=mu)


def _uniform(N, n, periodic, L=2.0):
    return fo.build(fo.ForestDesc(N, n, n, n, 2, (0.0, 0.0, 0.0), (L, L, L), periodic), None)


def _fsum(x):
    return math.fsum(x.reshape(-1).tolist())


def _sigma(op, q):
    """the gradient pass of the scheme, restated from its definition for the energy
    pin: sigma_d = (2/h_d) D_d q + the lifted central jump on the faces normal to d"""
    g2 = 2.0 / op.h
    dq = [torch.einsum('im,vekjm->vekji', op.D, q), torch.einsum('jm,vekmi->vekji', op.D, q),
          torch.einsum('km,vemji->vekji', op.D, q)]
    T = op._central_face_terms(q, lambda d: q, wall_zero_flux=False)
    return [g2[None, :, d, None, None, None] * dq[d] + T[d] for d in range(3)]


# ----------------------------------------------------------------------------- pins
def check_exact_polynomial(N=4, seed=4):
    """degree-4 bumps t^2 (2 - t)^2 on [0, 2]^3 (zero slope at both walls of every
    axis) combined per variable; the mesh has hanging faces"""
    m = amr_mesh(N, periodic=(0, 0, 0), seed=seed, hi=(2.0, 2.0, 2.0))
    op = eu.Operator(m, _phys())
    X, Y, Z = eu.node_xyz(m)

    def f(t):
        return t * t * (2 - t) ** 2

    def f2(t):
        return 12 * t * t - 24 * t + 8

    fx, fy, fz = f(X), f(Y), f(Z)
    q = torch.stack([fx, fy * fz, fx * fy * fz, fz + fx * fy, 3.0 + fy])
    lap = torch.stack([f2(X), f2(Y) * fz + fy * f2(Z), f2(X) * fy * fz + fx * f2(Y) * fz + fx * fy * f2(Z),
                       f2(Z) + f2(X) * fy + fx * f2(Y), f2(Y)])
    R = op.viscous(q)
    err = float((R - MU * lap).abs().max())
    # rounding of two differentiations: eps |q| (N^2 max 2/h)^2 times a modest constant
    amp = (N * N * float((2.0 / op.h).max())) ** 2
    bound = 64 * 2.2e-16 * MU * float(q.abs().max()) * amp
    print("exactness N=%d: error %.2e, rounding bound %.2e, |mu lap| %.1f" % (N, err, bound, float(MU * lap.abs().max())))
    assert err < bound, (err, bound)


def check_conservation(periodic, seed=3):
    m = amr_mesh(3, periodic=periodic, seed=seed, hi=(2.0, 2.0, 2.0))
    op = eu.Operator(m, _phys())
    q = rand_q(op, 7)
    R = op.viscous(q)
    JW = eu.quad_weights(op)
    for v in range(5):
        scale = float((JW * R[v].abs()).sum())
        assert abs(_fsum(JW * R[v])) < 1e-13 * scale, (v, _fsum(JW * R[v]), scale)


def check_energy_conforming(periodic, N=3, seed=2):
    m = _uniform(N, 3, periodic)
    op = eu.Operator(m, _phys())
    q = rand_q(op, seed)
    R = op.viscous(q)
    JW = eu.quad_weights(op)
    S = _sigma(op, q)
    for v in range(5):
        lhs = _fsum(JW * q[v] * R[v])
        rhs = -MU * _fsum(sum(JW * S[d][v] ** 2 for d in range(3)))
        assert abs(lhs - rhs) < 1e-12 * abs(rhs), (v, lhs, rhs)


def check_dissipative_amr(periodic, seed=5):
    m = amr_mesh(4, periodic=periodic, seed=seed, hi=(2.0, 2.0, 2.0))
    op = eu.Operator(m, _phys())
    q = rand_q(op, seed)
    R = op.viscous(q)
    JW = eu.quad_weights(op)
    S = _sigma(op, q)
    for v in range(5):
        lhs = _fsum(JW * q[v] * R[v])
        ref = -MU * _fsum(sum(JW * S[d][v] ** 2 for d in range(3)))
        assert lhs < 0.0, (v, lhs)
        assert abs(lhs - ref) < 1e-2 * abs(ref), (v, lhs, ref)


def _smooth_error(N, n, amr):
    L = 2.0
    desc = fo.ForestDesc(N, n, n, n, 2, (0.0, 0.0, 0.0), (L, L, L), (1, 1, 1))
    m = fo.build(desc, None)
    if amr:
        rng = np.random.default_rng(1)
        m = fo.build(desc, m, (rng.random(m.K) < 0.3).astype(np.int8), fo.PASS_REFINE)
        assert len(m.hang) > 0
    op = eu.Operator(m, _phys(1.0))
    X, Y, Z = eu.node_xyz(m)
    k = math.pi
    a = torch.sin(k * X) * torch.cos(k * Y) * torch.sin(k * Z + 0.3)
    b = torch.cos(k * X + 0.1) * torch.cos(k * Y)
    c = torch.sin(k * Z)
    q = torch.stack([a, 2 * a, b, c, a])
    lap = -k * k * torch.stack([3 * a, 6 * a, 2 * b, c, 3 * a])
    R = op.viscous(q)
    return math.sqrt(float((eu.quad_weights(op) * (R - lap) ** 2).sum()))


def check_consistency_rate(N, amr):
    e4, e8 = _smooth_error(N, 4, amr), _smooth_error(N, 8, amr)
    rate = math.log2(e4 / e8)
    assert rate >= N - 1.5, (N, amr, e4, e8, rate)


# ----------------------------------------------------------------------------- tests
def test_exact_for_polynomials_through_mortars():
    check_exact_polynomial(4)
    check_exact_polynomial(5, seed=6)


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 0, 1), (1, 1, 1)])
def test_conservation_walls_wraps_mortars(periodic):
    check_conservation(periodic)


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1)])
def test_energy_identity_conforming(periodic):
    check_energy_conforming(periodic)


@pytest.mark.parametrize("periodic", [(0, 0, 0), (0, 1, 1)])
def test_dissipative_with_hanging_faces(periodic):
    check_dissipative_amr(periodic)


@pytest.mark.parametrize("N,amr", [(3, False), (3, True), (4, True), (5, False)])
def test_consistency_rate(N, amr):
    check_consistency_rate(N, amr)


def test_zero_mu_adds_nothing():
    m = amr_mesh(3, seed=1, hi=(2.0, 2.0, 2.0))
    q = rand_q(eu.Operator(m, _phys(0.0)), 1)
    assert torch.equal(eu.Operator(m, _phys(0.0)).rhs(q), eu.Operator(m, eu.Phys(
        g=0.0, background=eu.BG_CONSTANT, rho0=1.0, Theta0=300.0)).rhs(q))
    op = eu.Operator(m, _phys())
    R = op.rhs(q) - eu.Operator(m, _phys(0.0)).rhs(q)
    assert float((R - op.viscous(q)).abs().max()) <= 1e-12 * float(op.viscous(q).abs().max())


# ----------------------------------------------------------------------------- planted mistakes
ORIG_TERMS = eu.Operator._central_face_terms
ORIG_INIT = eu.Operator.__init__


def _scale_pass(which, factor):
    """the lifted terms of one pass times factor: 0 drops them (the gradient pass:
    q* = q-), 2 turns the central average into the neighbour's value on
    conforming faces (and doubles the wall flux of the flux pass)"""
    def terms(self, X, sel, wall_zero_flux):
        T = ORIG_TERMS(self, X, sel, wall_zero_flux)
        return [t * factor for t in T] if wall_zero_flux == (which == "flux") else T
    return terms


def _no_wall_flux(self, X, sel, wall_zero_flux):
    return ORIG_TERMS(self, X, sel, False)


def _swap_interp(self, *a, **k):
    ORIG_INIT(self, *a, **k)
    self.I = [self.I[1], self.I[0]]


def _unscaled_projection(self, *a, **k):
    ORIG_INIT(self, *a, **k)
    self.Rm = [self.I[0].T.clone(), self.I[1].T.clone()]


MUTANTS = {
    "gradient pass without face terms": ("_central_face_terms", _scale_pass("grad", 0.0)),
    "flux pass one-sided": ("_central_face_terms", _scale_pass("flux", 2.0)),
    "gradient pass one-sided": ("_central_face_terms", _scale_pass("grad", 2.0)),
    "diffusive flux through walls": ("_central_face_terms", _no_wall_flux),
    "mortar interpolation of the wrong half": ("__init__", _swap_interp),
    "mortar projection by I_a^T": ("__init__", _unscaled_projection),
}


def _all_pins():
    check_exact_polynomial(4)
    for p in [(0, 0, 0), (1, 1, 1)]:
        check_conservation(p)
        check_energy_conforming(p)
    check_dissipative_amr((0, 0, 0))
    check_consistency_rate(3, True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(eu.Operator, attr, fn)
    with pytest.raises(AssertionError):
        _all_pins()
