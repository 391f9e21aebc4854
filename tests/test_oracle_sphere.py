"""Pins of the oracle's cubed-sphere shell (sections 3.4 and 4.4) and the library's
host tables and geometry against it (no GPU).

What the geometry and the physics fix, independently of the code:
  * the connectivity is closed and symmetric: every lateral face meets exactly one
    face, the relation is an involution, and the two sides' face nodes are the
    same points, bitwise, through the recorded orientation;
  * the discrete metric identities sum_i D_i (J a^i)_n = 0 hold to rounding (the
    curl form), and a uniform flow stays uniform through the volume and interior
    face terms;
  * the quadrature of J approaches the shell volume spectrally, and the spherical
    excess of the element footprints sums to the sphere's area exactly;
  * the isothermal background is hydrostatic in closed form, with the sound speed
    of section 4.4 (347.3 m/s at 300 K) at every height;
  * a rest state has a right-hand side of exactly zero; a uniform density
    perturbation at rest feels exactly -rho' g r_hat; the integral of R_rho and of
    R_Theta over the shell vanishes with walls at top and bottom (conservation);
  * the residual of a solid-body rotation (a steady divergence-free flow) falls as
    the panels are refined.
Planted mistakes at the end: each must make one of these fail.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state

F64 = torch.float64


def _op(N, n, nz, kind=sp.BG_ISOTHERMAL, ph=None):
    m = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz))
    return sp.SphereOperator(m, ph or eu.Phys(), kind)


def _fsum(t):
    return math.fsum(t.reshape(-1).tolist())


# ----------------------------------------------------------------------------- pins
def check_connectivity(n=3, nz=2):
    m = sp.SphereMesh(sp.SphereDesc(N=3, n=n, nz=nz))
    assert int((m.nb[:, :, 0] < 0).sum()) == 2 * 6 * n * n        # bottom and top walls
    for e in range(m.K):
        for f in range(6):
            e2, f2, flip = (int(x) for x in m.nb[e, f])
            if e2 < 0:
                assert f in (4, 5)
                continue
            assert tuple(int(x) for x in m.nb[e2, f2]) == (e, f, flip)


def check_face_points(N=4, n=2, nz=2):
    op = _op(N, n, nz)
    g, m = op.geo, op.mesh
    for e in range(m.K):
        for f in range(6):
            e2, f2, flip = (int(x) for x in m.nb[e, f])
            if e2 < 0:
                continue
            perm = torch.as_tensor(sp.face_perm(N, flip))
            for c in range(3):
                a = eu.face_slice(g.x[c], f, N)[e]
                b = eu.face_slice(g.x[c], f2, N)[e2][perm]
                assert torch.equal(a, b), (e, f, c)


def check_metric_identities(N=4, n=2, nz=2):
    g = _op(N, n, nz).geo
    for c in range(3):
        div = g.dxi(g.Ja[0][c], 0) + g.dxi(g.Ja[1][c], 1) + g.dxi(g.Ja[2][c], 2)
        scale = max(float(g.Ja[i][c].abs().max()) for i in range(3))
        assert float(div.abs().max()) <= 1e-11 * scale, (c, float(div.abs().max()), scale)


def check_free_stream(N=4, n=2, nz=2):
    op = _op(N, n, nz, sp.BG_CONSTANT, eu.Phys(g=0.0))
    q = torch.zeros(5, op.K, N + 1, N + 1, N + 1, dtype=F64)
    q[1], q[2], q[3] = 10.0, -3.0, 5.0
    R = op.volume(q) + op.surface(q, walls=False)
    Ft = op.contravariant(q)
    scale = max(float((f.abs() / op.geo.J[None]).max()) for f in Ft) * N * N
    assert float(R.abs().max()) <= 1e-13 * scale, (float(R.abs().max()), scale)


def check_rest_and_buoyancy(N=3, n=2, nz=2):
    op = _op(N, n, nz)
    q = torch.zeros(5, op.K, N + 1, N + 1, N + 1, dtype=F64)
    assert float(op.rhs(q).abs().max()) == 0.0
    eps = 1e-3
    q[0] = eps
    R = op.rhs(q)
    g = op.phys.g
    for c in range(3):
        ref = -eps * g * op.geo.rhat[c]
        assert float((R[1 + c] - ref).abs().max()) <= 1e-15 * eps * g, c
    assert float(R[0].abs().max()) == 0.0 and float(R[4].abs().max()) == 0.0


def check_conservation(N=3, n=2, nz=2, seed=3):
    op = _op(N, n, nz)
    q = torch.as_tensor(random_state(op.K, N, seed), dtype=F64).reshape(5, op.K, N + 1, N + 1, N + 1) * 0.1
    R = op.rhs(q)
    JW = sp.quad_weights(op)
    for v in (0, 4):
        tot, scale = _fsum(JW * R[v]), float((JW * R[v].abs()).sum())
        assert abs(tot) <= 1e-14 * scale, (v, tot, scale)


def _rotation_residual(N, n):
    op = _op(N, n, 1, sp.BG_CONSTANT, eu.Phys(g=0.0))
    x = op.geo.x
    Om = (0.3e-5, -0.5e-5, 1.0e-5)
    q = torch.zeros(5, op.K, N + 1, N + 1, N + 1, dtype=F64)
    q[1] = Om[1] * x[2] - Om[2] * x[1]
    q[2] = Om[2] * x[0] - Om[0] * x[2]
    q[3] = Om[0] * x[1] - Om[1] * x[0]
    return float(op.rhs(q)[0].abs().max())


def check_rotation_converges(N=4):
    r2, r4 = _rotation_residual(N, 2), _rotation_residual(N, 4)
    assert r4 <= r2 / 4.0, (r2, r4)


# ----------------------------------------------------------------------------- tests
def test_connectivity_closed_and_symmetric():
    check_connectivity()
    check_connectivity(n=1, nz=1)


def test_face_points_bitwise_through_orientation():
    check_face_points()


def test_metric_identities():
    check_metric_identities()
    check_metric_identities(N=5, n=1, nz=2)


def test_free_stream_through_volume_and_interior_faces():
    check_free_stream()


def test_volume_converges_and_areas_exact():
    errs = []
    for N in (2, 3, 4, 5):
        op = _op(N, 2, 1)
        d = op.mesh.desc
        V = _fsum(sp.quad_weights(op))
        Vex = 4.0 / 3.0 * math.pi * ((d.r_e + d.H) ** 3 - d.r_e ** 3)
        errs.append(abs(V - Vex) / Vex)
    assert errs[-1] < 1e-8 and all(errs[i + 1] < errs[i] for i in range(3)), errs
    m = sp.SphereMesh(sp.SphereDesc(N=3, n=3, nz=2))
    A = sp.element_areas(m, m.desc.r_e)
    layer = m.leaves[:, 4] == 0
    assert abs(math.fsum(A[layer]) - 4.0 * math.pi * m.desc.r_e ** 2) <= 1e-14 * 4.0 * math.pi * m.desc.r_e ** 2


def test_isothermal_background_closed_form():
    op = _op(3, 1, 2)
    ph = op.phys
    rho, Th, P = op.bg
    h = op.geo.height
    R, T0 = ph.R, ph.theta0
    # hydrostatic: dP/dh = -rho g, with P = P0 exp(-g h / (R T0))
    dPdh = -ph.g / (R * T0) * P
    assert float((dPdh + rho * ph.g).abs().max()) <= 1e-15 * float(P.max())
    # equation of state and the sound speed of section 4.4 at every height
    assert float((P - ph.P0 * (R * Th / ph.P0) ** ph.gamma).abs().max()) <= 1e-12 * float(P.max())
    c = torch.sqrt(ph.gamma * P / rho)
    assert float((c - 347.3).abs().max()) < 0.05


def test_rest_state_and_buoyancy_exact():
    check_rest_and_buoyancy()


def test_conservation_with_walls():
    check_conservation()


def test_rotation_residual_falls_with_refinement():
    check_rotation_converges()


# ----------------------------------------------------------------------------- library host side
def _lib_available():
    try:
        dg.lib()
        return True
    except RuntimeError:
        return False


@pytest.mark.skipif(not _lib_available(), reason="library not built")
@pytest.mark.parametrize("N,n,nz", [(2, 1, 3), (3, 2, 2), (4, 3, 1), (5, 2, 1)])
def test_library_tables_and_geometry_match(N, n, nz):
    lm = dg.dg_sphere_mesh_build(N, n, nz, host_only=True)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz))
    assert np.array_equal(dg.dg_sphere_faces(lm), om.nb.astype(np.int32))
    assert np.array_equal(lm.tables()["leaf"], om.leaves.astype(np.int32))
    metric, fgeo, c1d = dg.dg_sphere_geometry(lm)
    g = sp.SphereGeometry(om)
    J = g.J.reshape(om.K, -1).numpy()
    assert np.abs(metric[0] - J).max() <= 1e-13 * np.abs(J).max()
    for i in range(3):
        row = max(np.abs(g.Ja[i][c].numpy()).max() for c in range(3))
        for c in range(3):
            assert np.abs(metric[1 + 3 * i + c] - g.Ja[i][c].reshape(om.K, -1).numpy()).max() <= 1e-13 * row
    assert np.abs(fgeo[..., :3] - g.nrm.permute(1, 2, 3, 0).numpy()).max() <= 1e-13
    assert np.abs(fgeo[..., 3] - g.sJ.numpy()).max() <= 1e-13 * g.sJ.numpy().max()
    assert np.array_equal(c1d[2], g.h1)


@pytest.mark.skipif(not _lib_available(), reason="library not built")
def test_library_refuses_shell_refinement_and_high_order():
    lm = dg.dg_sphere_mesh_build(3, 1, 1, host_only=True)
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(prev=lm, flags=np.zeros(lm.K, np.int8), pass_=dg.DG_PASS_REFINE)
    assert e.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as e:
        dg.dg_sphere_mesh_build(6, 1, 1, host_only=True)
    assert e.value.code == dg.DG_EINVAL


# ----------------------------------------------------------------------------- planted mistakes
ORIG_GEO = sp.SphereGeometry.__init__
ORIG_SURF = sp.SphereOperator.surface
ORIG_PERM = sp.face_perm
ORIG_VOL = sp.SphereOperator.volume


def _cross_product_metrics(self, mesh):
    """J a^i from cross products of the interpolated tangent vectors instead of the
    curl form"""
    ORIG_GEO(self, mesh)
    dX = [[self.dxi(self.x[c], d) for d in range(3)] for c in range(3)]
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        a = [dX[c][j] for c in range(3)]
        b = [dX[c][k] for c in range(3)]
        self.Ja[i] = [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _no_flip(N, flip):
    return ORIG_PERM(N, 0)


def _buoyancy_sign(self, q):
    R = ORIG_VOL(self, q)
    g = self.phys.g
    for c in range(3):
        R[1 + c] = R[1 + c] + 2.0 * q[0] * g * self.geo.rhat[c]
    return R


def _all_pins():
    check_connectivity()
    check_face_points()
    check_metric_identities()
    check_free_stream()
    check_rest_and_buoyancy()
    check_conservation()


MUTANTS = {
    "cross-product metric terms": ("SphereGeometry", "__init__", _cross_product_metrics),
    "orientation of panel edges ignored": (None, "face_perm", _no_flip),
    "buoyancy sign": ("SphereOperator", "volume", _buoyancy_sign),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    cls, attr, fn = MUTANTS[name]
    monkeypatch.setattr(getattr(sp, cls) if cls else sp, attr, fn)
    with pytest.raises(AssertionError):
        _all_pins()
