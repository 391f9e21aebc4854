"""Pins of the oracle's refinement on the cubed-sphere shell (sections 3.1 and 3.3
on the curved elements of section 3.4), no GPU.

What the geometry and the definitions fix, independently of the code:
  * the face tables are closed: a conforming face points back, every fine face of a
    hanging row names its coarse leaf, face, quadrant and orientation, and the
    coarse face names its row; face neighbours differ by at most one level;
  * a fine face's nodes are the coarse face's mapping at the fine nodes' places in
    the recorded quadrant and orientation, up to the geometry's interpolation error;
  * refining every leaf once gives the cells of the unrefined shell with twice the
    resolution, and the operator on them is that shell's operator;
  * with hanging faces a rest state is exact, and the integrals of R_rho and
    R_Theta vanish to round-off (the mortars conserve mass and Theta);
  * for a smooth state, the right-hand side on fine leaves beside hanging faces is
    close to that on the uniformly refined shell (the mortar reads the coarse trace
    at the right places);
  * the transfers of a refinement pass keep the total mass exactly, those of a
    coarsening pass keep every family's J W integral of every field exactly, and a
    coarsening pass undoes a refinement pass on the leaves;
  * the shell's discrete adjoint (reverse-mode derivative of the operator, hanging
    faces included) and the transposed transfers of the passes agree with central
    differences of the operator and the transfers themselves, and
    the Gaussian theta vortex state has its stated amplitude, width and rest.
Planted mistakes at the end: each must make one of these fail.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd.synth import random_state

F64 = torch.float64


def _amr_mesh(N=3, n=2, nz=1, L=2, seed=1, frac=(0.3, 0.2)):
    d = sp.SphereDesc(N=N, n=n, nz=nz, max_level=L)
    m = sp.SphereMesh(d)
    rng = np.random.default_rng(seed)
    for fr in frac[:L]:
        m = sp.refine_pass(m, (rng.random(m.K) < fr).astype(int))
    return m


def _smooth_state(op):
    x = op.geo.x
    r = torch.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    q = torch.zeros(5, op.K, op.N + 1, op.N + 1, op.N + 1, dtype=F64)
    q[0] = 1e-3 * torch.exp(-((x[0] / r - 0.7) ** 2 + (x[1] / r - 0.5) ** 2) * 3.0) * torch.sin(
        math.pi * op.geo.height / op.mesh.desc.H)
    Om = (0.3e-5, -0.5e-5, 1.0e-5)
    q[1] = Om[1] * x[2] - Om[2] * x[1]
    q[2] = Om[2] * x[0] - Om[0] * x[2]
    q[3] = Om[0] * x[1] - Om[1] * x[0]
    q[4] = 600.0 * q[0]
    return q


# ----------------------------------------------------------------------------- pins
def check_tables(m=None):
    m = m or _amr_mesh()
    d = m.desc
    assert int((m.kind == sp.COARSE).sum()) == len(m.hang)
    assert int((m.kind == sp.FINE).sum()) == 4 * len(m.hang)
    for e in range(m.K):
        for f in range(6):
            k = int(m.kind[e, f])
            e2, f2, flip = (int(x) for x in m.nb[e, f])
            if k == sp.CONF:
                assert m.kind[e2, f2] == sp.CONF and tuple(int(x) for x in m.nb[e2, f2]) == (e, f, flip)
                assert m.leaves[e, 1] == m.leaves[e2, 1]
            elif k == sp.WALL:
                assert f >= 4
    for h, row in enumerate(m.hang):
        ec, fc = int(row[0]), int(row[1])
        assert m.kind[ec, fc] == sp.COARSE and int(m.nb[ec, fc, 0]) == h
        for quad in range(4):
            ef = int(row[2 + quad])
            ff = int(m.hang_ff[h])
            assert m.kind[ef, ff] == sp.FINE
            assert tuple(int(x) for x in m.nb[ef, ff]) == (ec, fc, int(m.hang_flip[h]))
            assert int(m.aux[ef, ff]) == quad
            assert m.leaves[ef, 1] == m.leaves[ec, 1] + 1
    # 2:1 across every face
    for e, lf in enumerate(map(tuple, m.leaves.tolist())):
        for f in range(6):
            got = sp.cell_neighbour(d, lf, f)
            if got is None:
                continue
            x = m.containing(got[0])
            assert x is None or lf[1] - x[1] <= 1


def check_hanging_geometry(N=4):
    m = _amr_mesh(N=N, n=2, nz=1, L=1, frac=(0.4,))
    op = sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL)
    g, re = op.geo, op.re
    I = [torch.as_tensor(M, dtype=F64) for M in re.I]
    err, width = 0.0, 0.5 * math.pi * m.desc.r_e / (2 * m.desc.n)
    assert len(m.hang) > 0
    for h, row in enumerate(m.hang):
        ec, fc, ff, flip = int(row[0]), int(row[1]), int(m.hang_ff[h]), int(m.hang_flip[h])
        perm = torch.as_tensor(sp.face_perm(N, flip))
        for quad in range(4):
            ef = int(row[2 + quad])
            for c in range(3):
                xc = eu.face_slice(g.x[c], fc, N)[ec]
                xm = eu.interp2(I[quad & 1], I[quad >> 1], xc, N)[perm]
                xf = eu.face_slice(g.x[c], ff, N)[ef]
                err = max(err, float((xf - xm).abs().max()))
    assert err <= 1e-3 * width, (err, width)


def check_refined_everywhere_is_the_finer_shell(N=3, n=2, nz=1, seed=4):
    d = sp.SphereDesc(N=N, n=n, nz=nz, max_level=1)
    m1 = sp.refine_pass(sp.SphereMesh(d), np.ones(6 * n * n * nz, dtype=int))
    mu = sp.SphereMesh(sp.SphereDesc(N=N, n=2 * n, nz=2 * nz))
    assert len(m1.hang) == 0 and m1.K == mu.K
    perm = np.array([mu.index[(p, 0, x, y, z)] for (p, _, x, y, z) in m1.leaves.tolist()])
    o1 = sp.SphereOperator(m1, eu.Phys(), sp.BG_ISOTHERMAL)
    ou = sp.SphereOperator(mu, eu.Phys(), sp.BG_ISOTHERMAL)
    for c in range(3):
        assert torch.equal(o1.geo.x[c], ou.geo.x[c][perm])
    q = torch.as_tensor(random_state(m1.K, N, seed), dtype=F64).reshape(5, m1.K, N + 1, N + 1, N + 1) * 0.1
    qu = torch.zeros_like(q)
    qu[:, perm] = q
    R1, Ru = o1.rhs(q), ou.rhs(qu)[:, perm]
    for v in range(5):
        assert float((R1[v] - Ru[v]).norm()) <= 1e-13 * float(Ru[v].norm()), v


def check_conservation_and_rest(N=3, seed=3):
    m = _amr_mesh(N=N)
    assert len(m.hang) > 0
    op = sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL)
    z = torch.zeros(5, m.K, N + 1, N + 1, N + 1, dtype=F64)
    assert float(op.rhs(z).abs().max()) == 0.0
    q = torch.as_tensor(random_state(m.K, N, seed), dtype=F64).reshape(5, m.K, N + 1, N + 1, N + 1) * 0.1
    R = op.rhs(q)
    JW = sp.quad_weights(op)
    for v in (0, 4):
        tot = math.fsum((JW * R[v]).reshape(-1).tolist())
        scale = float((JW * R[v].abs()).sum())
        assert abs(tot) <= 1e-14 * scale, (v, tot, scale)


def check_smooth_consistency(N=4):
    d = sp.SphereDesc(N=N, n=2, nz=1, max_level=1)
    m0 = sp.SphereMesh(d)
    fl = np.zeros(m0.K, dtype=int)
    fl[[0, 1, 5, 9, 14]] = 1
    ma, mf = sp.refine_pass(m0, fl), sp.refine_pass(m0, np.ones(m0.K, dtype=int))
    oa = sp.SphereOperator(ma, eu.Phys(), sp.BG_ISOTHERMAL)
    of = sp.SphereOperator(mf, eu.Phys(), sp.BG_ISOTHERMAL)
    Ra, Rf = oa.rhs(_smooth_state(oa)), of.rhs(_smooth_state(of))
    fine = sorted(set(int(x) for x in ma.hang[:, 2:].reshape(-1)))
    idx = [mf.index[tuple(ma.leaves[e].tolist())] for e in fine]
    for v in range(5):
        a, b = Ra[v][fine], Rf[v][idx]
        # measured 5e-5 .. 1e-4 (N = 4, elements of about 5000 km)
        assert float((a - b).norm()) <= 2e-3 * float(b.norm()), v


def check_adapt_transfers(N=3, seed=6):
    d = sp.SphereDesc(N=N, n=2, nz=1, max_level=1)
    m0 = sp.SphereMesh(d)
    fl = np.zeros(m0.K, dtype=int)
    fl[[0, 3, 7, 12, 20]] = 1
    m1 = sp.refine_pass(m0, fl)
    o0, o1 = (sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL) for m in (m0, m1))
    q0 = torch.as_tensor(random_state(m0.K, N, seed), dtype=F64).reshape(5, m0.K, N + 1, N + 1, N + 1) * 0.1
    q1, s = sp.adapt_project(o0, o1, q0)
    M0, M1 = sp.budgets(o0, q0)[1], sp.budgets(o1, q1)[1]
    assert abs(M1 - M0) <= 2e-16 * M0 and 0.0 < abs(s - 1.0) < 1e-3
    # coarsening every refined family back: the leaves return, the means balance
    back = -np.ones(m1.K, dtype=int)
    m2 = sp.coarsen_pass(m1, back)
    assert np.array_equal(m2.leaves, m0.leaves)
    o2 = sp.SphereOperator(m2, eu.Phys(), sp.BG_ISOTHERMAL)
    q2, s2 = sp.adapt_project(o1, o2, q1)
    assert s2 == 1.0
    JW1, JW2 = sp.quad_weights(o1), sp.quad_weights(o2)
    full1 = [o1.bg[0] + q1[0], q1[1], q1[2], q1[3], o1.bg[1] + q1[4]]
    full2 = [o2.bg[0] + q2[0], q2[1], q2[2], q2[3], o2.bg[1] + q2[4]]
    for e in range(m2.K):
        if m2.xfer_kind[e] != 8:
            assert torch.equal(q2[:, e], q1[:, int(m2.xfer_src[e])])
            continue
        fam = torch.arange(int(m2.xfer_src[e]), int(m2.xfer_src[e]) + 8)
        for v in range(5):
            inside = math.fsum((JW1[fam] * full1[v][fam]).reshape(-1).tolist())
            scale = math.fsum((JW1[fam] * full1[v][fam].abs()).reshape(-1).tolist())
            assert abs(math.fsum((JW2[e] * full2[v][e]).reshape(-1).tolist()) - inside) <= 1e-14 * scale
    M2 = sp.budgets(o2, q2)[1]
    assert abs(M2 - M1) <= 2e-16 * M1


# ----------------------------------------------------------------------------- tests
def test_tables_closed_and_balanced():
    check_tables()
    check_tables(_amr_mesh(N=2, n=1, nz=2, L=2, seed=9, frac=(0.5, 0.3)))


def test_hanging_face_geometry():
    check_hanging_geometry()


def test_refined_everywhere_is_the_finer_shell():
    check_refined_everywhere_is_the_finer_shell()


def test_conservation_and_rest_with_hanging_faces():
    check_conservation_and_rest()


def test_smooth_consistency_at_hanging_faces():
    check_smooth_consistency()


def test_transfers_of_the_passes():
    check_adapt_transfers()


def test_transfer_adjoint_against_central_differences():
    """adapt_project_adjoint (reverse mode through the transfer, the refinement's
    scale factor included) against central differences of adapt_project itself,
    for a refine pass and the coarsen pass that undoes it"""
    N = 2
    m = sp.SphereMesh(sp.SphereDesc(N=N, n=1, nz=1, max_level=2))
    m = sp.refine_pass(m, (np.arange(m.K) % 2 == 0).astype(np.int8))
    m2 = sp.refine_pass(m, (np.arange(m.K) % 3 == 1).astype(np.int8))
    m3 = sp.coarsen_pass(m2, -np.ones(m2.K, dtype=np.int8))
    o1, o2, o3 = (sp.SphereOperator(x, eu.Phys(), sp.BG_ISOTHERMAL) for x in (m, m2, m3))
    shape = lambda K: (5, K, N + 1, N + 1, N + 1)
    q = torch.as_tensor(random_state(m.K, N, 71)).reshape(shape(m.K)) * 0.1 + sp.acoustic_state(o1)
    for oa, ob, x in ((o1, o2, q), (o2, o3, sp.adapt_project(o1, o2, q)[0])):
        gb = torch.as_tensor(random_state(ob.K, N, 72)).reshape(shape(ob.K))
        v = torch.as_tensor(random_state(oa.K, N, 73)).reshape(shape(oa.K))
        ad = float((sp.adapt_project_adjoint(oa, ob, x, gb) * v).sum())
        eps = 1e-4
        fd = float((gb * (sp.adapt_project(oa, ob, x + eps * v)[0] - sp.adapt_project(oa, ob, x - eps * v)[0])).sum())
        fd /= 2 * eps
        assert abs(ad - fd) <= 1e-8 * abs(ad), (ad, fd)
    # the value of the transfer is unchanged by the derivative path
    a0, s0 = sp.adapt_project(o1, o2, q)
    a1, s1 = sp.adapt_project(o1, o2, q.clone().requires_grad_(True))
    assert torch.equal(a0, a1.detach()) and s0 == float(s1)


def test_shell_adjoint_against_central_differences():
    """<rhs_adjoint(q, lam), v> against <lam, (R(q + eps v) - R(q - eps v)) / (2 eps)>
    on a refined shell with hanging faces: the transposed derivative the library's
    shell adjoint is compared with, pinned by the operator alone"""
    N = 2
    m = sp.SphereMesh(sp.SphereDesc(N=N, n=1, nz=1, max_level=1))
    m = sp.refine_pass(m, (np.arange(m.K) % 3 == 0).astype(np.int8))
    assert len(m.hang) > 0
    op = sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL)
    shape = (5, m.K, N + 1, N + 1, N + 1)
    q = torch.as_tensor(random_state(m.K, N, 31)).reshape(shape) * 0.1 + sp.vortex_state(op, width=2.0e6)
    lam = torch.as_tensor(random_state(m.K, N, 32)).reshape(shape)
    v = torch.as_tensor(random_state(m.K, N, 33)).reshape(shape)
    ad = float((eu.rhs_adjoint(op, q, lam) * v).sum())
    eps = 1e-5
    fd = float((lam * (op.rhs(q + eps * v) - op.rhs(q - eps * v))).sum()) / (2 * eps)
    assert abs(ad - fd) <= 1e-7 * abs(ad), (ad, fd)


def test_shell_adjoint_at_rest_richardson():
    """At a state at rest (the vortex: u = 0 at every node) the Rusanov wave speed's
    |u.n| sits on its kink at every face node: the reverse mode differentiates it
    as 0 there and central differences see it symmetric, but where the kink meets a
    jump (a wall's mirror state, whose normal momentum jumps by 2 U.n under the
    perturbation) the central difference is off by a term linear in eps.  The gap
    halves with eps, and Richardson extrapolation 2 D(eps/2) - D(eps) agrees with
    the reverse mode far below the plain difference's gap."""
    N = 2
    m = sp.SphereMesh(sp.SphereDesc(N=N, n=1, nz=1, max_level=1))
    m = sp.refine_pass(m, (np.arange(m.K) % 3 == 0).astype(np.int8))
    op = sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL)
    shape = (5, m.K, N + 1, N + 1, N + 1)
    q = sp.vortex_state(op, width=2.0e6)
    assert float(q[1:4].abs().max()) == 0.0
    lam = torch.as_tensor(random_state(m.K, N, 34)).reshape(shape)
    v = torch.as_tensor(random_state(m.K, N, 35)).reshape(shape)
    ad = float((eu.rhs_adjoint(op, q, lam) * v).sum())

    def central(eps):
        return float((lam * (op.rhs(q + eps * v) - op.rhs(q - eps * v))).sum()) / (2 * eps)

    d1, d2 = central(1e-3), central(5e-4)
    g1, g2 = abs(d1 - ad), abs(d2 - ad)
    rich = abs(2 * d2 - d1 - ad)
    print("rest-state dot-product gaps: eps 1e-3", g1 / abs(ad), "eps 5e-4", g2 / abs(ad), "Richardson",
          rich / abs(ad), flush=True)
    assert 1.8 < g1 / g2 < 2.2
    assert rich <= 1e-3 * g2 and rich <= 1e-9 * abs(ad)


def test_vortex_state():
    """theta' = Theta'/rhobar is 1 K times exp(-(d / w)^2) in the great-circle distance
    d from the centre, rho' and the momentum vanish"""
    m = sp.SphereMesh(sp.SphereDesc(N=3, n=4, nz=1))
    op = sp.SphereOperator(m, eu.Phys(), sp.BG_ISOTHERMAL)
    q = sp.vortex_state(op, amp=1.0, width=5.0e5, lon=0.5, lat=0.2)
    assert float(q[:4].abs().max()) == 0.0
    thp = q[4] / op.bg[0]
    c = (math.cos(0.2) * math.cos(0.5), math.cos(0.2) * math.sin(0.5), math.sin(0.2))
    x = [op.geo.x[k] / (6.371e6 + op.geo.height) for k in range(3)]
    chord = torch.sqrt((x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2 + (x[2] - c[2]) ** 2)
    d = 2.0 * 6.371e6 * torch.arcsin(0.5 * chord)
    assert float((thp - torch.exp(-(d / 5.0e5) ** 2)).abs().max()) <= 1e-12
    assert 0.0 < float(thp.max()) <= 1.0


# ----------------------------------------------------------------------------- planted mistakes
ORIG_MORT = sp.SphereOperator.mortars


def _unflipped_mortar(mp):
    """the coarse trace read in the coarse face's order on every fine face (the
    orientation across a panel edge ignored by the mortars)"""
    orig = sp.SphereMesh._tables

    def tables(self):
        orig(self)
        self.hang_flip = np.zeros_like(self.hang_flip)
    mp.setattr(sp.SphereMesh, "_tables", tables)


def _scaled_projection(fac):
    def mortars(self, q, Ft):
        re = self.re
        saved = re.R
        re.R = [fac * M for M in saved]
        try:
            return ORIG_MORT(self, q, Ft)
        finally:
            re.R = saved
    return mortars


def _quadrants_swapped(mp):
    """the fine leaves of a hanging row taken in the order of the fine face's own
    axes instead of the coarse face's"""
    orig = sp.SphereMesh._tables

    def tables(self):
        orig(self)
        for h in range(len(self.hang)):
            if self.hang_flip[h]:
                r = self.hang[h].copy()
                self.hang[h, 2:] = r[[3, 2, 5, 4]]
    mp.setattr(sp.SphereMesh, "_tables", tables)


MUTANTS = {
    "orientation ignored on the mortars": (_unflipped_mortar, check_smooth_consistency),
    "coarse flux per fine reference area (the factor 4 dropped)": (
        lambda mp: mp.setattr(sp.SphereOperator, "mortars", _scaled_projection(0.25)), check_conservation_and_rest),
    "quadrants in the fine face's axes": (_quadrants_swapped, check_hanging_geometry),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    plant, check = MUTANTS[name]
    plant(monkeypatch)
    with pytest.raises(AssertionError):
        check()


# ----------------------------------------------------------------------------- library host side
def _lib_available():
    try:
        from paper_2404_16648_amd import dg
        dg.lib()
        return True
    except RuntimeError:
        return False


def _tables_match(lm, om):
    from paper_2404_16648_amd import dg
    t = lm.tables()
    assert np.array_equal(t["leaf"], om.leaves.astype(np.int32))
    assert np.array_equal(dg.dg_sphere_faces(lm), om.nb.astype(np.int32))
    assert np.array_equal(dg.dg_sphere_face_kinds(lm), (om.kind + 4 * om.aux).astype(np.int32))
    assert np.array_equal(t["hang"], om.hang.astype(np.int32))
    assert np.array_equal(t["xfer_src"], om.xfer_src.astype(np.int32))
    assert np.array_equal(t["xfer_kind"], om.xfer_kind.astype(np.int32))


@pytest.mark.skipif(not _lib_available(), reason="library not built")
@pytest.mark.parametrize("N,n,nz,L,seed", [(3, 2, 1, 2, 1), (2, 1, 2, 3, 2), (4, 3, 1, 1, 3)])
def test_library_passes_match_the_oracle(N, n, nz, L, seed):
    """random refine and coarsen flag sequences applied by the library's forest and
    the oracle's: bit-exact leaves, face tables, hanging rows and transfer plans,
    and dg_pass_changes against what each pass builds"""
    from paper_2404_16648_amd import dg
    lm = dg.dg_sphere_mesh_build(N, n, nz, host_only=True, max_level=L)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz, max_level=L))
    _tables_match(lm, om)
    rng = np.random.default_rng(seed)
    for step in range(5):
        refine = step % 3 != 2
        fl = np.where(rng.random(om.K) < (0.3 if refine else 0.7), 1 if refine else -1, 0).astype(np.int8)
        p = dg.DG_PASS_REFINE if refine else dg.DG_PASS_COARSEN
        changes = dg.dg_pass_changes(lm, fl, p)
        lm2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=p)
        om2 = sp.refine_pass(om, fl) if refine else sp.coarsen_pass(om, fl)
        _tables_match(lm2, om2)
        assert changes == (not np.array_equal(om2.leaves, om.leaves) or om2.K != om.K)
        lm, om = lm2, om2
    assert len(om.hang) > 0


@pytest.mark.skipif(not _lib_available(), reason="library not built")
def test_library_geometry_of_a_refined_shell():
    from paper_2404_16648_amd import dg
    N = 3
    lm = dg.dg_sphere_mesh_build(N, 2, 1, host_only=True, max_level=2)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=2, nz=1, max_level=2))
    rng = np.random.default_rng(5)
    for _ in range(2):
        fl = (rng.random(om.K) < 0.3).astype(np.int8)
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = sp.refine_pass(om, fl)
    _tables_match(lm, om)
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
    vol, (v_disc, v_exc) = dg.dg_sphere_volumes(lm)
    assert np.abs(vol - sp.element_volumes(om)).max() <= 1e-13 * vol.max()


@pytest.mark.skipif(not _lib_available(), reason="library not built")
def test_library_level_zero_tables_two_ways():
    """the unrefined shell's connectivity from the lattice matching (max_level 0)
    and from the forest's neighbour search (max_level 1) are the same"""
    from paper_2404_16648_amd import dg
    a = dg.dg_sphere_mesh_build(3, 3, 2, host_only=True)
    b = dg.dg_sphere_mesh_build(3, 3, 2, host_only=True, max_level=1)
    assert np.array_equal(dg.dg_sphere_faces(a), dg.dg_sphere_faces(b))
    assert np.array_equal(dg.dg_sphere_face_kinds(a), dg.dg_sphere_face_kinds(b))
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(prev=a, flags=np.ones(a.K, np.int8), pass_=dg.DG_PASS_REFINE)
    assert e.value.code == dg.DG_EUNSUPPORTED
