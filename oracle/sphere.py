"""Oracle: compressible Euler on a cubed-sphere shell with curvilinear elements
(test infrastructure only).

Written from the paper's statements on spherical geometry (section 3.4) and its
global tests (section 4.4), with the same perturbation form, Rusanov flux and
strong-form dGSEM as the box operator in ``euler.py``:

* Grid: the cubed sphere of six panels, each split into n x n elements along
  the two equiangular panel coordinates and nz layers along the radius between
  r_e and r_e + H; elements are isoparametric (the mapping is interpolated by
  the same LGL polynomials as the fields, section 4.4).
* Curvilinear strong form: with x(xi) the element mapping, J its Jacobian and
  J a^i the contravariant metric terms, dq/dt = -(1/J) sum_i d/dxi_i (J a^i . F)
  + S - (1/(J w_N)) (s F*(n) - J a^d . F(q-) sgn) at face nodes, s = |J a^d| the
  face Jacobian and n the unit outward normal.
* Radial gravity: the buoyancy is -rho' g r_hat on the momentum; the background
  is hydrostatic in the height h = |x| - r_e (neutral, isothermal or constant).

Readings where the paper is silent (listed in the design notes):

* Equiangular gnomonic panels: a panel point is the cube point (1, tan a, tan b)
  rotated to the panel, normalised to radius r.
* Metric terms in the conservative curl form of Kopriva (2006), so the discrete
  divergence of the metric terms vanishes and a uniform flow stays uniform up to
  rounding: (J a^i)_n = -(curl_xi (X_l grad_xi X_m))_i with (n, m, l) cyclic, X
  the interpolated coordinates, X_l relative to the element's first node.
* The face normal and face Jacobian of a face shared by two elements are taken
  from the element with the smaller (leaf, face) pair, and its neighbour uses
  the same values with the normal reversed (both see bitwise-opposite normals).
* Walls at r_e and r_e + H: mirror state (rho', U - 2 (U.n) n, Theta').
* Isothermal background at T0: Pbar = P0 exp(-g h / (R T0)), rhobar = Pbar/(R T0),
  Thetabar from the equation of state.

Elements are ordered panel, layer, row, column: e = ((p nz + ir) n + ib) n + ia.
Local axes: xi along the panel's first coordinate, eta along the second, zeta
outward (every panel frame is right-handed, so J > 0).  Fields are [5, K, N+1,
N+1, N+1] indexed [v][e][k][j][i] like the box operator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import euler as eu
from .refelem import refelem

F64 = torch.float64
BG_NEUTRAL, BG_CONSTANT, BG_ISOTHERMAL = 0, 1, 2


@dataclass(frozen=True)
class SphereDesc:
    N: int
    n: int                 # elements per panel edge
    nz: int                # radial layers
    r_e: float = 6.371e6   # the earth radius of section 4.4
    H: float = 1.0e4       # model top of section 4.4
    max_level: int = 0     # refinement levels allowed above the unrefined shell


# cube point of local panel coordinates (X, Y) with the panel's fixed coordinate c
# (c = 1 for real coordinates, c = n for the integer lattice of grid lines)
def panel_point(p, X, Y, c=1):
    return [(c, X, Y), (-X, c, Y), (-c, -X, Y), (X, -c, Y), (-Y, X, c), (Y, X, -c)][p]


def leaf_index(desc: SphereDesc, p, ia, ib, ir):
    return ((p * desc.nz + ir) * desc.n + ib) * desc.n + ia


WALL, CONF, FINE, COARSE = 0, 1, 2, 3     # face kinds


def _panel_coords(p, P, m):
    """(X, Y) of the cube point P on panel p (P[fixed axis] = +-m), or None if
    P does not lie on that panel"""
    x, y, z = P
    fixed = [(x, m), (y, m), (x, -m), (y, -m), (z, m), (z, -m)][p]
    if fixed[0] != fixed[1]:
        return None
    return [(y, z), (-x, z), (-y, z), (x, z), (y, -x), (y, x)][p]


def lateral_neighbour(p, m, gx, gy, f):
    """Same-size neighbour across lateral face f of the cell (gx, gy) of panel p at
    resolution m (cells per panel edge): (p2, gx2, gy2, f2, flip), flip = 1 when the
    two faces' first axes run opposite.  Found on the integer lattice of grid lines
    (a cell face's end points are cube points with integer coordinates in units of
    half a cell), so faces across a panel edge match exactly."""
    X0, Y0 = 2 * gx - m, 2 * gy - m
    X1, Y1 = X0 + 2, Y0 + 2
    a0, a1 = [((X0, Y0), (X0, Y1)), ((X1, Y0), (X1, Y1)), ((X0, Y0), (X1, Y0)), ((X0, Y1), (X1, Y1))][f]
    step = [(-1, 0), (1, 0), (0, -1), (0, 1)][f]
    gx2, gy2 = gx + step[0], gy + step[1]
    if 0 <= gx2 < m and 0 <= gy2 < m:
        return p, gx2, gy2, f ^ 1, 0
    P0, P1 = panel_point(p, *a0, c=m), panel_point(p, *a1, c=m)
    for p2 in range(6):
        if p2 == p:
            continue
        b0, b1 = _panel_coords(p2, P0, m), _panel_coords(p2, P1, m)
        if b0 is None or b1 is None:
            continue
        if b0[0] == b1[0]:              # a face of constant X: faces 0 / 1, first axis Y
            f2 = 0 if b0[0] == -m else 1
            gx2, gy2 = (0 if f2 == 0 else m - 1), (min(b0[1], b1[1]) + m) // 2
            first = b0[1] < b1[1]       # does P0 sit at the neighbour face's a = 0 end
        else:                           # constant Y: faces 2 / 3, first axis X
            f2 = 2 if b0[1] == -m else 3
            gx2, gy2 = (min(b0[0], b1[0]) + m) // 2, (0 if f2 == 2 else m - 1)
            first = b0[0] < b1[0]
        return p2, gx2, gy2, f2, 0 if first else 1
    raise RuntimeError("no panel across a panel edge")


def cell_neighbour(desc: SphereDesc, cell, f):
    """Same-level neighbour of cell (p, l, gx, gy, gz) across face f: (cell2, f2,
    flip), or None at the bottom and top walls"""
    p, l, gx, gy, gz = cell
    if f >= 4:
        gz2 = gz + (1 if f == 5 else -1)
        if not 0 <= gz2 < desc.nz << l:
            return None
        return (p, l, gx, gy, gz2), f ^ 1, 0
    p2, gx2, gy2, f2, flip = lateral_neighbour(p, desc.n << l, gx, gy, f)
    return (p2, l, gx2, gy2, gz), f2, flip


def cell_children(cell):
    """child c = bx + 2 by + 4 bz"""
    p, l, gx, gy, gz = cell
    return [(p, l + 1, 2 * gx + (c & 1), 2 * gy + ((c >> 1) & 1), 2 * gz + (c >> 2)) for c in range(8)]


def cell_parent(cell):
    p, l, gx, gy, gz = cell
    return (p, l - 1, gx >> 1, gy >> 1, gz >> 1)


def cell_child_id(cell):
    return (cell[2] & 1) | ((cell[3] & 1) << 1) | ((cell[4] & 1) << 2)


def _tangential(d):
    return [(1, 2), (0, 2), (0, 1)][d]


def leaf_key(desc: SphereDesc, cell):
    """order: panel, root element (layer, row, column of the unrefined shell), then
    the Morton key of the position inside the root at the finest level (x least
    significant); the unrefined shell keeps e = ((p nz + ir) n + ib) n + ia"""
    p, l, gx, gy, gz = cell
    L = desc.max_level
    lx, ly, lz = (g & ((1 << l) - 1) for g in (gx, gy, gz))
    lx, ly, lz = lx << (L - l), ly << (L - l), lz << (L - l)
    key = 0
    for bit in range(L):
        key |= (((lx >> bit) & 1) | (((ly >> bit) & 1) << 1) | (((lz >> bit) & 1) << 2)) << (3 * bit)
    return (p, gz >> l, gy >> l, gx >> l, key)


class SphereMesh:
    """Leaves (p, l, gx, gy, gz): panel, level, and the cell's column, row and layer
    among the n 2^l x n 2^l x nz 2^l cells of its panel at that level.  The
    unrefined shell (level 0 everywhere) unless leaves are given.  Face tables per
    leaf and face: kind[e, f] (WALL at the bottom and top, CONF, FINE: this leaf is
    one of four fine sides of a hanging face, COARSE: its coarse side);
    nb[e, f] = (neighbour leaf, its face, flip) for CONF, (coarse leaf, its face,
    flip) for FINE, (hanging row, the fine leaves' face, flip) for COARSE,
    (-1, -1, 0) at walls; aux[e, f] = the quadrant in the coarse face's axes for
    FINE.  Hanging rows hang[h] = (coarse leaf, its face, the fine leaves by
    quadrant qa + 2 qb over the coarse face's first and second axes), with the
    fine leaves' face hang_ff[h] and flip hang_flip[h].  flip = 1 when the two
    faces' first axes run opposite.  Transfer plan xfer_src, xfer_kind as for the
    brick forest (-1 copy, 0..7 child, 8 family)."""

    def __init__(self, desc: SphereDesc, leaves=None, xfer=None):
        n, nz = desc.n, desc.nz
        self.desc, self.N = desc, desc.N
        if leaves is None:
            leaves = [(p, 0, ia, ib, ir) for p in range(6) for ir in range(nz) for ib in range(n) for ia in range(n)]
        leaves = sorted(set(tuple(int(x) for x in lf) for lf in leaves), key=lambda c: leaf_key(desc, c))
        self.leaves = np.array(leaves, dtype=np.int64).reshape(-1, 5)
        self.K = len(leaves)
        self.index = {lf: e for e, lf in enumerate(leaves)}
        if xfer is None:
            xfer = (np.arange(self.K), -np.ones(self.K, dtype=np.int64))
        self.xfer_src, self.xfer_kind = (np.asarray(x, dtype=np.int64) for x in xfer)
        self._tables()

    def containing(self, cell):
        """the leaf equal to or containing the cell, or None (the cell is refined)"""
        p, l, gx, gy, gz = cell
        for lv in range(l, -1, -1):
            sh = l - lv
            c = (p, lv, gx >> sh, gy >> sh, gz >> sh)
            if c in self.index:
                return c
        return None

    def _tables(self):
        K = self.K
        kind = np.zeros((K, 6), dtype=np.int64)
        nb = -np.ones((K, 6, 3), dtype=np.int64)
        nb[:, :, 2] = 0
        aux = np.zeros((K, 6), dtype=np.int64)
        hang, hang_ff, hang_flip = [], [], []
        for e, lf in enumerate(map(tuple, self.leaves.tolist())):
            for f in range(6):
                got = cell_neighbour(self.desc, lf, f)
                if got is None:
                    continue
                c, f2, flip = got
                x = self.containing(c)
                if x is not None and x[1] == lf[1]:
                    kind[e, f], nb[e, f] = CONF, (self.index[x], f2, flip)
                elif x is not None:
                    # fine side: c lies inside the coarse leaf x; its quadrant on x's
                    # face f2 is given by c's bits along that face's two axes
                    t1, t2 = _tangential(f2 // 2)
                    bits = (c[2] & 1, c[3] & 1, c[4] & 1)
                    kind[e, f], nb[e, f], aux[e, f] = FINE, (self.index[x], f2, flip), bits[t1] + 2 * bits[t2]
                else:
                    # coarse side: the four children of c on its face f2, placed by
                    # their bits along c's face axes (the first reversed when flipped)
                    d2, s2 = f2 // 2, f2 % 2
                    t1, t2 = _tangential(d2)
                    fine = [None] * 4
                    for ch in cell_children(c):
                        b = (ch[2] & 1, ch[3] & 1, ch[4] & 1)
                        if b[d2] != s2:
                            continue
                        qa = 1 - b[t1] if flip else b[t1]
                        fine[qa + 2 * b[t2]] = self.index[ch]
                    kind[e, f], nb[e, f] = COARSE, (len(hang), f2, flip)
                    hang.append((e, f) + tuple(fine))
                    hang_ff.append(f2)
                    hang_flip.append(flip)
        self.kind, self.nb, self.aux = kind, nb, aux
        self.hang = np.array(hang, dtype=np.int64).reshape(-1, 6)
        self.hang_ff = np.array(hang_ff, dtype=np.int64)
        self.hang_flip = np.array(hang_flip, dtype=np.int64)


def _ripple(desc, mesh_leaves):
    """leaves with a face neighbour two or more levels finer (the 2:1 face balance)"""
    tmp = SphereMesh.__new__(SphereMesh)
    tmp.index = {lf: 0 for lf in mesh_leaves}
    out = set()
    for lf in mesh_leaves:
        for f in range(6):
            got = cell_neighbour(desc, lf, f)
            if got is None:
                continue
            x = SphereMesh.containing(tmp, got[0])
            if x is not None and x[1] <= lf[1] - 2:
                out.add(x)
    return out


def refine_pass(prev: SphereMesh, flags) -> SphereMesh:
    """section 3.1 refinement on the shell: leaves flagged +1 below max_level are
    split, then every leaf with a face neighbour two levels finer, to a fixed point"""
    desc = prev.desc
    leaves = set(map(tuple, prev.leaves.tolist()))
    for e, lf in enumerate(map(tuple, prev.leaves.tolist())):
        if flags[e] > 0 and lf[1] < desc.max_level:
            leaves.discard(lf)
            leaves.update(cell_children(lf))
    while True:
        todo = _ripple(desc, leaves)
        if not todo:
            break
        for x in todo:
            leaves.discard(x)
            leaves.update(cell_children(x))
    new = sorted(leaves, key=lambda c: leaf_key(desc, c))
    src, kind = np.zeros(len(new), dtype=np.int64), np.zeros(len(new), dtype=np.int64)
    for e, lf in enumerate(new):
        if lf in prev.index:
            src[e], kind[e] = prev.index[lf], -1
        else:
            par = cell_parent(lf)
            if par not in prev.index:
                raise RuntimeError("a leaf was refined twice in one pass")
            src[e], kind[e] = prev.index[par], cell_child_id(lf)
    return SphereMesh(desc, new, (src, kind))


def coarsen_pass(prev: SphereMesh, flags) -> SphereMesh:
    """section 3.1 coarsening on the shell: a family of eight leaves, all flagged -1,
    is replaced by its parent unless a leaf face-adjacent to the parent is two or
    more levels finer than the parent (judged on the mesh before the pass)"""
    desc = prev.desc
    parents = set()
    for e, lf in enumerate(map(tuple, prev.leaves.tolist())):
        if lf[1] == 0 or flags[e] >= 0:
            continue
        par = cell_parent(lf)
        if par in parents:
            continue
        fam = cell_children(par)
        if not all(c in prev.index and flags[prev.index[c]] < 0 for c in fam):
            continue
        vetoed = False
        for f in range(6):
            got = cell_neighbour(desc, par, f)
            if got is None:
                continue
            c, f2, _ = got
            if prev.containing(c) is not None:
                continue
            d2, s2 = f2 // 2, f2 % 2
            for ch in cell_children(c):
                if (ch[2 + d2] & 1) == s2 and ch not in prev.index:
                    vetoed = True
        if not vetoed:
            parents.add(par)
    leaves = set(map(tuple, prev.leaves.tolist()))
    for par in parents:
        leaves.difference_update(cell_children(par))
        leaves.add(par)
    new = sorted(leaves, key=lambda c: leaf_key(desc, c))
    src, kind = np.zeros(len(new), dtype=np.int64), np.zeros(len(new), dtype=np.int64)
    for e, lf in enumerate(new):
        if lf in prev.index:
            src[e], kind[e] = prev.index[lf], -1
        else:
            src[e], kind[e] = prev.index[cell_children(lf)[0]], 8
    return SphereMesh(desc, new, (src, kind))


LD = np.longdouble
PI_LD = np.longdouble("3.141592653589793238462643383279502884")


def _tan_grid(s, n):
    """tan of the equiangular angle s pi/(4n) in long double, exactly +-1 on the
    panel edges (n may be an array broadcast against s)"""
    s = np.asarray(s, dtype=LD)
    n = np.asarray(n)
    t = np.tan(s * PI_LD / (LD(4) * n.astype(LD)))
    t = np.where(s == n, LD(1), t)
    return np.where(s == -n, LD(-1), t)


def face_perm(N, flip):
    """index map m -> m' of face-local nodes m = a + (N+1) b to the neighbour's face"""
    n1 = N + 1
    m = np.arange(n1 * n1)
    a, b = m % n1, m // n1
    return (N - a) + n1 * b if flip else m


def _dxi(D, t, d):
    """derivative along reference axis d of a nodal field [K, k, j, i] (numpy),
    applied to the field minus its value at the line's first node (D annihilates
    constants; the shift keeps an offset far larger than the variation along the
    line, such as the earth radius in a node position, out of the sums)"""
    if d == 0:
        return np.einsum('im,ekjm->ekji', D, t - t[..., :1])
    if d == 1:
        return np.einsum('jm,ekmi->ekji', D, t - t[..., :1, :])
    return np.einsum('km,emji->ekji', D, t - t[:, :1, :, :])


def _face(t, f, N):
    """numpy version of the face trace [K, (N+1)^2] of a nodal field [K, k, j, i]"""
    d, s = f // 2, f % 2
    idx = N if s == 1 else 0
    tr = t[..., idx] if d == 0 else (t[..., idx, :] if d == 1 else t[..., idx, :, :])
    return tr.reshape(*tr.shape[:-2], (N + 1) ** 2)


class SphereGeometry:
    """Nodes, metric terms, Jacobian, radial unit vector and face normals.

    The geometry of a thin shell is ill-conditioned in float64 (the curl-form
    metric terms cancel in proportion to the element aspect ratio, several hundred
    for the shells of section 4.4), so it is evaluated in long double and rounded
    once to float64."""

    def __init__(self, mesh: SphereMesh):
        desc, N = mesh.desc, mesh.N
        n, nz = desc.n, desc.nz
        re = refelem(N)
        K, n1 = mesh.K, N + 1
        self.N, self.K = N, K
        xi = np.asarray(re.x, dtype=np.float64).astype(LD)
        Dl = np.asarray(re.D, dtype=np.float64).astype(LD)
        self.D = torch.as_tensor(re.D, dtype=F64)
        p, lv, gx, gy, gz = (mesh.leaves[:, c] for c in range(5))
        m = (n << lv)[:, None]                     # cells per panel edge at each leaf's level
        mz = (nz << lv).astype(LD)[:, None]
        # 1-D node parameters per leaf: X = tan alpha, Y = tan beta, height h
        sX = (2 * gx - (n << lv)).astype(LD)[:, None] + (xi[None, :] + LD(1))
        sY = (2 * gy - (n << lv)).astype(LD)[:, None] + (xi[None, :] + LD(1))
        X1, Y1 = _tan_grid(sX, m), _tan_grid(sY, m)                      # [K, N+1]
        h1 = LD(desc.H) * (gz.astype(LD)[:, None] + LD(0.5) * (xi[None, :] + LD(1))) / mz
        self.X1, self.Y1, self.h1 = X1.astype(np.float64), Y1.astype(np.float64), h1.astype(np.float64)
        X = np.broadcast_to(X1[:, None, None, :], (K, n1, n1, n1))
        Y = np.broadcast_to(Y1[:, None, :, None], (K, n1, n1, n1))
        r = np.broadcast_to((LD(desc.r_e) + h1)[:, :, None, None], (K, n1, n1, n1))
        cube = [np.zeros((K, n1, n1, n1), dtype=LD) for _ in range(3)]
        for pp in range(6):
            sel = p == pp
            v = panel_point(pp, X[sel], Y[sel], np.ones_like(X[sel]))
            for c in range(3):
                cube[c][sel] = v[c]
        norm = np.sqrt(cube[0] ** 2 + cube[1] ** 2 + cube[2] ** 2)
        rhat = [c / norm for c in cube]
        x = [r * u for u in rhat]
        dX = [[_dxi(Dl, x[c], d) for d in range(3)] for c in range(3)]   # dX[c][d] = d x_c / d xi_d
        J = (dX[0][0] * (dX[1][1] * dX[2][2] - dX[1][2] * dX[2][1])
             - dX[0][1] * (dX[1][0] * dX[2][2] - dX[1][2] * dX[2][0])
             + dX[0][2] * (dX[1][0] * dX[2][1] - dX[1][1] * dX[2][0]))
        # curl form: Ja[i][n] = -(curl_xi V)_i, V_d = X_l d_d X_m, (n, m, l) cyclic; X_l
        # is taken relative to the element's first node (the discrete curl of
        # c grad X_m vanishes for a constant c, so the shift changes only the rounding)
        Ja = [[None] * 3 for _ in range(3)]
        for nn in range(3):
            m, l = (nn + 1) % 3, (nn + 2) % 3
            Xl = x[l] - x[l][:, :1, :1, :1]
            V = [Xl * dX[m][d] for d in range(3)]
            curl = [_dxi(Dl, V[2], 1) - _dxi(Dl, V[1], 2), _dxi(Dl, V[0], 2) - _dxi(Dl, V[2], 0),
                    _dxi(Dl, V[1], 0) - _dxi(Dl, V[0], 1)]
            for i in range(3):
                Ja[i][nn] = -curl[i]
        # face normals and face Jacobians, [K, 6, (N+1)^2] each; shared faces from the
        # (leaf, face) pair that comes first
        nf = n1 * n1
        own_n = np.zeros((3, K, 6, nf), dtype=LD)
        own_s = np.zeros((K, 6, nf), dtype=LD)
        for f in range(6):
            d, sgn = f // 2, (LD(1) if f % 2 else LD(-1))
            v = [sgn * _face(Ja[d][c], f, N) for c in range(3)]
            sf = np.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
            own_s[:, f] = sf
            for c in range(3):
                own_n[c, :, f] = v[c] / sf
        own_n, own_s = own_n.astype(np.float64), own_s.astype(np.float64)
        nrm = np.zeros((3, K, 6, nf))
        sJ = np.zeros((K, 6, nf))
        for e in range(K):
            for f in range(6):
                e2, f2, flip = (int(x_) for x_ in mesh.nb[e, f])
                if mesh.kind[e, f] != CONF or (e, f) < (e2, f2):
                    nrm[:, e, f] = own_n[:, e, f]
                    sJ[e, f] = own_s[e, f]
                else:
                    perm = face_perm(N, flip)
                    nrm[:, e, f] = -own_n[:, e2, f2][:, perm]
                    sJ[e, f] = own_s[e2, f2][perm]
        t64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64))
        self.rhat = [t64(u) for u in rhat]                      # radial unit vector
        self.x = [t64(c) for c in x]                            # node positions
        self.height = t64(r - LD(desc.r_e))
        self.J = t64(J)
        self.Ja = [[t64(Ja[i][c]) for c in range(3)] for i in range(3)]
        self.nrm, self.sJ = t64(nrm), t64(sJ)

    def dxi(self, t, d):
        """derivative along reference axis d of a float64 nodal field [K, k, j, i]"""
        D = self.D
        if d == 0:
            return torch.einsum('im,ekjm->ekji', D, t)
        if d == 1:
            return torch.einsum('jm,ekmi->ekji', D, t)
        return torch.einsum('km,emji->ekji', D, t)

    def face_positions(self, f):
        return [eu.face_slice(x, f, self.N) for x in self.x]


def background(geo: SphereGeometry, phys: eu.Phys, kind):
    """(rhobar, Thetabar, Pbar) at every node as functions of the height h."""
    h = geo.height
    R, gam = phys.R, phys.gamma
    if kind == BG_ISOTHERMAL:
        T0 = phys.theta0
        P_b = phys.P0 * torch.exp(-phys.g * h / (R * T0))
        rho_b = P_b / (R * T0)
        Th_b = (phys.P0 / R) * (P_b / phys.P0) ** (1.0 / gam)
        return rho_b, Th_b, P_b
    if kind == BG_NEUTRAL:
        exner = 1.0 - phys.g * h / (phys.cp * phys.theta0)
        rho_b = phys.P0 * exner ** (phys.cv / R) / (R * phys.theta0)
        Th_b = rho_b * phys.theta0
    elif kind == BG_CONSTANT:
        rho_b = torch.full_like(h, phys.rho0)
        Th_b = torch.full_like(h, phys.Theta0)
    else:
        raise ValueError("unknown background")
    P_b = phys.P0 * (R * Th_b / phys.P0) ** gam
    return rho_b, Th_b, P_b


def flux_normal(q, bg, phys, nv):
    """F.n for the unit vector n = (n0, n1, n2) (tensors of the trace's shape)."""
    rho, u, Pp, _ = eu.primitives(q, bg, phys)
    un = u[0] * nv[0] + u[1] * nv[1] + u[2] * nv[2]
    Th = bg[1] + q[4]
    return torch.stack([q[1] * nv[0] + q[2] * nv[1] + q[3] * nv[2],
                        q[1] * un + Pp * nv[0], q[2] * un + Pp * nv[1], q[3] * un + Pp * nv[2], Th * un])


def rusanov_normal(qL, bgL, qR, bgR, phys, nv):
    """F*.n = {F.n} + 1/2 lambda (q'- - q'+), lambda = max(|u.n| + c) of both sides."""
    rhoL, uL, _, PL = eu.primitives(qL, bgL, phys)
    rhoR, uR, _, PR = eu.primitives(qR, bgR, phys)
    lamL = torch.abs(uL[0] * nv[0] + uL[1] * nv[1] + uL[2] * nv[2]) + eu.sound_speed(rhoL, PL, phys.gamma)
    lamR = torch.abs(uR[0] * nv[0] + uR[1] * nv[1] + uR[2] * nv[2]) + eu.sound_speed(rhoR, PR, phys.gamma)
    lam = torch.maximum(lamL, lamR)
    return 0.5 * (flux_normal(qL, bgL, phys, nv) + flux_normal(qR, bgR, phys, nv)) + 0.5 * lam * (qL - qR)


class SphereOperator:
    """The curvilinear right-hand side on a cubed-sphere shell."""

    def __init__(self, mesh: SphereMesh, phys: eu.Phys, background_kind=BG_ISOTHERMAL):
        self.mesh, self.phys, self.N, self.K = mesh, phys, mesh.N, mesh.K
        self.geo = SphereGeometry(mesh)
        self.bg = background(self.geo, phys, background_kind)
        self.wN = 2.0 / (self.N * (self.N + 1))
        re = refelem(self.N)
        self.re = re

    def contravariant(self, q):
        F = [eu.flux_dir(q, self.bg, self.phys, c) for c in range(3)]   # Cartesian fluxes
        Ja = self.geo.Ja
        return [Ja[i][0][None] * F[0] + Ja[i][1][None] * F[1] + Ja[i][2][None] * F[2] for i in range(3)]

    def volume(self, q):
        """-(1/J) sum_i D_i (J a^i . F) + S, S = -rho' g r_hat on the momentum"""
        Ft = self.contravariant(q)
        D = self.geo.D
        div = (torch.einsum('im,vekjm->vekji', D, Ft[0]) + torch.einsum('jm,vekmi->vekji', D, Ft[1])
               + torch.einsum('km,vemji->vekji', D, Ft[2]))
        R = -div / self.geo.J[None]
        g = self.phys.g
        z = torch.zeros_like(q[0])
        S = torch.stack([z] + [-q[0] * g * self.geo.rhat[c] for c in range(3)] + [z])
        return R + S

    def surface(self, q, walls=True):
        """Lifted face terms -(1/(J w_N)) (s F*(n) - sgn J a^d . F(q-)) at the face nodes
        of conforming faces and walls, then the hanging faces (mortars)."""
        N, K, ph, geo = self.N, self.K, self.phys, self.geo
        Ft = self.contravariant(q)
        R = torch.zeros(5, K, N + 1, N + 1, N + 1, dtype=F64)
        nb = torch.as_tensor(self.mesh.nb)
        kind = torch.as_tensor(self.mesh.kind)
        for f in range(6):
            d, sgn = f // 2, (1.0 if f % 2 else -1.0)
            qL = eu.face_slice(q, f, N)
            bL = tuple(eu.face_slice(b, f, N) for b in self.bg)
            nv = [geo.nrm[c, :, f] for c in range(3)]
            s = geo.sJ[:, f]
            qR = qL.clone()
            bR = tuple(b.clone() for b in bL)
            wall, conf = kind[:, f] == WALL, kind[:, f] == CONF
            for f2 in range(6):
                for flip in (0, 1):
                    sel = conf & (nb[:, f, 1] == f2) & (nb[:, f, 2] == flip)
                    if not bool(sel.any()):
                        continue
                    e2 = nb[sel, f, 0]
                    perm = torch.as_tensor(face_perm(N, flip))
                    qR[:, sel] = eu.face_slice(q, f2, N)[:, e2][:, :, perm]
                    for bi in range(3):
                        bR[bi][sel] = eu.face_slice(self.bg[bi], f2, N)[e2][:, perm]
            if bool(wall.any()):
                w = wall
                Un = qL[1][w] * nv[0][w] + qL[2][w] * nv[1][w] + qL[3][w] * nv[2][w]
                for c in range(3):
                    qR[1 + c][w] = qL[1 + c][w] - 2.0 * Un * nv[c][w]
            act = conf | wall if walls else conf
            Fs = rusanov_normal(qL, bL, qR, bR, ph, nv)
            delta = s[None] * Fs - sgn * eu.face_slice(Ft[d], f, N)
            JF = eu.face_slice(geo.J, f, N)
            delta = torch.where(act[None, :, None], delta / (JF[None] * self.wN), torch.zeros_like(delta))
            R = R - eu.face_embed(delta, f, N, K)
        return R + self.mortars(q, Ft)

    def mortars(self, q, Ft):
        """Hanging faces (section 3.3 on curved faces): on each fine face the coarse
        trace is interpolated to the fine face nodes (I_qa x I_qb in the coarse face's
        axes, reordered by the orientation) and the Riemann problem is solved there
        along the fine face's own normal and with the fine nodes' background; the fine
        side lifts s_f F* like a conforming face.  The coarse side takes the flux with
        the sign reversed per coarse reference area, 4 s_f (-F*) (a fine face covers a
        quarter of the coarse reference face), projected back with R_qa x R_qb and
        summed over the four quadrants: both sides see the same flux integral."""
        N, K, ph, geo, re = self.N, self.K, self.phys, self.geo, self.re
        mesh = self.mesh
        R = torch.zeros(5, K, N + 1, N + 1, N + 1, dtype=F64)
        I = [torch.as_tensor(M, dtype=F64) for M in re.I]
        Rm = [torch.as_tensor(M, dtype=F64) for M in re.R]
        for h in range(len(mesh.hang)):
            ec, fc = int(mesh.hang[h, 0]), int(mesh.hang[h, 1])
            ff, flip = int(mesh.hang_ff[h]), int(mesh.hang_flip[h])
            perm = torch.as_tensor(face_perm(N, flip))
            tc = eu.face_slice(q, fc, N)[:, ec]                              # [5, NF]
            proj = torch.zeros_like(tc)
            for quad in range(4):
                qa, qb = quad & 1, quad >> 1
                ef = int(mesh.hang[h, 2 + quad])
                tf = eu.face_slice(q, ff, N)[:, ef]
                qm = eu.interp2(I[qa], I[qb], tc, N)[:, perm]                # at the fine face nodes
                bf = tuple(eu.face_slice(b, ff, N)[ef] for b in self.bg)
                nv = [geo.nrm[c, ef, ff] for c in range(3)]
                sf = geo.sJ[ef, ff]
                Fs = rusanov_normal(tf, bf, qm, bf, ph, nv)
                sgn_f = 1.0 if ff % 2 else -1.0
                delta = sf[None] * Fs - sgn_f * eu.face_slice(Ft[ff // 2], ff, N)[:, ef]
                JF = eu.face_slice(geo.J, ff, N)[ef]
                d = torch.zeros(5, K, (N + 1) ** 2, dtype=F64)
                d[:, ef] = delta / (JF[None] * self.wN)
                R = R - eu.face_embed(d, ff, N, K)
                g = (4.0 * sf)[None] * (-Fs)
                proj = proj + eu.interp2(Rm[qa], Rm[qb], g[:, perm], N)
            sgn_c = 1.0 if fc % 2 else -1.0
            delta = proj - sgn_c * eu.face_slice(Ft[fc // 2], fc, N)[:, ec]
            JF = eu.face_slice(geo.J, fc, N)[ec]
            d = torch.zeros(5, K, (N + 1) ** 2, dtype=F64)
            d[:, ec] = delta / (JF[None] * self.wN)
            R = R - eu.face_embed(d, fc, N, K)
        return R

    def rhs(self, q):
        return self.volume(q) + self.surface(q)


def quad_weights(op: SphereOperator):
    """J W at every node (the element volume quadrature)."""
    w = torch.as_tensor(op.re.w, dtype=F64)
    return op.geo.J * w[:, None, None] * w[None, :, None] * w[None, None, :]


def budgets(op: SphereOperator, q):
    """(mass', total mass, integral of Theta', energy) with the potential energy
    rho g h (h the height above r_e), each an exactly rounded sum."""
    ph = op.phys
    JW = quad_weights(op)
    rho_b, Th_b, P_b = op.bg
    rho = rho_b + q[0]
    P = P_b + eu.pressure_perturbation(q[4], Th_b, P_b, ph.gamma)
    E = P / (ph.gamma - 1.0) + (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / (2.0 * rho) + rho * ph.g * op.geo.height

    def fsum(t):
        return math.fsum(t.detach().reshape(-1).tolist())

    return (fsum(JW * q[0]), fsum(JW * rho), fsum(JW * q[4]), fsum(JW * E))


# ----------------------------------------------------------------------------- areas (section 3.4)

def _angle(A, B, C):
    """interior angle at A of the spherical triangle ABC (unit vectors)"""
    tB = B - np.dot(A, B) * A
    tC = C - np.dot(A, C) * A
    return math.atan2(np.linalg.norm(np.cross(tB, tC)), np.dot(tB, tC))


def spherical_excess(A, B, C):
    """area of the spherical triangle ABC on the unit sphere: the sum of its
    interior angles minus pi"""
    return _angle(A, B, C) + _angle(B, C, A) + _angle(C, A, B) - math.pi


def element_areas(mesh: SphereMesh, radius):
    """area of every element's footprint on the sphere of the given radius, as
    two spherical triangles of its corner points (section 3.4's area formula)"""
    out = np.zeros(mesh.K)
    for e, (p, lv, ia, ib, _) in enumerate(mesh.leaves):
        n = mesh.desc.n << int(lv)
        corners = []
        for sx, sy in ((2 * ia - n, 2 * ib - n), (2 * ia + 2 - n, 2 * ib - n), (2 * ia + 2 - n, 2 * ib + 2 - n),
                       (2 * ia - n, 2 * ib + 2 - n)):
            v = np.array(panel_point(p, float(_tan_grid(sx, n)), float(_tan_grid(sy, n))), dtype=np.float64)
            corners.append(v / np.linalg.norm(v))
        out[e] = radius * radius * (spherical_excess(corners[0], corners[1], corners[2])
                                    + spherical_excess(corners[0], corners[2], corners[3]))
    return out


def element_volumes(mesh: SphereMesh):
    """volume of every element from its spherical-excess footprint on the unit
    sphere (section 3.4's area formula) times the radial integral of r^2:
    A_1 (r_top^3 - r_bot^3)/3, the difference of cubes written as (r_top - r_bot)
    (r_top^2 + r_top r_bot + r_bot^2)/3 to keep its digits"""
    d = mesh.desc
    A1 = element_areas(mesh, 1.0)
    ir = mesh.leaves[:, 4].astype(np.float64)
    mz = (d.nz << mesh.leaves[:, 1]).astype(np.float64)
    r0 = d.r_e + d.H * ir / mz
    r1 = d.r_e + d.H * (ir + 1.0) / mz
    return A1 * (r1 - r0) * (r1 * r1 + r1 * r0 + r0 * r0) / 3.0


def discrete_volume(op: SphereOperator):
    """the volume the isoparametric elements enclose, sum of J W over all nodes"""
    return math.fsum(quad_weights(op).reshape(-1).tolist())


# ----------------------------------------------------------------------------- shell transfers (section 3.4)
#
# Transfers between two uniform shells, the fine one with twice the elements per
# panel edge and twice the layers: every element of the coarse shell is the parent
# of the eight fine elements (p, 2 ia + ax, 2 ib + ay, 2 ir + az), child
# a = ax + 2 ay + 4 az, whose reference box is half ax, ay, az of the parent's along
# its three local axes.  Only the reference-element matrices are used (I_a, R_a),
# corrected as the paper prescribes for curved elements:
#
# * coarsening: the parent is the sum over its children of R_ax x R_ay x R_az q_a
#   (the reference projection) plus, per conserved field (rho and Theta with their
#   background), the constant that makes the parent's J W integral the sum of its
#   children's: each child contributes its own volume integral, the finite-volume
#   balance on the elements' discrete volumes, so the quadrature the solver
#   conserves between regrids is kept exactly;
# * refinement: every child takes I_ax x I_ay x I_az of its parent, then one scale
#   factor s, the total mass before over the total mass after (the J W quadrature
#   of rho = rhobar + rho' on each shell), multiplies every conserved field,
#   rho, rho u and Theta (background included), in every child; velocity and
#   potential temperature keep their interpolated values.

def _check_pair(coarse: SphereMesh, fine: SphereMesh):
    dc, df = coarse.desc, fine.desc
    if (df.n, df.nz, df.N) != (2 * dc.n, 2 * dc.nz, dc.N) or (df.r_e, df.H) != (dc.r_e, dc.H):
        raise ValueError("the fine shell must have twice the elements per edge and layers of the coarse one")


def children(coarse: SphereMesh, fine: SphereMesh):
    """ch[e, a] = index of child a of coarse element e in the fine shell"""
    _check_pair(coarse, fine)
    ch = np.zeros((coarse.K, 8), dtype=np.int64)
    for e, (p, _, ia, ib, ir) in enumerate(coarse.leaves):
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
            ch[e, a] = leaf_index(fine.desc, p, 2 * ia + ax, 2 * ib + ay, 2 * ir + az)
    return ch


def _apply3(A, B, C, t):
    """(C x B x A) applied to nodal fields [..., k, j, i]: A along i, B along j, C along k"""
    A, B, C = (torch.as_tensor(M, dtype=F64) for M in (A, B, C))
    return torch.einsum('im,jn,kl,...lnm->...kji', A, B, C, t)


def refine_shell(op_c: SphereOperator, op_f: SphereOperator, q_c):
    """section 3.4 (b): reference interpolation into the children, then one mass
    scale factor s applied to all conserved fields.  Returns (q_f, s)."""
    ch = children(op_c.mesh, op_f.mesh)
    I = op_c.re.I
    q_f = torch.zeros(5, op_f.K, *q_c.shape[2:], dtype=F64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
        q_f[:, torch.as_tensor(ch[:, a])] = _apply3(I[ax], I[ay], I[az], q_c)
    mass_c = budgets(op_c, q_c)[1]
    mass_f = budgets(op_f, q_f)[1]
    s = mass_c / mass_f
    rho_b, Th_b, _ = op_f.bg
    out = q_f.clone()
    out[0] = s * q_f[0] + (s - 1.0) * rho_b
    out[1:4] = s * q_f[1:4]
    out[4] = s * q_f[4] + (s - 1.0) * Th_b
    return out, s


def _conserved_background(op: SphereOperator):
    """the background part of each conserved field, [rhobar, 0, 0, 0, Thetabar]"""
    rho_b, Th_b, _ = op.bg
    z = torch.zeros_like(rho_b)
    return torch.stack([rho_b, z, z, z, Th_b])


def _family_constant(JW_kids, full_kids, JW_par, full_par):
    """per field, (sum of the children's J W integrals - the parent's) / the
    parent's J W volume, on the conserved fields (background included)"""
    inside = (JW_kids[None] * full_kids).sum(dim=(-4, -3, -2, -1))
    mine = (JW_par[None] * full_par).sum(dim=(-3, -2, -1))
    return (inside - mine) / JW_par.sum()


def coarsen_shell(op_f: SphereOperator, op_c: SphereOperator, q_f):
    """section 3.4 (a): the children's reference projections, plus per conserved
    field the constant that keeps each family's J W integral (background included).
    Returns q_c."""
    ch = children(op_c.mesh, op_f.mesh)
    Rm = op_c.re.R
    JWf, JWc = quad_weights(op_f), quad_weights(op_c)
    q_c = torch.zeros(5, op_c.K, *q_f.shape[2:], dtype=F64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
        q_c = q_c + _apply3(Rm[ax], Rm[ay], Rm[az], q_f[:, torch.as_tensor(ch[:, a])])
    Bf, Bc = _conserved_background(op_f), _conserved_background(op_c)
    for e in range(op_c.K):
        kids = torch.as_tensor(ch[e])
        c = _family_constant(JWf[kids], Bf[:, kids] + q_f[:, kids], JWc[e], Bc[:, e] + q_c[:, e])
        q_c[:, e] = q_c[:, e] + c[:, None, None, None]
    return q_c


def reference_means(q):
    """mean of each field over each element's reference cube, (1/8) sum W q, as
    [5, K] (the quantity the finite-volume reading of the coarsening conserves)"""
    N = q.shape[-1] - 1
    w = torch.as_tensor(refelem(N).w, dtype=F64)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return (q * W).sum(dim=(-3, -2, -1)) / 8.0


# ----------------------------------------------------------------------------- acoustic wave (section 4.4)

def acoustic_state(op: SphereOperator, h_max=100.0, r_c=None, lon=0.0, lat=0.0, n_v=1):
    """Section 4.4's acoustic wave around the globe: a pressure perturbation
    p' = f g on the background at rest, f the cosine bell (amplitude h_max, zero
    beyond the geodesic radius r_c, r_e/3 by default) about longitude lon and
    latitude lat (radians), g = sin(n_v pi h / H) with h the height.  Reading:
    potential temperature is left unperturbed (the pressure rise is isentropic),
    so Theta = (P0/R) (P/P0)^(1/gamma) at P = Pbar + p' and rho' = Theta'/thetabar.
    Returns the state [5, K, N+1, N+1, N+1]."""
    d, ph, geo = op.mesh.desc, op.phys, op.geo
    if r_c is None:
        r_c = d.r_e / 3.0
    cx = (math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat))
    cosang = geo.rhat[0] * cx[0] + geo.rhat[1] * cx[1] + geo.rhat[2] * cx[2]
    dist = d.r_e * torch.arccos(torch.clamp(cosang, -1.0, 1.0))
    f = torch.where(dist <= r_c, 0.5 * h_max * (1.0 + torch.cos(math.pi * dist / r_c)), torch.zeros_like(dist))
    g = torch.sin(n_v * math.pi * geo.height / d.H)
    pp = f * g
    rho_b, Th_b, P_b = op.bg
    Th = (ph.P0 / ph.R) * ((P_b + pp) / ph.P0) ** (1.0 / ph.gamma)
    Thp = Th - Th_b
    q = torch.zeros(5, *pp.shape, dtype=F64)
    q[4] = Thp
    q[0] = Thp * rho_b / Th_b
    return q


def vortex_state(op: SphereOperator, amp=1.0, width=5.0e5, lon=0.0, lat=0.0):
    """A Gaussian potential-temperature perturbation theta' = amp exp(-(d / width)^2),
    d the great-circle distance from longitude lon, latitude lat (radians), at
    unperturbed density (rho' = 0, Theta' = rhobar theta'), at rest.  Returns the
    state [5, K, N+1, N+1, N+1]."""
    d, geo = op.mesh.desc, op.geo
    cx = (math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat))
    cosang = geo.rhat[0] * cx[0] + geo.rhat[1] * cx[1] + geo.rhat[2] * cx[2]
    dist = d.r_e * torch.arccos(torch.clamp(cosang, -1.0, 1.0))
    q = torch.zeros(5, *dist.shape, dtype=F64)
    q[4] = op.bg[0] * (amp * torch.exp(-(dist / width) ** 2))
    return q


# ----------------------------------------------------------------------------- transfers of a refinement pass (section 3.4)

def _subset_mass(op: SphereOperator, q, elems):
    """J W quadrature of rho = rhobar + rho' over the given leaves, exactly rounded.
    When q carries a gradient the value is the same exactly rounded sum, returned
    as a tensor whose derivative is that of the plain sum (for the adjoint)."""
    JW = quad_weights(op)[elems]
    rho = op.bg[0][elems] + q[0][elems]
    exact = math.fsum((JW * rho).reshape(-1).tolist())
    if not q.requires_grad:
        return exact
    plain = (JW * rho).sum()
    return exact + (plain - plain.detach())


def adapt_project(op_from: SphereOperator, op_to: SphereOperator, q):
    """Section 3.4's transfer along the plan of a refine or coarsen pass (op_to's
    mesh built from op_from's): kept leaves are copied; a child takes the
    reference interpolation of its parent, and one scale factor s (the mass of the
    refined parents over the mass of their interpolated children) multiplies every
    conserved field of every child, background included; a merged family becomes
    the sum of its children's reference projections plus, per conserved field, the
    constant that keeps the family's J W integral (background included).  Returns
    (q_to, s), s = 1 when nothing was refined."""
    mesh = op_to.mesh
    src, kind = mesh.xfer_src, mesh.xfer_kind
    I, Rm = op_to.re.I, op_to.re.R
    out = torch.zeros(5, op_to.K, *q.shape[2:], dtype=F64)
    JW_from, JW_to = quad_weights(op_from), quad_weights(op_to)
    B_from, B_to = _conserved_background(op_from), _conserved_background(op_to)
    children_new, parents_old = [], set()
    for e in range(op_to.K):
        k, sidx = int(kind[e]), int(src[e])
        if k == -1:
            out[:, e] = q[:, sidx]
        elif k < 8:
            ax, ay, az = k & 1, (k >> 1) & 1, k >> 2
            out[:, e] = _apply3(I[ax], I[ay], I[az], q[:, sidx][:, None])[:, 0]
            children_new.append(e)
            parents_old.add(sidx)
        else:
            fam = list(range(sidx, sidx + 8))
            acc = torch.zeros_like(q[:, sidx])
            for a, ea in enumerate(fam):
                ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
                acc = acc + _apply3(Rm[ax], Rm[ay], Rm[az], q[:, ea][:, None])[:, 0]
            kids = torch.as_tensor(fam)
            c = _family_constant(JW_from[kids], B_from[:, kids] + q[:, kids], JW_to[e], B_to[:, e] + acc)
            out[:, e] = acc + c[:, None, None, None]
    s = 1.0
    if children_new:
        s = _subset_mass(op_from, q, sorted(parents_old)) / _subset_mass(op_to, out, children_new)
        ch = torch.as_tensor(children_new)
        rho_b, Th_b, _ = op_to.bg
        out[0, ch] = s * out[0, ch] + (s - 1.0) * rho_b[ch]
        out[1:4, ch] = s * out[1:4, ch]
        out[4, ch] = s * out[4, ch] + (s - 1.0) * Th_b[ch]
    return out, s


def adapt_project_adjoint(op_from: SphereOperator, op_to: SphereOperator, q, qbar_to):
    """The transpose of the derivative of adapt_project at q: qbar_from = (d q_to /
    d q)^T qbar_to in the Euclidean inner product on the DOF vectors, by
    reverse-mode differentiation of adapt_project (the refinement's scale factor
    depends on q, so the map is affine only for a coarsening)."""
    x = q.detach().clone().requires_grad_(True)
    out, _ = adapt_project(op_from, op_to, x)
    (g,) = torch.autograd.grad(out, x, grad_outputs=qbar_to)
    return g


# ----------------------------------------------------------------------------- regrid indicator (section 4.4)

IND_THETA, IND_PPRIME = 0, 2


def indicator(op: SphereOperator, q, kind=IND_PPRIME):
    """Per-leaf eta: max over its nodes of |theta'| (IND_THETA) or of |P'|
    (IND_PPRIME, the pressure perturbation section 4.4 regrids on)."""
    rho_b, Th_b, P_b = op.bg
    if kind == IND_PPRIME:
        val = torch.abs(eu.pressure_perturbation(q[4], Th_b, P_b, op.phys.gamma))
    else:
        val = torch.abs((Th_b + q[4]) / (rho_b + q[0]) - Th_b / rho_b)
    return val.reshape(op.K, -1).max(dim=1).values


def flags_from_indicator(mesh: SphereMesh, eta, thr):
    """+1 where eta > thr below max_level; -1 where eta <= thr above level 0; else 0"""
    lev = mesh.leaves[:, 1]
    eta = np.asarray(eta)
    fl = np.zeros(mesh.K, dtype=np.int8)
    fl[(eta > thr) & (lev < mesh.desc.max_level)] = 1
    fl[(eta <= thr) & (lev > 0)] = -1
    return fl
