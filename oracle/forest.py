"""Oracle: brick forest of oct-trees, 2:1 face balance and the mesh tables
(test infrastructure only).

Paper: each cell of the coarse mesh is the root of a tree, only active leaves are
kept, and cells marked for refinement or coarsening are replaced by their
children or parent (section 3.1); the tree-based runs keep 2:1 balance across
all levels (section 4.3, rising thermal bubble).  The paper does not fix an
ordering, a balance algorithm or table formats; the readings implemented here
are:

* A leaf is (r, l, ix, iy, iz): root index r = rx + nx*(ry + ny*rz), level l and
  integer anchor (ix, iy, iz) in [0, 2^l)^3 inside the root.  Leaves are sorted
  by (root key, Morton key): the root key interleaves the bits of (rx, ry, rz),
  the Morton key those of anchor * 2^(Lmax - l), x the least significant bit in
  both, so the whole brick is one space-filling curve.  Child c = a + 2b + 4c'
  (x, y, z bits).
* Balance is 2:1 across faces only (including periodic wraps).  A refine pass
  applies the +1 flags (l < Lmax) and then refines every leaf that has a face
  neighbour two or more levels finer, repeated to a fixed point.
* A coarsen pass replaces a family of 8 sibling leaves, all flagged -1, by its
  parent only if every leaf face-adjacent to the parent has level <= l_parent+1,
  judged against the mesh before the pass.
* Face tables, enumerated by leaf e ascending, then face f = 2d + s ascending
  (d = axis, s = 0 minus side, 1 plus side):
    BND  (e, f)               face on a no-flux wall
    CONF (eM, eP, d)          from the plus face of eM; same-level neighbour eP
    HANG (ec, f, e0..e3)      from the coarse side; fine leaves by quadrant
                              q = a + 2b over the two tangential axes in
                              increasing axis order
* Transfer plan, per new leaf: (src, kind) with kind -1 = copy of old leaf src,
  0..7 = child kind of old leaf src, 8 = parent of the 8 old leaves src..src+7.
* Node coordinates: x = lo + (hi - lo)/n * (r + (anchor + (1 + xi)/2) / 2^l),
  evaluated in exactly this association so that nodes shared by two leaves
  are bitwise identical.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PASS_COARSEN = 0
PASS_REFINE = 1

KIND_COPY = -1
KIND_FAMILY = 8


@dataclass(frozen=True)
class ForestDesc:
    N: int
    nx: int
    ny: int
    nz: int
    max_level: int
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (0, 0, 0)

    @property
    def nroot(self):
        return (self.nx, self.ny, self.nz)


def morton_key(desc: ForestDesc, leaf) -> int:
    r, l, ix, iy, iz = leaf
    sh = desc.max_level - l
    X, Y, Z = ix << sh, iy << sh, iz << sh
    key = 0
    for b in range(desc.max_level):
        key |= ((X >> b) & 1) << (3 * b)
        key |= ((Y >> b) & 1) << (3 * b + 1)
        key |= ((Z >> b) & 1) << (3 * b + 2)
    return key


def root_key(desc: ForestDesc, r) -> int:
    """Bits of the root coordinates (rx, ry, rz) interleaved, rx least significant."""
    rc = root_coords(desc, r)
    key = 0
    for b in range(max(desc.nroot).bit_length()):
        for a in range(3):
            key |= ((rc[a] >> b) & 1) << (3 * b + a)
    return key


def sort_leaves(desc, leaves):
    return sorted(leaves, key=lambda lf: (root_key(desc, lf[0]), morton_key(desc, lf)))


def root_coords(desc, r):
    nx, ny, _ = desc.nroot
    return (r % nx, (r // nx) % ny, r // (nx * ny))


def root_index(desc, rc):
    nx, ny, _ = desc.nroot
    return rc[0] + nx * (rc[1] + ny * rc[2])


def children(leaf):
    r, l, ix, iy, iz = leaf
    return [(r, l + 1, 2 * ix + (c & 1), 2 * iy + ((c >> 1) & 1), 2 * iz + ((c >> 2) & 1))
            for c in range(8)]


def parent(leaf):
    r, l, ix, iy, iz = leaf
    return (r, l - 1, ix >> 1, iy >> 1, iz >> 1)


def child_id(leaf):
    _, _, ix, iy, iz = leaf
    return (ix & 1) + 2 * (iy & 1) + 4 * (iz & 1)


def same_level_neighbor(desc, cell, f):
    """Cell of the same level across face f = 2d + s, or None at a wall."""
    r, l, ix, iy, iz = cell
    d, s = f // 2, f % 2
    a = [ix, iy, iz]
    rc = list(root_coords(desc, r))
    a[d] += 1 if s == 1 else -1
    n = 1 << l
    if a[d] < 0 or a[d] >= n:
        a[d] = n - 1 if a[d] < 0 else 0
        rc[d] += 1 if s == 1 else -1
        nd = desc.nroot[d]
        if rc[d] < 0 or rc[d] >= nd:
            if not desc.periodic[d]:
                return None
            rc[d] %= nd
    return (root_index(desc, rc), l, a[0], a[1], a[2])


def tangential_axes(d):
    return [t for t in range(3) if t != d]


class _LeafSet:
    def __init__(self, leaves):
        self.set = set(leaves)

    def containing(self, cell):
        """Leaf equal to ``cell`` or an ancestor of it, or None."""
        c = cell
        while True:
            if c in self.set:
                return c
            if c[1] == 0:
                return None
            c = parent(c)


def _face_children(cell, d, side):
    """The 4 children of ``cell`` that touch its face on ``side`` of axis d,
    ordered by quadrant a + 2b over the tangential axes."""
    t1, t2 = tangential_axes(d)
    out = []
    for b in range(2):
        for a in range(2):
            bits = [0, 0, 0]
            bits[d] = side
            bits[t1] = a
            bits[t2] = b
            out.append(children(cell)[bits[0] + 2 * bits[1] + 4 * bits[2]])
    return out


def _needs_ripple(desc, ls: _LeafSet):
    """Leaves that have a face neighbour two or more levels finer."""
    out = set()
    for z in ls.set:
        for f in range(6):
            c = same_level_neighbor(desc, z, f)
            if c is None:
                continue
            x = ls.containing(c)
            if x is not None and x[1] <= z[1] - 2:
                out.add(x)
    return out


@dataclass
class Mesh:
    desc: ForestDesc
    leaves: list
    conf: np.ndarray = field(default=None)     # [n_conf, 3]  (eM, eP, d)
    bnd: np.ndarray = field(default=None)      # [n_bnd, 2]   (e, f)
    hang: np.ndarray = field(default=None)     # [n_hang, 6]  (ec, f, e0, e1, e2, e3)
    xfer_src: np.ndarray = field(default=None)  # [K]
    xfer_kind: np.ndarray = field(default=None)  # [K]

    @property
    def K(self):
        return len(self.leaves)

    @property
    def N(self):
        return self.desc.N

    def levels(self):
        return np.array([lf[1] for lf in self.leaves], dtype=np.int32)


def _build_tables(mesh: Mesh):
    desc = mesh.desc
    index = {lf: e for e, lf in enumerate(mesh.leaves)}
    ls = _LeafSet(mesh.leaves)
    conf, bnd, hang = [], [], []
    for e, lf in enumerate(mesh.leaves):
        for f in range(6):
            d, s = f // 2, f % 2
            c = same_level_neighbor(desc, lf, f)
            if c is None:
                bnd.append((e, f))
                continue
            x = ls.containing(c)
            if x is not None and x[1] == lf[1]:
                if s == 1:
                    conf.append((e, index[x], d))
            elif x is not None:
                pass  # this leaf is the fine side; emitted by the coarse leaf
            else:
                fine = _face_children(c, d, 1 - s)
                hang.append((e, f) + tuple(index[q] for q in fine))
    mesh.conf = np.array(conf, dtype=np.int32).reshape(-1, 3)
    mesh.bnd = np.array(bnd, dtype=np.int32).reshape(-1, 2)
    mesh.hang = np.array(hang, dtype=np.int32).reshape(-1, 6)
    return mesh


def uniform(desc: ForestDesc) -> Mesh:
    nroots = desc.nx * desc.ny * desc.nz
    leaves = sort_leaves(desc, [(r, 0, 0, 0, 0) for r in range(nroots)])
    m = Mesh(desc, leaves)
    m.xfer_src = np.arange(len(leaves), dtype=np.int32)
    m.xfer_kind = np.full(len(leaves), KIND_COPY, dtype=np.int32)
    return _build_tables(m)


def refine_pass(prev: Mesh, flags) -> Mesh:
    desc = prev.desc
    flags = np.asarray(flags)
    new = set(prev.leaves)
    for e, lf in enumerate(prev.leaves):
        if flags[e] > 0 and lf[1] < desc.max_level:
            new.discard(lf)
            new.update(children(lf))
    ls = _LeafSet(new)
    while True:
        todo = _needs_ripple(desc, ls)
        if not todo:
            break
        for x in todo:
            ls.set.discard(x)
            ls.set.update(children(x))
    leaves = sort_leaves(desc, ls.set)
    old_index = {lf: e for e, lf in enumerate(prev.leaves)}
    src = np.empty(len(leaves), dtype=np.int32)
    kind = np.empty(len(leaves), dtype=np.int32)
    for e, lf in enumerate(leaves):
        if lf in old_index:
            src[e], kind[e] = old_index[lf], KIND_COPY
        else:
            p = parent(lf)
            if p not in old_index:
                raise RuntimeError("a leaf was refined twice in one pass")
            src[e], kind[e] = old_index[p], child_id(lf)
    m = Mesh(desc, leaves, xfer_src=src, xfer_kind=kind)
    return _build_tables(m)


def _family_vetoed(desc, ls: _LeafSet, par):
    """True if some leaf face-adjacent to ``par`` is 2+ levels finer than it."""
    for f in range(6):
        d, s = f // 2, f % 2
        c = same_level_neighbor(desc, par, f)
        if c is None:
            continue
        if ls.containing(c) is not None:
            continue  # neighbour leaf at level <= l_par
        for q in _face_children(c, d, 1 - s):
            if q not in ls.set:
                return True
    return False


def coarsen_pass(prev: Mesh, flags) -> Mesh:
    desc = prev.desc
    flags = np.asarray(flags)
    ls = _LeafSet(prev.leaves)
    idx = {lf: e for e, lf in enumerate(prev.leaves)}
    parents = set()
    for e, lf in enumerate(prev.leaves):
        if lf[1] == 0 or flags[e] >= 0:
            continue
        p = parent(lf)
        if p in parents:
            continue
        fam = children(p)
        if all(c in idx and flags[idx[c]] < 0 for c in fam):
            if not _family_vetoed(desc, ls, p):
                parents.add(p)
    new = set(prev.leaves)
    for p in parents:
        for c in children(p):
            new.discard(c)
        new.add(p)
    leaves = sort_leaves(desc, new)
    src = np.empty(len(leaves), dtype=np.int32)
    kind = np.empty(len(leaves), dtype=np.int32)
    for e, lf in enumerate(leaves):
        if lf in idx:
            src[e], kind[e] = idx[lf], KIND_COPY
        else:
            src[e], kind[e] = idx[children(lf)[0]], KIND_FAMILY
    m = Mesh(desc, leaves, xfer_src=src, xfer_kind=kind)
    return _build_tables(m)


def build(desc: ForestDesc, prev: Mesh | None, flags=None, pass_=PASS_REFINE) -> Mesh:
    if prev is None:
        return uniform(desc)
    if pass_ == PASS_REFINE:
        return refine_pass(prev, flags)
    if pass_ == PASS_COARSEN:
        return coarsen_pass(prev, flags)
    raise ValueError("unknown pass")


# ----------------------------------------------------------------------------- geometry

def elem_lo_h(mesh: Mesh):
    """Per-leaf lower corner and edge lengths, float64 arrays [K, 3]."""
    desc = mesh.desc
    lo = np.zeros((mesh.K, 3))
    h = np.zeros((mesh.K, 3))
    for e, lf in enumerate(mesh.leaves):
        r, l, *anc = lf
        rc = root_coords(desc, r)
        for d in range(3):
            w = (desc.hi[d] - desc.lo[d]) / desc.nroot[d]
            lo[e, d] = desc.lo[d] + w * (rc[d] + (anc[d] + 0.0) / 2 ** l)
            h[e, d] = w / 2 ** l
    return lo, h


def node_coords_1d(mesh: Mesh, xi):
    """c[d][e, j] = coordinate along axis d of the j-th LGL node of leaf e."""
    desc = mesh.desc
    out = np.zeros((3, mesh.K, len(xi)))
    for e, lf in enumerate(mesh.leaves):
        r, l, *anc = lf
        rc = root_coords(desc, r)
        for d in range(3):
            w = (desc.hi[d] - desc.lo[d]) / desc.nroot[d]
            for j, x in enumerate(xi):
                out[d, e, j] = desc.lo[d] + w * (rc[d] + (anc[d] + (1.0 + x) / 2.0) / 2 ** l)
    return out


def leaf_boxes(mesh: Mesh):
    """Integer boxes [K, 2, 3] in units of the finest cell (global index space)."""
    desc = mesh.desc
    L = desc.max_level
    out = np.zeros((mesh.K, 2, 3), dtype=np.int64)
    for e, (r, l, *anc) in enumerate(mesh.leaves):
        rc = root_coords(desc, r)
        size = 1 << (L - l)
        for d in range(3):
            out[e, 0, d] = (rc[d] << L) + anc[d] * size
            out[e, 1, d] = out[e, 0, d] + size
    return out


def buffer_flags(mesh: Mesh, flags, B: int):
    """Buffer zone around refinement (section 3.2: a margin of B coarse cells between a
    feature and the coarse-fine interface; the tree-based code uses the same B).
    Reading: B rounds of face-neighbour dilation of the +1 flags; in each round
    every leaf that shares a face with a leaf flagged +1 is flagged +1 (0 and -1
    alike).  Face adjacency from the mesh's own lists: CONF pairs and the coarse
    leaf of each HANG row with each of its four fine leaves."""
    K = mesh.K
    adj = [set() for _ in range(K)]
    for eM, eP, _d in mesh.conf:
        adj[int(eM)].add(int(eP))
        adj[int(eP)].add(int(eM))
    for row in mesh.hang:
        ec = int(row[0])
        for x in row[2:]:
            adj[ec].add(int(x))
            adj[int(x)].add(ec)
    out = [int(v) for v in flags]
    for _ in range(B):
        cur = list(out)
        for e in range(K):
            if cur[e] > 0:
                for x in adj[e]:
                    out[x] = 1
    return np.array(out, dtype=np.int8)

