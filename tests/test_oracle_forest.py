"""Pins of the oracle's forest (section 3.1 forest of trees, section 4.3 2:1
balance): brute-force geometric checks on tiny forests with random flags.

The geometry here is recomputed independently from integer boxes in the global
finest-cell index space, so a wrong neighbour, quadrant, balance rule or table
entry in the oracle fails one of these checks.
"""
import itertools

import numpy as np
import pytest

from oracle import forest as fo
from paper_2404_16648_amd.synth import random_flags


def _boxes(mesh):
    return fo.leaf_boxes(mesh)


def _extent(desc):
    return [desc.nroot[d] << desc.max_level for d in range(3)]


def _face_contact(desc, A, B, d):
    """Area of contact between the plus face (axis d) of box A and the minus face of
    box B, counting a periodic wrap; 0 if they do not touch there."""
    ext = _extent(desc)
    ahi, blo = A[1, d], B[0, d]
    touch = ahi == blo or (desc.periodic[d] and ahi == ext[d] and blo == 0)
    if not touch:
        return 0
    area = 1
    for t in range(3):
        if t == d:
            continue
        ov = min(A[1, t], B[1, t]) - max(A[0, t], B[0, t])
        if ov <= 0:
            return 0
        area *= ov
    return area


def _adjacent_pairs(mesh):
    """All (e1, e2, d, area) with e1's plus face touching e2's minus face."""
    bx = _boxes(mesh)
    out = []
    for e1 in range(mesh.K):
        for e2 in range(mesh.K):
            for d in range(3):
                a = _face_contact(mesh.desc, bx[e1], bx[e2], d)
                if a > 0:
                    out.append((e1, e2, d, a))
    return out


def _balanced(mesh):
    lev = mesh.levels()
    return all(abs(int(lev[a]) - int(lev[b])) <= 1 for a, b, _, _ in _adjacent_pairs(mesh))


def _random_balanced_mesh(desc, seed, rounds=3):
    m = fo.build(desc, None)
    rng = np.random.default_rng(seed)
    for _ in range(rounds):
        fl = (rng.random(m.K) < 0.3).astype(np.int8)
        m = fo.build(desc, m, fl, fo.PASS_REFINE)
    return m


DESCS = [
    fo.ForestDesc(2, 2, 2, 2, 3, periodic=(0, 0, 0)),
    fo.ForestDesc(2, 2, 1, 2, 3, periodic=(1, 0, 1)),
    fo.ForestDesc(2, 1, 2, 1, 2, periodic=(1, 1, 1)),
    # root counts that are not powers of two: the Morton curve over the roots
    # differs from the lexicographic root order
    fo.ForestDesc(2, 3, 2, 3, 2, periodic=(1, 0, 0)),
]


@pytest.mark.parametrize("di,seed", list(itertools.product(range(len(DESCS)), range(6))))
def test_refine_pass_balanced_minimal(di, seed):
    desc = DESCS[di]
    prev = _random_balanced_mesh(desc, 100 + seed, rounds=2)
    assert _balanced(prev)
    flags = (np.random.default_rng(seed).random(prev.K) < 0.25).astype(np.int8)
    m = fo.build(desc, prev, flags, fo.PASS_REFINE)
    assert _balanced(m)
    # every flagged leaf below Lmax was refined, kept leaves are copies
    for e, lf in enumerate(prev.leaves):
        if flags[e] > 0 and lf[1] < desc.max_level:
            assert lf not in set(m.leaves)
    # minimality: every refinement not asked for by a flag is forced, i.e. merging
    # the family back would leave its parent next to a leaf two levels finer
    bx = _boxes(m)
    lev = m.levels()
    idx_prev = {lf: e for e, lf in enumerate(prev.leaves)}
    for e, lf in enumerate(m.leaves):
        if int(m.xfer_kind[e]) == 0:       # first child of a refined old leaf
            p = prev.leaves[int(m.xfer_src[e])]
            if flags[idx_prev[p]] > 0:
                continue
            pb = fo.leaf_boxes(fo.Mesh(desc, [p]))[0]
            forced = False
            for e2 in range(m.K):
                if lev[e2] < p[1] + 2:
                    continue
                for d in range(3):
                    if _face_contact(desc, pb, bx[e2], d) or _face_contact(desc, bx[e2], pb, d):
                        forced = True
            assert forced, "ripple refinement that balance did not require"
    # transfer plan: children of src have the right child id
    for e, lf in enumerate(m.leaves):
        k, s = int(m.xfer_kind[e]), int(m.xfer_src[e])
        if k == fo.KIND_COPY:
            assert prev.leaves[s] == lf
        else:
            assert fo.parent(lf) == prev.leaves[s] and fo.child_id(lf) == k


@pytest.mark.parametrize("di,seed", list(itertools.product(range(len(DESCS)), range(6))))
def test_coarsen_pass_veto(di, seed):
    desc = DESCS[di]
    prev = _random_balanced_mesh(desc, 200 + seed, rounds=3)
    flags = random_flags(prev.K, seed, p_refine=0.0, p_coarsen=0.8)
    m = fo.build(desc, prev, flags, fo.PASS_COARSEN)
    assert _balanced(m)
    idx = {lf: e for e, lf in enumerate(prev.leaves)}
    new = set(m.leaves)
    bx_prev = _boxes(prev)
    lev_prev = prev.levels()
    seen = set()
    for e, lf in enumerate(prev.leaves):
        if lf[1] == 0:
            continue
        p = fo.parent(lf)
        if p in seen:
            continue
        seen.add(p)
        fam = fo.children(p)
        if not all(c in idx for c in fam):
            assert p not in new
            continue
        all_flag = all(flags[idx[c]] < 0 for c in fam)
        # brute force veto: a leaf of the old mesh touching the parent box, 2+ levels finer
        pb = fo.leaf_boxes(fo.Mesh(desc, [p]))[0]
        vetoed = False
        for e2 in range(prev.K):
            if prev.leaves[e2] in fam or lev_prev[e2] < p[1] + 2:
                continue
            for d in range(3):
                if _face_contact(desc, pb, bx_prev[e2], d) or _face_contact(desc, bx_prev[e2], pb, d):
                    vetoed = True
        assert (p in new) == (all_flag and not vetoed)
    for e, lf in enumerate(m.leaves):
        k, s = int(m.xfer_kind[e]), int(m.xfer_src[e])
        if k == fo.KIND_COPY:
            assert prev.leaves[s] == lf
        else:
            assert k == fo.KIND_FAMILY
            assert [prev.leaves[s + c] for c in range(8)] == fo.children(lf)


@pytest.mark.parametrize("di,seed", list(itertools.product(range(len(DESCS)), range(5))))
def test_face_tables_cover_every_face_once(di, seed):
    desc = DESCS[di]
    m = _random_balanced_mesh(desc, 300 + seed, rounds=3)
    bx = _boxes(m)
    lev = m.levels()
    # volumes sum to the domain volume
    ext = _extent(desc)
    vol = sum(int(np.prod(b[1] - b[0])) for b in bx)
    assert vol == ext[0] * ext[1] * ext[2]
    # leaves in the order of one Morton curve over the whole brick: the bits of
    # the global integer lower corner interleaved (x least significant) increase
    def zkey(corner):
        k = 0
        for b in range(int(max(ext)).bit_length()):
            for a in range(3):
                k |= ((int(corner[a]) >> b) & 1) << (3 * b + a)
        return k
    keys = [zkey(b[0]) for b in bx]
    assert all(keys[i] < keys[i + 1] for i in range(len(keys) - 1))
    covered = {}
    for eM, eP, d in m.conf:
        assert lev[eM] == lev[eP]
        assert _face_contact(desc, bx[eM], bx[eP], d) == int(np.prod([bx[eM][1, t] - bx[eM][0, t] for t in range(3) if t != d]))
        for key in ((eM, 2 * d + 1), (eP, 2 * d)):
            covered[key] = covered.get(key, 0) + 1
    for e, f in m.bnd:
        d, s = f // 2, f % 2
        coord = bx[e][1, d] if s else bx[e][0, d]
        assert not desc.periodic[d] and coord == (ext[d] if s else 0)
        covered[(e, f)] = covered.get((e, f), 0) + 1
    for row in m.hang:
        ec, f = row[0], row[1]
        d, s = f // 2, f % 2
        t1, t2 = [t for t in range(3) if t != d]
        covered[(ec, f)] = covered.get((ec, f), 0) + 1
        half = (bx[ec][1, t1] - bx[ec][0, t1]) // 2
        for q in range(4):
            ef = row[2 + q]
            a, b = q & 1, q >> 1
            assert lev[ef] == lev[ec] + 1
            assert bx[ef][0, t1] == bx[ec][0, t1] + a * half
            assert bx[ef][0, t2] == bx[ec][0, t2] + b * half
            if s:
                assert _face_contact(desc, bx[ec], bx[ef], d) > 0
            else:
                assert _face_contact(desc, bx[ef], bx[ec], d) > 0
            fkey = (ef, 2 * d + (1 - s))
            covered[fkey] = covered.get(fkey, 0) + 1
    for e in range(m.K):
        for f in range(6):
            assert covered.get((e, f), 0) == 1, (e, f)
    # every geometric adjacency appears in the tables
    for e1, e2, d, area in _adjacent_pairs(m):
        if lev[e1] == lev[e2]:
            assert any((r[0] == e1 and r[1] == e2 and r[2] == d) for r in m.conf)
        else:
            ec, ef = (e1, e2) if lev[e1] < lev[e2] else (e2, e1)
            fc = 2 * d + (1 if ec == e1 else 0)
            assert any(r[0] == ec and r[1] == fc and ef in r[2:] for r in m.hang)


def test_uniform_counts():
    """4x4x4 walls: 144 interior faces and 96 boundary faces; 16^3: 11520 and 1536."""
    m = fo.build(fo.ForestDesc(4, 4, 4, 4, 2), None)
    assert (m.K, len(m.conf), len(m.bnd), len(m.hang)) == (64, 144, 96, 0)
    m = fo.build(fo.ForestDesc(4, 16, 16, 16, 0), None)
    assert (m.K, len(m.conf), len(m.bnd), len(m.hang)) == (4096, 11520, 1536, 0)


def test_node_coordinates_shared_faces_bitwise():
    desc = fo.ForestDesc(4, 3, 2, 2, 3, lo=(0.0, 0.0, 0.0), hi=(1000.0, 300.0, 700.0))
    m = _random_balanced_mesh(desc, 7, rounds=3)
    from oracle.refelem import refelem
    c = fo.node_coords_1d(m, refelem(4).x)
    for eM, eP, d in m.conf:
        if not desc.periodic[d]:
            assert c[d, eM, -1] == c[d, eP, 0]
    for row in m.hang:
        ec, f = row[0], row[1]
        d, s = f // 2, f % 2
        for ef in row[2:]:
            assert c[d, ec, -1 if s else 0] == c[d, ef, 0 if s else -1]


@pytest.mark.parametrize("di,seed", list(itertools.product(range(len(DESCS)), range(4))))
def test_buffer_flags_is_face_hop_distance(di, seed):
    """Buffer zone (section 3.2, B): a leaf ends +1 iff it was +1 or lies within B
    face hops of a +1 leaf, with face contact taken from the integer boxes (not
    from the oracle's tables); other flags are kept."""
    desc = DESCS[di]
    m = _random_balanced_mesh(desc, 500 + seed, rounds=2)
    rng = np.random.default_rng(900 + seed)
    fl = rng.choice(np.array([-1, 0, 0, 0, 1], dtype=np.int8), size=m.K)
    nbrs = [set() for _ in range(m.K)]
    for a, b, _, _ in _adjacent_pairs(m):
        nbrs[a].add(b)
        nbrs[b].add(a)
    dist = [None] * m.K
    front = [e for e in range(m.K) if fl[e] > 0]
    for e in front:
        dist[e] = 0
    while front:
        nxt = []
        for e in front:
            for x in nbrs[e]:
                if dist[x] is None:
                    dist[x] = dist[e] + 1
                    nxt.append(x)
        front = nxt
    for B in range(4):
        got = fo.buffer_flags(m, fl, B)
        want = np.array([1 if dist[e] is not None and dist[e] <= B else int(fl[e]) for e in range(m.K)],
                        dtype=np.int8)
        assert np.array_equal(got, want), (B, np.nonzero(got != want))
