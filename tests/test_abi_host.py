"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, rejects bad arguments, and its forest builder
reproduces the oracle's integer tables bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import forest as fo
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_flags
from tests.helpers import oracle_desc, tables_equal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dg.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dg.EXPORTED)


def test_bad_arguments_are_rejected():
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(1, (1, 1, 1), 0, host_only=True)
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(4, (1, 1, 1), 13, host_only=True)
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError):
        dg.dg_mesh_build(4, (1, 1, 1), 2, lo=(0, 0, 0), hi=(1, 0, 1), host_only=True)
    m = dg.dg_mesh_build(4, (2, 1, 1), 2, host_only=True)
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(prev=m, flags=np.zeros(2, np.int8), pass_=7)
    assert e.value.code == dg.DG_EINVAL
    # field calls on a host-only mesh fail with DG_EINVAL (no device touched)
    L = dg.lib()
    p = dg.PhysParams().c()
    code = L.dg_rhs(m.handle, ctypes.byref(p), None, None, None)
    assert code == dg.DG_EINVAL
    assert b"host_only" in L.dg_last_error()
    # bad physics
    m2 = dg.dg_mesh_build(4, (1, 1, 1), 0, host_only=True)
    bad = dg.PhysParams(cp=700.0).c()
    assert L.dg_budgets(m2.handle, ctypes.byref(bad), None, None, None) == dg.DG_EINVAL


CASES = [
    dict(N=4, nroot=(4, 4, 4), L=2, periodic=(0, 0, 0)),
    dict(N=3, nroot=(3, 2, 2), L=3, periodic=(1, 0, 1)),
    dict(N=2, nroot=(1, 2, 1), L=3, periodic=(1, 1, 1)),
    dict(N=7, nroot=(2, 2, 2), L=2, periodic=(0, 1, 0)),
]


@pytest.mark.parametrize("ci,seed", [(c, s) for c in range(len(CASES)) for s in range(4)])
def test_forest_tables_match_oracle(ci, seed):
    c = CASES[ci]
    lo, hi = (0.0, 0.0, 0.0), (1000.0, 500.0, 700.0)
    lm = dg.dg_mesh_build(c["N"], c["nroot"], c["L"], lo, hi, c["periodic"], host_only=True)
    od = oracle_desc(c["N"], c["nroot"], c["L"], lo, hi, c["periodic"])
    om = fo.build(od, None)
    assert tables_equal(lm.tables(), om)
    rng = np.random.default_rng(seed)
    for step in range(6):
        if step % 3 == 2:
            fl = random_flags(om.K, 1000 * seed + step, p_refine=0.0, p_coarsen=0.9)
            pas, opas = dg.DG_PASS_COARSEN, fo.PASS_COARSEN
        else:
            fl = (rng.random(om.K) < 0.3).astype(np.int8)
            pas, opas = dg.DG_PASS_REFINE, fo.PASS_REFINE
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=pas)
        om = fo.build(od, om, fl, opas)
        assert lm.K == om.K
        assert tables_equal(lm.tables(), om), (ci, seed, step)
        info = lm.info
        assert (info.n_conf, info.n_bnd, info.n_hang) == (len(om.conf), len(om.bnd), len(om.hang))


def test_uniform_config_counts():
    m = dg.dg_mesh_build(4, (16, 16, 16), 0, host_only=True)
    assert (m.K, m.info.n_conf, m.info.n_bnd, m.info.n_hang) == (4096, 11520, 1536, 0)


def test_passes_that_change_no_leaf():
    """A refine pass without an effective flag and a coarsen pass whose only family
    is vetoed by 2:1 balance keep every leaf and table, with the identity transfer
    plan, as the oracle's passes do (the library takes its copy path here)."""
    lo, hi = (0.0, 0.0, 0.0), (1000.0, 1000.0, 1000.0)
    od = oracle_desc(3, (2, 1, 1), 2, lo, hi, (0, 0, 0))
    om = fo.build(od, None)
    lm = dg.dg_mesh_build(3, (2, 1, 1), 2, lo, hi, host_only=True)
    # refine both roots, then the children of root 1 that touch root 0 (x = 0 side)
    fl = np.ones(om.K, np.int8)
    om = fo.build(od, om, fl, fo.PASS_REFINE)
    lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    fl = np.array([1 if (lf[0] == 1 and lf[2] == 0) else 0 for lf in om.leaves], np.int8)
    om = fo.build(od, om, fl, fo.PASS_REFINE)
    lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    assert tables_equal(lm.tables(), om) and om.levels().max() == 2
    K = om.K
    identity = np.arange(K, dtype=np.int32)
    # (a) refine pass: nothing flagged, then only leaves already at max_level flagged
    for fl in (np.zeros(K, np.int8), np.where(om.levels() == 2, 1, 0).astype(np.int8)):
        om2 = fo.build(od, om, fl, fo.PASS_REFINE)
        lm2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        assert tables_equal(lm2.tables(), om2) and om2.leaves == om.leaves
        assert np.array_equal(om2.xfer_src, identity) and np.all(om2.xfer_kind == fo.KIND_COPY)
        assert lm2.info.n_refined == 0
    # (b) coarsen pass: root 0's children form a family, but its parent would face
    # level-2 leaves of root 1, so the family is vetoed
    fl = np.array([-1 if (lf[0] == 0 and lf[1] == 1) else 0 for lf in om.leaves], np.int8)
    assert (fl < 0).sum() == 8
    om2 = fo.build(od, om, fl, fo.PASS_COARSEN)
    lm2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_COARSEN)
    assert tables_equal(lm2.tables(), om2) and om2.leaves == om.leaves
    assert np.array_equal(om2.xfer_src, identity) and lm2.info.n_coarsened == 0
    # a coarsen pass that does merge (root 1's level-2 families) still matches
    fl = np.where(om.levels() == 2, -1, 0).astype(np.int8)
    om3 = fo.build(od, om, fl, fo.PASS_COARSEN)
    lm3 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_COARSEN)
    assert tables_equal(lm3.tables(), om3) and lm3.info.n_coarsened > 0


@pytest.mark.parametrize("ci,seed", [(c, s) for c in range(len(CASES)) for s in range(2)])
def test_flags_buffer_matches_oracle(ci, seed):
    """Buffer zone (B rounds of face-neighbour dilation of the +1 flags): the
    library's host implementation against the oracle's, bit-exact, on AMR meshes
    with hanging faces and periodic wraps."""
    c = CASES[ci]
    lo, hi = (0.0, 0.0, 0.0), (1000.0, 500.0, 700.0)
    lm = dg.dg_mesh_build(c["N"], c["nroot"], c["L"], lo, hi, c["periodic"], host_only=True)
    od = oracle_desc(c["N"], c["nroot"], c["L"], lo, hi, c["periodic"])
    om = fo.build(od, None)
    rng = np.random.default_rng(70 + seed)
    for _ in range(2):
        fl = (rng.random(om.K) < 0.3).astype(np.int8)
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
        om = fo.build(od, om, fl, fo.PASS_REFINE)
    fl = rng.choice(np.array([-1, 0, 0, 0, 0, 0, 1], dtype=np.int8), size=om.K)
    for B in range(4):
        assert np.array_equal(dg.dg_flags_buffer(lm, fl, B), fo.buffer_flags(om, fl, B)), B
    with pytest.raises(dg.DGError):
        dg.dg_flags_buffer(lm, fl, -1)


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_pass_changes_predicts_the_pass(ci):
    """dg_pass_changes answers whether the pass changes a leaf without building a
    mesh: it must agree with what dg_mesh_build then does (n_refined /
    n_coarsened), on flag patterns that do and do not change the mesh: random
    flags, all -1 (complete families, some vetoed), -1 only on level-0 leaves
    (no family), +1 only at max_level (nothing to refine)."""
    c = CASES[ci]
    lo, hi = (0.0, 0.0, 0.0), (1000.0, 500.0, 700.0)
    lm = dg.dg_mesh_build(c["N"], c["nroot"], c["L"], lo, hi, c["periodic"], host_only=True)
    rng = np.random.default_rng(90 + ci)
    for _ in range(2):
        lm = dg.dg_mesh_build(prev=lm, flags=(rng.random(lm.K) < 0.3).astype(np.int8), pass_=dg.DG_PASS_REFINE)
    lvl = lm.tables()["leaf"][:, 1]
    patterns = [rng.choice(np.array([-1, 0, 1], dtype=np.int8), size=lm.K) for _ in range(4)]
    patterns += [np.full(lm.K, -1, np.int8), np.where(lvl == 0, -1, 0).astype(np.int8),
                 np.where(lvl == c["L"], 1, 0).astype(np.int8), np.zeros(lm.K, np.int8)]
    seen = set()
    for fl in patterns:
        for pass_ in (dg.DG_PASS_COARSEN, dg.DG_PASS_REFINE):
            pred = dg.dg_pass_changes(lm, fl, pass_)
            m2 = dg.dg_mesh_build(prev=lm, flags=fl, pass_=pass_)
            got = (m2.info.n_coarsened if pass_ == dg.DG_PASS_COARSEN else m2.info.n_refined) > 0
            assert pred == got, (pass_, pred, got)
            seen.add((pass_, pred))
    assert len(seen) == 4  # both answers for both passes
    with pytest.raises(dg.DGError):
        dg.dg_pass_changes(lm, np.zeros(lm.K, np.int8), 7)


def test_size_limit_at_the_kernels_indexing_bound():
    """5 K Np must stay below 2^31 (the kernels' 32-bit field offsets): N = 7 (Np =
    512) allows K < 838,861, so a 94^3 forest (830,584 leaves) builds and a 95^3
    one (857,375) is refused with DG_EINVAL before any device work."""
    m = dg.dg_mesh_build(7, (94, 94, 94), 0, host_only=True)
    assert m.K == 94 ** 3 and 5 * m.K * m.Np < 2 ** 31
    del m
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_build(7, (95, 95, 95), 0, host_only=True)
    assert e.value.code == dg.DG_EINVAL and "too large" in str(e.value)


@pytest.mark.parametrize("seed", range(4))
def test_flags_after_coarsen(seed):
    """dg_flags_after_coarsen against the cycle read off the oracle's own coarsen
    pass: a kept leaf keeps a +1 flag, a parent made by the pass and every other
    leaf get 0; with a pass that changes nothing the flags carry over."""
    c = dict(N=3, nroot=(3, 2, 2), L=2, periodic=(1, 0, 0))
    od = oracle_desc(c["N"], c["nroot"], c["L"], (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), c["periodic"])
    om = fo.build(od, None)
    lm = dg.dg_mesh_build(c["N"], c["nroot"], c["L"], (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), c["periodic"],
                          host_only=True)
    rng = np.random.default_rng(seed)
    for _ in range(2):
        fl = (rng.random(om.K) < 0.4).astype(np.int8)
        om = fo.build(od, om, fl, fo.PASS_REFINE)
        lm = dg.dg_mesh_build(prev=lm, flags=fl, pass_=dg.DG_PASS_REFINE)
    flags = random_flags(om.K, 100 + seed, p_refine=0.3, p_coarsen=0.6)
    oc = fo.build(od, om, flags, fo.PASS_COARSEN)
    lc = dg.dg_mesh_build(prev=lm, flags=flags, pass_=dg.DG_PASS_COARSEN)
    assert tables_equal(lc.tables(), oc)
    want = np.zeros(oc.K, np.int8)
    for e in range(oc.K):
        if oc.xfer_kind[e] == fo.KIND_COPY and flags[oc.xfer_src[e]] > 0:
            want[e] = 1
    assert np.array_equal(dg.dg_flags_after_coarsen(lc, flags), want)
    # no family flagged: the identity plan carries the flags over (-1 dropped)
    flags2 = np.where(flags < 0, 0, flags).astype(np.int8)
    lc2 = dg.dg_mesh_build(prev=lm, flags=flags2, pass_=dg.DG_PASS_COARSEN)
    assert np.array_equal(dg.dg_flags_after_coarsen(lc2, flags2), flags2)
