"""Shared helpers of the library-vs-oracle tests (no arithmetic of the method)."""
import numpy as np
import torch

from oracle import euler as eu
from oracle import forest as fo

F64 = torch.float64

# per-variable relative L2 bound for float64 results (a few hundred ulps of
# reassociation on sums of O(N) terms per node, far below any modelling error)
TOL_FP64 = 1e-12


def to_nodes(q):
    """oracle layout [5, K, N+1, N+1, N+1] -> library layout [5, K, Np] (same order)."""
    return q.reshape(q.shape[0], q.shape[1], -1).contiguous()


def to_elem(q, N):
    n1 = N + 1
    return q.reshape(q.shape[0], q.shape[1], n1, n1, n1)


def field_errors(a, b):
    """Relative L2 errors of the three fields rho', momentum (rho u, rho v, rho w as
    one vector field) and Theta'; where the reference field is 0, inf unless a is 0.

    The momentum is compared as a vector: a per-component bound is not rotation
    invariant, and a component that vanishes by symmetry (the horizontal momentum
    of a centred bubble after one step, ~1e-10) sits below the rounding floor of
    the problem (a one-ulp change of the background moves it by ~3e-12 relative)."""
    a = a.detach().double().cpu().reshape(a.shape[0], -1)
    b = b.detach().double().cpu().reshape(b.shape[0], -1)
    out = []
    for sl in (slice(0, 1), slice(1, 4), slice(4, 5)):
        nb = float(torch.linalg.vector_norm(b[sl]))
        nd = float(torch.linalg.vector_norm(a[sl] - b[sl]))
        out.append((0.0 if nd == 0.0 else float("inf")) if nb == 0.0 else nd / nb)
    return out


def rel_l2(a, b):
    """Per-variable ||a - b|| / ||b||; where ||b|| = 0, inf unless a is exactly 0 too."""
    a = a.detach().double().cpu().reshape(a.shape[0], -1)
    b = b.detach().double().cpu().reshape(b.shape[0], -1)
    out = []
    for v in range(a.shape[0]):
        nb = float(torch.linalg.vector_norm(b[v]))
        nd = float(torch.linalg.vector_norm(a[v] - b[v]))
        if nb == 0.0:
            out.append(0.0 if nd == 0.0 else float("inf"))
        else:
            out.append(nd / nb)
    return out


def assert_fields(a, b, tol, what="", vector_momentum=False):
    """Print the per-field and per-component relative L2 errors of a against b
    (library layout [5, K, Np]) and assert the bound.  By default every one of the
    five components is held to tol (random states: no component vanishes).  With
    vector_momentum the momentum is held to tol as one vector field, for states
    whose horizontal momentum vanishes by symmetry (the centred bubbles and the
    density current), where a per-component bound sits below the rounding floor."""
    err = field_errors(a, b)
    comp = rel_l2(a, b)
    print(what, "fields", ["%.2e" % x for x in err], "components", ["%.2e" % x for x in comp], flush=True)
    bound = err if vector_momentum else comp
    assert max(bound) <= tol, (what, err, comp)


def assert_conserved_fields(a, b, bg, tol, what=""):
    """As assert_fields, but rho' and Theta' compared as the full conserved fields
    rhobar + rho' and Thetabar + Theta' (bg = (rhobar, Thetabar) in the library
    layout [K, Np]): for a result that carries a constant fixed on the full fields
    (the coarsening's integral balance), whose rounding is relative to them."""
    import torch
    a = a.detach().double().cpu().clone()
    b = b.detach().double().cpu().clone()
    for v, bv in ((0, bg[0]), (4, bg[1])):
        a[v] += bv
        b[v] += bv
    assert_fields(a, b, tol, what)


def phys_for(periodic, **kw):
    """Library physics for a mesh with the given periodicity: a periodic z axis
    takes g = 0 (the neutral background is then constant; a hydrostatic profile
    cannot be periodic in z)."""
    from paper_2404_16648_amd import dg
    if periodic[2]:
        kw.setdefault("g", 0.0)
    return dg.PhysParams(**kw)


def oracle_phys(p):
    """oracle Phys with the same constants as a binding PhysParams."""
    return eu.Phys(cp=p.cp, cv=p.cv, P0=p.P0, g=p.g, background=p.background,
                   theta0=p.theta0, rho0=p.rho0, Theta0=p.Theta0, mu=p.mu)


def oracle_desc(N, nroot, max_level, lo, hi, periodic):
    return fo.ForestDesc(N, nroot[0], nroot[1], nroot[2], max_level, tuple(lo), tuple(hi), tuple(periodic))


def tables_equal(lib_tables, om):
    """Bit-exact comparison of the library's exported tables with the oracle mesh."""
    ok = (np.array_equal(lib_tables["leaf"], np.array(om.leaves, dtype=np.int32).reshape(-1, 5))
          and np.array_equal(lib_tables["conf"], om.conf)
          and np.array_equal(lib_tables["bnd"], om.bnd)
          and np.array_equal(lib_tables["hang"], om.hang)
          and np.array_equal(lib_tables["xfer_src"], om.xfer_src)
          and np.array_equal(lib_tables["xfer_kind"], om.xfer_kind))
    return ok


def random_refinements(desc, rounds, seed, p=0.35):
    """Flag sequences for `rounds` refine passes from the uniform mesh (oracle side)."""
    m = fo.build(desc, None)
    rng = np.random.default_rng(seed)
    seq = []
    for _ in range(rounds):
        fl = (rng.random(m.K) < p).astype(np.int8)
        seq.append(fl)
        m = fo.build(desc, m, fl, fo.PASS_REFINE)
    return seq
