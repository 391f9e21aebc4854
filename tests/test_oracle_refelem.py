"""Pins of the oracle's 1-D reference-element operators (section 3.3).

Each check compares against something other than the oracle itself: closed-form
LGL nodes and weights, exact polynomial calculus with numpy's polynomial
module, and the defining L2-orthogonality of the projections.
"""
import json
import math
import os

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle.refelem import refelem

HERE = os.path.dirname(__file__)


def test_lgl_closed_forms():
    r2 = refelem(2)
    assert np.allclose(r2.x, [-1, 0, 1], atol=0, rtol=0) or np.allclose(r2.x, [-1, 0, 1], atol=1e-16)
    assert np.allclose(r2.w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    r3 = refelem(3)
    assert np.allclose(r3.x, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    assert np.allclose(r3.w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    r4 = refelem(4)
    s = math.sqrt(3 / 7)
    assert np.allclose(r4.x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(r4.w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_lgl_quadrature_degree(N):
    re = refelem(N)
    for k in range(0, 2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(re.w, re.x ** k) - exact) < 1e-14
    # LGL is exact to degree 2N-1, not 2N
    k = 2 * N
    assert abs(np.dot(re.w, re.x ** k) - 2 / (k + 1)) > 1e-6
    assert np.all(np.diff(re.x) > 0)
    assert np.array_equal(re.x, -re.x[::-1])


@pytest.mark.parametrize("N", [2, 4, 7])
def test_derivative_exact_on_monomials(N):
    re = refelem(N)
    for k in range(0, N + 1):
        f = re.x ** k
        df = k * re.x ** (k - 1) if k > 0 else np.zeros_like(re.x)
        assert np.max(np.abs(re.D @ f - df)) < 1e-12 * max(1, k * k)
    # summation-by-parts: W D + D^T W = diag(-1, 0, ..., 0, 1)
    W = np.diag(re.w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1, 1
    assert np.max(np.abs(W @ re.D + re.D.T @ W - B)) < 1e-13
    # first derivative of a degree N+1 polynomial is NOT exact
    f = re.x ** (N + 1)
    assert np.max(np.abs(re.D @ f - (N + 1) * re.x ** N)) > 1e-6


@pytest.mark.parametrize("N", [2, 4, 7])
def test_half_interval_interpolation(N):
    re = refelem(N)
    rng = np.random.default_rng(N)
    c = rng.standard_normal(N + 1)            # a random degree-N polynomial
    for a in (0, 1):
        y = (re.x + 2 * a - 1) / 2
        assert np.max(np.abs(re.I[a] @ P.polyval(re.x, c) - P.polyval(y, c))) < 1e-13


@pytest.mark.parametrize("N", [2, 4, 7])
def test_exact_mass_matrix(N):
    re = refelem(N)
    rng = np.random.default_rng(10 + N)
    for _ in range(3):
        c1, c2 = rng.standard_normal(N + 1), rng.standard_normal(N + 1)
        prod = P.polymul(c1, c2)
        integ = P.polyint(prod)
        exact = P.polyval(1.0, integ) - P.polyval(-1.0, integ)
        got = P.polyval(re.x, c1) @ re.M @ P.polyval(re.x, c2)
        assert abs(got - exact) < 1e-13 * max(1, abs(exact))
    assert np.max(np.abs(re.M.sum(axis=1) - re.w)) < 1e-14


@pytest.mark.parametrize("N", [2, 4, 7])
def test_restriction_is_l2_projection(N):
    re = refelem(N)
    # prolong then restrict is the identity
    S = re.R[0] @ re.I[0] + re.R[1] @ re.I[1]
    assert np.max(np.abs(S - np.eye(N + 1))) < 1e-13
    # integrals preserved: w^T R_a = w^T / 2
    for a in (0, 1):
        assert np.max(np.abs(re.w @ re.R[a] - 0.5 * re.w)) < 1e-15
    # L2 orthogonality against a discontinuous piecewise polynomial
    rng = np.random.default_rng(20 + N)
    cL, cR = rng.standard_normal(N + 1), rng.standard_normal(N + 1)
    fa = [P.polyval(re.x, cL), P.polyval(re.x, cR)]        # nodal values on each half
    p = re.R[0] @ fa[0] + re.R[1] @ fa[1]                   # nodal values on parent
    # monomial coefficients of p through its nodal values (exact degree N)
    cp = np.linalg.solve(np.vander(re.x, N + 1, increasing=True), p)
    for k in range(N + 1):
        # int_{-1}^{1} (p - f) x^k dx with f(x) = cL(2x+1) on [-1,0], cR(2x-1) on [0,1]
        def integ(c, lo, hi):
            ci = P.polyint(c)
            return P.polyval(hi, ci) - P.polyval(lo, ci)
        xk = np.zeros(k + 1); xk[k] = 1
        left = P.polymul(_compose_affine(cL, 2.0, 1.0), xk)
        right = P.polymul(_compose_affine(cR, 2.0, -1.0), xk)
        val = integ(P.polymul(cp, xk), -1, 1) - integ(left, -1, 0) - integ(right, 0, 1)
        assert abs(val) < 1e-13


def _compose_affine(c, s, t):
    """Coefficients of x -> p(s x + t)."""
    out = np.zeros(1)
    base = np.array([t, s])
    pw = np.ones(1)
    for ck in c:
        out = P.polyadd(out, ck * pw)
        pw = P.polymul(pw, base)
    return out


def test_lumped_mass_would_break_projection():
    """Special case showing the pin is discriminating: replacing the exact mass
    by the diagonal LGL mass breaks prolong-then-restrict = identity."""
    re = refelem(4)
    Mw = np.diag(re.w)
    R = [0.5 * np.linalg.solve(Mw, re.I[a].T @ Mw) for a in (0, 1)]
    S = R[0] @ re.I[0] + R[1] @ re.I[1]
    assert np.max(np.abs(S - np.eye(5))) > 0.1


def test_sound_speed_matches_paper():
    """The paper quotes the sound speed at 300 K (section 4.4); the oracle's
    default gas constants reproduce it to the printed digit."""
    from oracle.euler import Phys
    g = json.load(open(os.path.join(HERE, "golden", "sound_speed.json")))
    ph = Phys()
    c = math.sqrt(ph.gamma * ph.R * 300.0)
    assert round(c, g["digits"]) == g["sound_speed_300K_m_per_s"]
