"""Oracle: 1-D reference-element operators on [-1, 1] (test infrastructure only).

The paper builds its element operators on the reference element once and applies
them as tensor products (section 3.3, conservative coarsening by LGL integration;
mortar projections P = M^{-1} S built from the mass matrix M and the mixed mass
matrix S, with the reverse projection scaled by s = 1/2 for a 2:1 tree).  The
collocation points are the Legendre-Gauss-Lobatto (LGL) nodes, whose quadrature
gives the diagonal mass matrix of section 2.2.

Everything here is plain numpy float64, written from the definitions:
  * LGL nodes  : -1, +1 and the roots of P_N'(x)   (Newton on P_N')
  * LGL weights: w_j = 2 / (N (N+1) P_N(x_j)^2)
  * D[i, j]    : derivative of the j-th Lagrange basis polynomial at x_i
  * I_a[m, j]  : l_j evaluated at the image of node x_m in half-interval a
                 (a = 0 -> [-1, 0], a = 1 -> [0, 1])
  * M[j, k]    : exact integral of l_j l_k (Gauss-Legendre with N+2 points)
  * R_a        : 1/2 M^{-1} I_a^T M, the L2 projection from half-interval a
                 back to the parent interval (sum over both halves gives the
                 full projection; section 3.3 reverse projection with s = 1/2).
"""
from __future__ import annotations

import functools

import numpy as np


def legendre(N: int, x):
    """P_N(x) and P_{N-1}(x) by the three-term recurrence (Bonnet)."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for n in range(1, N):
        p_next = ((2 * n + 1) * x * p - n * p_prev) / (n + 1)
        p_prev, p = p, p_next
    return p, p_prev


def lgl_nodes_weights(N: int):
    """LGL nodes x_0 = -1 < ... < x_N = 1 and weights (section 3.3 LGL integration)."""
    if N < 1:
        raise ValueError("N >= 1 required")
    # initial guess: Chebyshev-Gauss-Lobatto points
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    inner = x[1:-1].copy()
    for _ in range(100):
        p, pm1 = legendre(N, inner)
        # (1 - x^2) P_N' = N (P_{N-1} - x P_N)
        dp = N * (pm1 - inner * p) / (1.0 - inner * inner)
        # Legendre ODE: (1 - x^2) P_N'' = 2 x P_N' - N (N+1) P_N
        d2p = (2.0 * inner * dp - N * (N + 1) * p) / (1.0 - inner * inner)
        step = dp / d2p
        inner = inner - step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x = np.concatenate(([-1.0], inner, [1.0]))
    # enforce exact symmetry x_{N-j} = -x_j
    x = 0.5 * (x - x[::-1])
    if N % 2 == 0:
        x[N // 2] = 0.0
    p, _ = legendre(N, x)
    w = 2.0 / (N * (N + 1) * p * p)
    return x, w


def lagrange_eval(xnodes, y):
    """L[m, j] = l_j(y_m), product formula for the Lagrange basis on ``xnodes``."""
    xnodes = np.asarray(xnodes, dtype=np.float64)
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    n = len(xnodes)
    L = np.ones((len(y), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (y - xnodes[k]) / (xnodes[j] - xnodes[k])
    return L


def derivative_matrix(xnodes):
    """D[i, j] = l_j'(x_i) from barycentric weights; D[i, i] = -sum_{j != i} D[i, j]."""
    x = np.asarray(xnodes, dtype=np.float64)
    n = len(x)
    lam = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                lam[j] /= (x[j] - x[k])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, np.arange(n) != i])
    return D


def half_interp(xnodes, a: int):
    """I_a[m, j] = l_j((x_m + 2a - 1)/2): parent nodal values -> nodes of half a."""
    x = np.asarray(xnodes, dtype=np.float64)
    return lagrange_eval(x, (x + 2 * a - 1) / 2.0)


def pointwise_from_half(xnodes, a: int):
    """P_a[m, j] = c_a(m) l_j(2 x_m - (2a - 1)): the polynomial of half a (nodal
    values on its own LGL nodes) evaluated at the parent's node m, for pointwise
    matching at a non-conforming face (section 3.3, alternative (a)).  c_a(m) = 1
    when x_m lies inside half a, 1/2 on the midpoint x_m = 0 shared by both halves
    (the two values are averaged), 0 otherwise."""
    x = np.asarray(xnodes, dtype=np.float64)
    inside = (x <= 0.0) if a == 0 else (x >= 0.0)
    c = np.where(inside, np.where(x == 0.0, 0.5, 1.0), 0.0)
    return c[:, None] * lagrange_eval(x, 2.0 * x - (2 * a - 1))


def exact_mass(xnodes):
    """M[j, k] = integral over [-1,1] of l_j l_k, exact (Gauss-Legendre, N+2 points)."""
    x = np.asarray(xnodes, dtype=np.float64)
    g, wg = np.polynomial.legendre.leggauss(len(x) + 1)
    L = lagrange_eval(x, g)
    return (L * wg[:, None]).T @ L


def restriction(xnodes, a: int):
    """R_a = 1/2 M^{-1} I_a^T M (section 3.3 reverse projection, s = 1/2)."""
    M = exact_mass(xnodes)
    Ia = half_interp(xnodes, a)
    return 0.5 * np.linalg.solve(M, Ia.T @ M)


class RefElem:
    """All 1-D operators for polynomial order N (float64 numpy arrays)."""

    def __init__(self, N: int):
        self.N = N
        self.x, self.w = lgl_nodes_weights(N)
        self.D = derivative_matrix(self.x)
        self.I = [half_interp(self.x, 0), half_interp(self.x, 1)]
        self.M = exact_mass(self.x)
        self.R = [restriction(self.x, 0), restriction(self.x, 1)]
        self.P = [pointwise_from_half(self.x, 0), pointwise_from_half(self.x, 1)]


@functools.lru_cache(maxsize=None)
def refelem(N: int) -> RefElem:
    return RefElem(N)
