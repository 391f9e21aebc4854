"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds no arithmetic of the method: only seeded random numbers with stated
scales and shapes.  Both the library checks and the oracle checks draw their
random states and flags from here.
"""
from __future__ import annotations

import numpy as np

# per-variable scales of a random perturbation (rho', rhou, rhov, rhow, Theta')
DEFAULT_SCALES = (1e-3, 0.1, 0.1, 0.1, 0.3)


def random_state(K: int, N: int, seed: int, scales=DEFAULT_SCALES) -> np.ndarray:
    """float64 array [5, K, (N+1)^3]: i.i.d. N(0,1) per DOF times the per-variable scale."""
    rng = np.random.default_rng(seed)
    Np = (N + 1) ** 3
    out = rng.standard_normal((5, K, Np))
    return out * np.asarray(scales, dtype=np.float64)[:, None, None]


def random_flags(K: int, seed: int, p_refine=0.2, p_coarsen=0.5) -> np.ndarray:
    """int8 array [K] with +1 (refine), -1 (coarsen) or 0 (keep)."""
    rng = np.random.default_rng(seed)
    u = rng.random(K)
    fl = np.zeros(K, dtype=np.int8)
    fl[u < p_refine] = 1
    fl[(u >= p_refine) & (u < p_refine + p_coarsen)] = -1
    return fl


def random_direction(K: int, N: int, seed: int, scales=DEFAULT_SCALES) -> np.ndarray:
    """A seeded direction for finite-difference checks (same recipe as random_state)."""
    return random_state(K, N, seed, scales)
