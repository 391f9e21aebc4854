"""Measurements behind the oracle's physics pins (no assertions here).

Each function runs the oracle on an input whose right answer is fixed by the
mathematics or by a number the paper prints, and returns what it measured; the
tests in ``test_oracle_physics.py`` assert the bounds, and
``test_oracle_mutations.py`` plants plausible mistakes in the oracle and shows
that each one moves a measurement out of its bound.

What fixes the answers (nothing here calls the oracle's own formulas):
  * the equation of state P = P0 (R Theta / P0)^gamma of section 2.1, evaluated
    in 50-digit arithmetic (mpmath);
  * exact solutions of the Euler equations: a hydrostatic atmosphere of another
    potential temperature (its perturbation about the background has a zero
    time derivative), the isentropic vortex of section 4.1 (rigid translation),
    and a manufactured state whose exact time derivative -div F + S is formed
    by automatic differentiation of the physical fluxes written from the full
    pressure P (not the perturbation form);
  * the speed of sound at 300 K printed in section 4.4 (347.3 m/s), measured
    from the oscillation of a standing acoustic wave;
  * the Rusanov dissipation read back through the whole operator on two
    elements of constant state, against max(|u.n| + c) with c from the
    50-digit equation of state.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
import torch

from oracle import euler as eu
from oracle import forest as fo

F64 = torch.float64


# ----------------------------------------------------------------------------- equation of state

def eos_mp(Th, ph, dps=50):
    """P = P0 (R Theta / P0)^gamma (section 2.1) with 50 significant digits; the
    constants are taken as the float64 numbers the oracle is given."""
    with mp.workdps(dps):
        R, gam, P0 = mp.mpf(ph.R), mp.mpf(ph.gamma), mp.mpf(ph.P0)
        return P0 * (R * mp.mpf(Th) / P0) ** gam


def pprime_relative_errors(Thb, xs, ph):
    """Relative error of eu.pressure_perturbation(Theta' = x Thetabar) against the
    exact difference P(Thetabar + Theta') - P(Thetabar), for each x in xs."""
    Pb = float(eos_mp(Thb, ph))
    Thp = torch.tensor([x * Thb for x in xs], dtype=F64)
    got = eu.pressure_perturbation(Thp, torch.full_like(Thp, Thb), torch.full_like(Thp, Pb), ph.gamma)
    out = []
    with mp.workdps(50):
        for i in range(len(xs)):
            want = eos_mp(mp.mpf(Thb) + mp.mpf(float(Thp[i])), ph) - eos_mp(Thb, ph)
            out.append(float(abs((mp.mpf(float(got[i])) - want) / want)))
    return out


# ----------------------------------------------------------------------------- hydrostatic state of another theta

def rebased_hydrostatic(N, nz, theta1=330.0, H=10000.0, ph=None):
    """A neutral hydrostatic atmosphere of potential temperature theta1, at rest,
    written as a perturbation of the oracle's theta0 background.  It is an exact
    steady solution, so the discrete right-hand side is only the truncation error.
    One column of nz cubes of side H/nz, periodic in x and y, walls at z = 0, H.
    Returns max |R_v| per variable and the scales max |rho' g| and max |P'|."""
    ph = ph or eu.Phys()
    h = H / nz
    m = fo.build(fo.ForestDesc(N, 1, 1, nz, 0, (0.0, 0.0, 0.0), (h, h, H), (1, 1, 0)), None)
    op = eu.Operator(m, ph)
    _, _, Z = eu.node_xyz(m)
    R_gas = ph.cp - ph.cv
    exner1 = 1.0 - ph.g * Z / (ph.cp * theta1)
    rho1 = ph.P0 * exner1 ** (ph.cv / R_gas) / (R_gas * theta1)
    rho_b, Th_b, P_b = op.bg
    q = torch.stack([rho1 - rho_b, torch.zeros_like(Z), torch.zeros_like(Z), torch.zeros_like(Z),
                     rho1 * theta1 - Th_b])
    Rq = op.rhs(q)
    P1 = ph.P0 * exner1 ** (ph.cp / R_gas)
    return {"R_max": [float(Rq[v].abs().max()) for v in range(5)],
            "buoyancy_scale": float((q[0] * ph.g).abs().max()),
            "pprime_scale": float((P1 - P_b).abs().max()), "h": h}


# ----------------------------------------------------------------------------- isentropic vortex

VORTEX_PHYS = eu.Phys(cp=3.5, cv=2.5, P0=1.0, g=0.0, background=eu.BG_CONSTANT, rho0=1.0, Theta0=1.0)


def vortex_mesh(N, n, L=12.0, amr=False):
    """[-6, 6]^2 in n x n roots, extruded one cube thick along z; periodic.  With
    amr, the roots whose centre is within 3 of the vortex centre are refined once."""
    h = L / n
    desc = fo.ForestDesc(N, n, n, 1, 1 if amr else 0, (-L / 2, -L / 2, 0.0), (L / 2, L / 2, h), (1, 1, 1))
    m = fo.build(desc, None)
    if amr:
        lo, hh = fo.elem_lo_h(m)
        c = lo + 0.5 * hh
        fl = ((c[:, 0] ** 2 + c[:, 1] ** 2) < 9.0).astype(np.int8)
        m = fo.build(desc, m, fl, fo.PASS_REFINE)
    return m


def vortex_rhs_errors(N, n, amr=False):
    """max |R_v(q(0)) - dq_v/dt(0)| per variable, with the exact time derivative of
    the translating vortex from forward-mode differentiation of its formula in t,
    and max |dq_v/dt| for scale."""
    import torch.autograd.forward_ad as fwAD
    m = vortex_mesh(N, n, amr=amr)
    op = eu.Operator(m, VORTEX_PHYS)
    X, Y, _ = eu.node_xyz(m)
    q0 = eu.isentropic_vortex(X, Y, 0.0, gamma=VORTEX_PHYS.gamma)
    with fwAD.dual_level():
        t = fwAD.make_dual(torch.tensor(0.0, dtype=F64), torch.tensor(1.0, dtype=F64))
        dqdt = fwAD.unpack_dual(eu.isentropic_vortex(X, Y, t, gamma=VORTEX_PHYS.gamma)).tangent
    Rq = op.rhs(q0)
    return ([float((Rq[v] - dqdt[v]).abs().max()) for v in range(5)],
            [float(dqdt[v].abs().max()) for v in range(5)], len(m.hang))


def vortex_solution_errors(N, n, T, cfl=0.2):
    """L2 norm (LGL quadrature) of q_v(T) - q_v,exact(T) per variable after SSP-RK3
    steps to time T (Courant number cfl on the smallest node spacing at speed 3)."""
    m = vortex_mesh(N, n)
    op = eu.Operator(m, VORTEX_PHYS)
    X, Y, _ = eu.node_xyz(m)
    q = eu.isentropic_vortex(X, Y, 0.0, gamma=VORTEX_PHYS.gamma)
    xs = op.re.x
    dx = (12.0 / n) / 2.0 * float(xs[1] - xs[0])
    steps = int(math.ceil(T / (cfl * dx / 3.0)))
    for _ in range(steps):
        q = eu.ssp_rk3_step(op, T / steps, q)
    ex = eu.isentropic_vortex(X, Y, T, gamma=VORTEX_PHYS.gamma)
    JW = eu.quad_weights(op)
    return [float((JW * (q[v] - ex[v]) ** 2).sum().sqrt()) for v in range(5)]


# ----------------------------------------------------------------------------- manufactured state

def _mms_fields(X, Y, Z, ph, L):
    """Smooth full state on [0, L]^3, periodic in x and y, w = 0 on z = 0 and z = L,
    over the neutral background; returns (perturbation state, exact -div F + S),
    the latter by automatic differentiation of the physical fluxes written with
    the full pressure P = P0 (R Theta/P0)^gamma minus the analytic hydrostatic
    Pbar = P0 exner^(cp/R)."""
    Rg = ph.cp - ph.cv
    k, kz = 2 * math.pi / L, math.pi / L
    X, Y, Z = (t.detach().clone().requires_grad_(True) for t in (X, Y, Z))
    exner = 1.0 - ph.g * Z / (ph.cp * ph.theta0)
    rho_b = ph.P0 * exner ** (ph.cv / Rg) / (Rg * ph.theta0)
    P_b = ph.P0 * exner ** (ph.cp / Rg)
    rho = rho_b * (1.0 + 0.05 * (torch.sin(k * X) * torch.cos(k * Y) + 0.5 * torch.cos(kz * Z)))
    u = 1.5 + torch.sin(k * Y + 0.3)
    v = -0.5 + torch.cos(k * X) * torch.sin(kz * Z + 0.4)
    w = 0.8 * torch.sin(kz * Z) * torch.cos(k * X + 0.1)
    theta = ph.theta0 + 2.0 * torch.sin(k * X) * torch.sin(k * Y + 0.5) * torch.cos(kz * Z)
    Th = rho * theta
    P = ph.P0 * (Rg * Th / ph.P0) ** ph.gamma
    Pp = P - P_b
    vel = (u, v, w)
    mom = (rho * u, rho * v, rho * w)
    coords = (X, Y, Z)
    rhs = [torch.zeros_like(X) for _ in range(5)]
    for d in range(3):
        Fd = [mom[d]] + [mom[mm] * vel[d] + (Pp if mm == d else 0.0) for mm in range(3)] + [Th * vel[d]]
        for c in range(5):
            (g,) = torch.autograd.grad(Fd[c].sum(), coords[d], retain_graph=True)
            rhs[c] = rhs[c] - g
    rhs[3] = rhs[3] - (rho - rho_b) * ph.g
    Th_b = rho_b * ph.theta0
    q = torch.stack([rho - rho_b, mom[0], mom[1], mom[2], Th - Th_b]).detach()
    return q, torch.stack([r.detach() for r in rhs])


def mms_mesh(N, n, L=1000.0, amr=False):
    """n^3 roots on [0, L]^3, periodic in x and y, walls in z; with amr every root
    in the octant x, y, z < L/2 is refined once (hanging faces on three planes)."""
    desc = fo.ForestDesc(N, n, n, n, 1 if amr else 0, (0.0, 0.0, 0.0), (L, L, L), (1, 1, 0))
    m = fo.build(desc, None)
    if amr:
        lo, hh = fo.elem_lo_h(m)
        c = lo + 0.5 * hh
        fl = np.all(c < L / 2, axis=1).astype(np.int8)
        m = fo.build(desc, m, fl, fo.PASS_REFINE)
    return m


def mms_rhs_errors(N, n, amr=False, ph=None):
    """max |R_v(q) - (-div F + S)_v| per variable on the manufactured state, and the
    scale max |(-div F + S)_v|."""
    ph = ph or eu.Phys()
    m = mms_mesh(N, n, amr=amr)
    op = eu.Operator(m, ph)
    X, Y, Z = eu.node_xyz(m)
    q, exact = _mms_fields(X, Y, Z, ph, 1000.0)
    Rq = op.rhs(q)
    return ([float((Rq[v] - exact[v]).abs().max()) for v in range(5)],
            [float(exact[v].abs().max()) for v in range(5)], len(m.hang))


# ----------------------------------------------------------------------------- acoustic wave speed

def acoustic_speed(N=4, n=8, L=1000.0, T_kelvin=300.0, amp=1e-6, ph=None):
    """Speed of sound measured from a standing acoustic wave in a uniform
    atmosphere at rest at temperature T (pressure P0, no gravity), periodic along
    x: rho' = amp rhobar sin(kx), Theta' = amp Thetabar sin(kx) (isentropic), U = 0.
    rho'(t) = amp rhobar sin(kx) cos(c k t) to first order, so c is read from the
    projection of rho'(T1) on sin(kx) at T1 near a quarter period."""
    ph0 = ph or eu.Phys()
    Rg = ph0.cp - ph0.cv
    rho0 = ph0.P0 / (Rg * T_kelvin)           # P = P0 at T: R Theta / P0 = 1
    Th0 = ph0.P0 / Rg
    ph = eu.Phys(cp=ph0.cp, cv=ph0.cv, P0=ph0.P0, g=0.0, background=eu.BG_CONSTANT, rho0=rho0, Theta0=Th0)
    h = L / n
    m = fo.build(fo.ForestDesc(N, n, 1, 1, 0, (0.0, 0.0, 0.0), (L, h, h), (1, 1, 1)), None)
    op = eu.Operator(m, ph)
    X, _, _ = eu.node_xyz(m)
    k = 2 * math.pi / L
    s = torch.sin(k * X)
    z = torch.zeros_like(X)
    q = torch.stack([amp * rho0 * s, z, z, z, amp * Th0 * s])
    JW = eu.quad_weights(op)
    proj0 = float((JW * q[0] * s).sum())
    c_guess = 340.0
    T1 = 0.5 * math.pi / (c_guess * k) * 0.8    # ~0.8 of a quarter period: cos well away from 0 and 1
    dx = h / 2.0 * float(op.re.x[1] - op.re.x[0])
    steps = int(math.ceil(T1 / (0.3 * dx / c_guess)))
    for _ in range(steps):
        q = eu.ssp_rk3_step(op, T1 / steps, q)
    ratio = float((JW * q[0] * s).sum()) / proj0
    ratio = min(1.0, max(-1.0, ratio))
    return math.acos(ratio) / (k * T1)


# ----------------------------------------------------------------------------- Rusanov wave speed

def rusanov_wave_speed(N, qL, qR, h=100.0, ph=None):
    """Two elements side by side along x, each holding a constant state (walls in
    x, periodic in y and z), so the only non-zero part of R_rho at the shared face
    is the Rusanov dissipation: at the minus element's face nodes
    R_rho = -lift (1/2 (F_rho(qR) - F_rho(qL)) + 1/2 lambda (rho'_L - rho'_R)),
    lift = (2/h) N (N + 1)/2.  qL and qR are 5-tuples with the same rho u (so the
    F_rho difference vanishes).  Returns lambda read back from R at every face
    node of the minus element (an array)."""
    ph = ph or eu.Phys(g=0.0, background=eu.BG_CONSTANT, rho0=1.2, Theta0=360.0)
    m = fo.build(fo.ForestDesc(N, 2, 1, 1, 0, (0.0, 0.0, 0.0), (2 * h, h, h), (0, 1, 1)), None)
    op = eu.Operator(m, ph)
    n1 = N + 1
    q = torch.zeros(5, 2, n1, n1, n1, dtype=F64)
    for v in range(5):
        q[v, 0] = qL[v]
        q[v, 1] = qR[v]
    Rq = op.rhs(q)
    lift = (2.0 / h) * N * (N + 1) / 2.0
    face = Rq[0, 0, :, :, N]                   # minus element, face x = h (i = N)
    return (-2.0 * face / (lift * (qL[0] - qR[0]))).reshape(-1).numpy()


def max_wave_speed_mp(qs, ph):
    """max over the states of |u_x| + c, c = sqrt(gamma P / rho), with P from the
    50-digit equation of state of the full Theta = Thetabar + Theta'."""
    best = None
    with mp.workdps(50):
        for q in qs:
            rho = mp.mpf(ph.rho0) + mp.mpf(q[0])
            Th = mp.mpf(ph.Theta0) + mp.mpf(q[4])
            P = eos_mp(Th, ph)
            c = mp.sqrt(mp.mpf(ph.gamma) * P / rho)
            lam = abs(mp.mpf(q[1]) / rho) + c
            best = lam if best is None or lam > best else best
    return float(best)
