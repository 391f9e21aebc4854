"""Oracle: compressible Euler in hydrostatic-perturbation form, strong-form
dGSEM with Rusanov fluxes and L2 mortars, SSP-RK3 stage, budgets, adaptation
indicator and conservative refine/coarsen transfer (test infrastructure only).

Plain PyTorch CPU float64 code written from the paper's statements:

* Equations (section 2.1): q = (rho, U = rho u, Theta = rho theta); fluxes
  (U, U u^T + P I, Theta u); source (0, F, 0) with F the buoyancy; equation of
  state P = P0 (R Theta / P0)^gamma, R = cp - cv, gamma = cp/cv; density and
  pressure written as perturbations about a hydrostatic background
  rho = rhobar(z) + rho', P = Pbar(z) + P'.
* Strong form (section 2.2): d q/dt = -div F + S - lift of (F* - F).n on the
  element boundary; LGL collocation with the diagonal mass matrix.
* Rusanov flux (section 2.2): F* = {F} + n |c|/2 [[q]].
* Mortars (section 3.3): the coarse face trace is projected onto the two
  half-interval mortars per tangential axis (the fine side projection is the
  identity), the Rusanov flux is evaluated at the mortar points and it is
  projected back with sum_i s_i M^{-1} S^T, s_i = 1/2 per axis.
* Pointwise matching (section 3.3, the simpler alternative the paper compares
  the mortars with; ``Operator(..., nonconforming="pointwise")``): each side
  solves the Riemann problem at its own face nodes against the other side's
  polynomial evaluated there, with no projection, so the two sides' fluxes do
  not balance and the scheme loses discrete conservation.
* Conservative coarsening by LGL integration and refinement by the same
  tensor-product projection matrices (section 3.3).

Readings where the paper is silent (each is listed in the design notes):

* The state carried is the perturbation q' = (rho', U, V, W, Theta'); the
  momentum flux carries P' and the momentum source is the buoyancy -rho' g on
  W, so a rest state q' = 0 has a right-hand side that is exactly zero.
* P' = Pbar * expm1(gamma * log1p(Theta'/Thetabar)), the cancellation-free
  form of P(Thetabar + Theta') - P(Thetabar).
* |c| in the Rusanov flux is the local maximum wave speed
  lambda = max(|u.n| + c) over both sides, c = sqrt(gamma P / rho); the jump is
  taken on the perturbation variables, with the dissipative sign q'- - q'+.
* No-flux walls use the mirror state (rho', U - 2 (U.n) n, Theta').
* Background on a mortar is that of the fine face nodes.
* Pointwise matching: the fine side is the mortar method's fine side (the
  coarse polynomial at the fine nodes); at a coarse node the fine polynomial of
  the quadrant containing it, the average of the two (four) quadrants on a
  shared mid-line (mid-point), against the coarse trace with the coarse node's
  background.
* Lift: at a face node the boundary integral divided by the LGL volume weight
  gives R -= (2/h_d) / w_N * (F*.n - F(q-).n), w_N = 2/(N(N+1)).

Array layout: fields are torch float64 tensors [5, K, N+1, N+1, N+1] indexed
[v][e][k][j][i] (node n = i + (N+1)(j + (N+1) k), x fastest); variables
v = (rho', rhou, rhov, rhow, Theta').
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import forest as fo
from .refelem import refelem

F64 = torch.float64

BG_NEUTRAL = 0
BG_CONSTANT = 1


@dataclass(frozen=True)
class Phys:
    """Gas constants and background.  Defaults: cp, cv chosen so that the
    sound speed at 300 K is 347.3 m/s, the value the paper quotes (section
    4.4); g and P0 are the usual constants."""
    cp: float = 1004.67
    cv: float = 717.5
    P0: float = 1.0e5
    g: float = 9.80616
    background: int = BG_NEUTRAL
    theta0: float = 300.0
    rho0: float = 1.0
    Theta0: float = 300.0
    mu: float = 0.0          # artificial viscosity (m^2/s), 0: none

    @property
    def R(self):
        return self.cp - self.cv

    @property
    def gamma(self):
        return self.cp / self.cv


# ----------------------------------------------------------------------------- geometry helpers

def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=F64)


def node_xyz(mesh: fo.Mesh):
    """Node coordinates as three tensors [K, N+1, N+1, N+1] (x, y, z)."""
    re = refelem(mesh.N)
    c = fo.node_coords_1d(mesh, re.x)  # [3, K, N+1]
    n1 = mesh.N + 1
    X = _t(c[0])[:, None, None, :].expand(-1, n1, n1, n1)
    Y = _t(c[1])[:, None, :, None].expand(-1, n1, n1, n1)
    Z = _t(c[2])[:, :, None, None].expand(-1, n1, n1, n1)
    return X, Y, Z


def background(mesh: fo.Mesh, phys: Phys):
    """(rhobar, Thetabar, Pbar) at every node, tensors [K, N+1, N+1, N+1].

    Neutral atmosphere with constant theta0 (section 4.3):
    Exner pi = 1 - g z / (cp theta0), P = P0 pi^(cp/R), rho = P0 pi^(cv/R) / (R theta0);
    Thetabar = rhobar theta0 and Pbar taken from the equation of state."""
    _, _, Z = node_xyz(mesh)
    R, gam = phys.R, phys.gamma
    if phys.background == BG_NEUTRAL:
        exner = 1.0 - phys.g * Z / (phys.cp * phys.theta0)
        rho_b = phys.P0 * exner ** (phys.cv / R) / (R * phys.theta0)
        Th_b = rho_b * phys.theta0
    elif phys.background == BG_CONSTANT:
        rho_b = torch.full_like(Z, phys.rho0)
        Th_b = torch.full_like(Z, phys.Theta0)
    else:
        raise ValueError("unknown background")
    P_b = phys.P0 * (R * Th_b / phys.P0) ** gam
    return rho_b, Th_b, P_b


# ----------------------------------------------------------------------------- pointwise physics

def pressure_perturbation(Thp, Th_b, P_b, gamma):
    """P' = P(Thetabar + Theta') - Pbar written as Pbar expm1(gamma log1p(Theta'/Thetabar))."""
    return P_b * torch.expm1(gamma * torch.log1p(Thp / Th_b))


def primitives(q, bg, phys):
    """Full density, velocity, P' and P from the perturbation state."""
    rho_b, Th_b, P_b = bg
    rho = rho_b + q[0]
    u = (q[1] / rho, q[2] / rho, q[3] / rho)
    Pp = pressure_perturbation(q[4], Th_b, P_b, phys.gamma)
    return rho, u, Pp, P_b + Pp


def flux_dir(q, bg, phys, d):
    """F^d(q) (5 components) along axis d, with P' in the momentum flux."""
    rho, u, Pp, _ = primitives(q, bg, phys)
    Th = bg[1] + q[4]
    comps = [q[1 + d]]
    for m in range(3):
        c = q[1 + m] * u[d]
        if m == d:
            c = c + Pp
        comps.append(c)
    comps.append(Th * u[d])
    return torch.stack(comps)


def sound_speed(rho, P, gamma):
    return torch.sqrt(gamma * P / rho)


def rusanov(qL, bgL, qR, bgR, phys, d, sgn):
    """F*.n for n = sgn e_d: {F.n} + 1/2 lambda (q'- - q'+), lambda = max |u.n| + c."""
    rhoL, uL, _, PL = primitives(qL, bgL, phys)
    rhoR, uR, _, PR = primitives(qR, bgR, phys)
    FL = flux_dir(qL, bgL, phys, d) * sgn
    FR = flux_dir(qR, bgR, phys, d) * sgn
    lamL = torch.abs(uL[d]) + sound_speed(rhoL, PL, phys.gamma)
    lamR = torch.abs(uR[d]) + sound_speed(rhoR, PR, phys.gamma)
    lam = torch.maximum(lamL, lamR)
    return 0.5 * (FL + FR) + 0.5 * lam * (qL - qR)


# ----------------------------------------------------------------------------- face traces

def face_slice(t, f, N):
    """Trace of t[..., K, k, j, i] on face f = 2d+s -> [..., K, (N+1)^2], m = a + (N+1) b."""
    d, s = f // 2, f % 2
    idx = N if s == 1 else 0
    if d == 0:
        tr = t[..., idx]           # [.., K, k, j]  (b = k, a = j)
    elif d == 1:
        tr = t[..., idx, :]        # [.., K, k, i]  (b = k, a = i)
    else:
        tr = t[..., idx, :, :]     # [.., K, j, i]  (b = j, a = i)
    return tr.reshape(*tr.shape[:-2], (N + 1) ** 2)


def face_embed(delta, f, N, K):
    """Inverse of face_slice: zeros everywhere except face f which holds delta."""
    d, s = f // 2, f % 2
    idx = N if s == 1 else 0
    n1 = N + 1
    out = torch.zeros(delta.shape[0], K, n1, n1, n1, dtype=delta.dtype)
    sq = delta.reshape(delta.shape[0], K, n1, n1)
    if d == 0:
        out[..., idx] = sq
    elif d == 1:
        out[..., idx, :] = sq
    else:
        out[..., idx, :, :] = sq
    return out


def interp2(Ia, Ib, tr, N):
    """(I_a (x) I_b) applied to face data [..., (N+1)^2] with m = a + (N+1) b."""
    n1 = N + 1
    t = tr.reshape(*tr.shape[:-1], n1, n1)          # [.., b, a]
    t = torch.einsum('pb,...ba->...pa', Ib, t)
    t = torch.einsum('qa,...pa->...pq', Ia, t)
    return t.reshape(*tr.shape[:-1], n1 * n1)


# ----------------------------------------------------------------------------- operator

class Operator:
    """Geometry and tables of one mesh, prepared once (plain tensors)."""

    def __init__(self, mesh: fo.Mesh, phys: Phys, nonconforming: str = "mortar"):
        if nonconforming not in ("mortar", "pointwise"):
            raise ValueError("nonconforming must be 'mortar' or 'pointwise'")
        # a hydrostatic background that varies with z cannot be periodic in z
        if mesh.desc.periodic[2] and phys.background == BG_NEUTRAL and phys.g != 0.0:
            raise ValueError("a periodic z axis needs a background constant in z (g = 0 or BG_CONSTANT)")
        self.mesh, self.phys = mesh, phys
        self.nonconforming = nonconforming
        N = mesh.N
        self.N, self.K = N, mesh.K
        re = refelem(N)
        self.re = re
        self.D = _t(re.D)
        self.I = [_t(re.I[0]), _t(re.I[1])]
        self.Rm = [_t(re.R[0]), _t(re.R[1])]
        self.P = [_t(re.P[0]), _t(re.P[1])]
        self.wN = 2.0 / (N * (N + 1))
        _, h = fo.elem_lo_h(mesh)
        self.h = _t(h)                       # [K, 3]
        self.bg = background(mesh, phys)
        self.conf = torch.as_tensor(mesh.conf, dtype=torch.long)
        self.bnd = torch.as_tensor(mesh.bnd, dtype=torch.long)
        self.hang = torch.as_tensor(mesh.hang, dtype=torch.long)

    # volume term: -sum_d (2/h_d) D_d F^d + S   (section 2.2 strong form)
    def volume(self, q):
        ph = self.phys
        g2 = 2.0 / self.h                    # [K, 3]
        Fx = flux_dir(q, self.bg, ph, 0)
        Fy = flux_dir(q, self.bg, ph, 1)
        Fz = flux_dir(q, self.bg, ph, 2)
        dFx = torch.einsum('im,vekjm->vekji', self.D, Fx)
        dFy = torch.einsum('jm,vekmi->vekji', self.D, Fy)
        dFz = torch.einsum('km,vemji->vekji', self.D, Fz)
        R = -(g2[None, :, 0, None, None, None] * dFx
              + g2[None, :, 1, None, None, None] * dFy
              + g2[None, :, 2, None, None, None] * dFz)
        buoy = -q[0] * ph.g
        R = R + torch.stack([torch.zeros_like(buoy), torch.zeros_like(buoy),
                             torch.zeros_like(buoy), buoy, torch.zeros_like(buoy)])
        return R

    def _trace(self, q, f, elems):
        N = self.N
        qt = face_slice(q, f, N)[:, elems]
        bgt = tuple(face_slice(b, f, N)[elems] for b in self.bg)
        return qt, bgt

    def surface(self, q):
        """Face contributions (F*.n - F(q-).n) per element face, lifted into R."""
        N, K, ph = self.N, self.K, self.phys
        nf = (N + 1) ** 2
        delta = [torch.zeros(5, K, nf, dtype=F64) for _ in range(6)]
        lift = 2.0 / self.wN / self.h        # (2/h_d)/w_N, [K, 3]

        # conforming faces: minus element's plus face, plus element's minus face
        for d in range(3):
            sel = self.conf[:, 2] == d
            if not bool(sel.any()):
                continue
            eM, eP = self.conf[sel, 0], self.conf[sel, 1]
            qL, bL = self._trace(q, 2 * d + 1, eM)
            qR, bR = self._trace(q, 2 * d, eP)
            Fs = rusanov(qL, bL, qR, bR, ph, d, 1.0)                # F*.n, n = +e_d
            dM = Fs - flux_dir(qL, bL, ph, d)
            dP = -Fs + flux_dir(qR, bR, ph, d)                       # n = -e_d
            delta[2 * d + 1] = delta[2 * d + 1].index_add(1, eM, dM)
            delta[2 * d] = delta[2 * d].index_add(1, eP, dP)

        # no-flux walls: mirror state
        for f in range(6):
            sel = self.bnd[:, 1] == f
            if not bool(sel.any()):
                continue
            d, s = f // 2, f % 2
            sgn = 1.0 if s == 1 else -1.0
            e = self.bnd[sel, 0]
            qL, bL = self._trace(q, f, e)
            qR = torch.stack([qL[0]] + [(-qL[1 + m] if m == d else qL[1 + m]) for m in range(3)]
                             + [qL[4]])
            Fs = rusanov(qL, bL, qR, bL, ph, d, sgn)
            delta[f] = delta[f].index_add(1, e, Fs - sgn * flux_dir(qL, bL, ph, d))

        # hanging faces: mortars (section 3.3)
        for f in range(6):
            sel = self.hang[:, 1] == f
            if not bool(sel.any()):
                continue
            d, s = f // 2, f % 2
            sgn = 1.0 if s == 1 else -1.0
            fo_ = 2 * d + (1 - s)                                    # fine side face
            ec = self.hang[sel, 0]
            qc, bc = self._trace(q, f, ec)
            proj = torch.zeros_like(qc)   # mortar: projected flux; pointwise: fine state at coarse nodes
            for quad in range(4):
                a, b = quad & 1, quad >> 1
                ef = self.hang[sel, 2 + quad]
                qf, bf = self._trace(q, fo_, ef)
                qm = interp2(self.I[a], self.I[b], qc, N)             # coarse -> mortar
                Fs = rusanov(qm, bf, qf, bf, ph, d, sgn)             # F*.n_c on mortar
                if self.nonconforming == "mortar":
                    proj = proj + interp2(self.Rm[a], self.Rm[b], Fs, N)  # mortar -> coarse
                else:
                    proj = proj + interp2(self.P[a], self.P[b], qf, N)    # fine polynomial at coarse nodes
                dF = -Fs + sgn * flux_dir(qf, bf, ph, d)             # fine side, n_f = -n_c
                delta[fo_] = delta[fo_].index_add(1, ef, dF)
            if self.nonconforming == "pointwise":
                proj = rusanov(qc, bc, proj, bc, ph, d, sgn)         # F*.n_c at the coarse nodes
            delta[f] = delta[f].index_add(1, ec, proj - sgn * flux_dir(qc, bc, ph, d))

        R = torch.zeros(5, K, N + 1, N + 1, N + 1, dtype=F64)
        for f in range(6):
            d = f // 2
            R = R - face_embed(delta[f] * lift[None, :, d, None], f, N, K)
        return R

    def rhs(self, q):
        R = self.volume(q) + self.surface(q)
        if self.phys.mu > 0.0:
            R = R + self.viscous(q)
        return R

    # ------------------------------------------------------------------ artificial viscosity
    def _central_face_terms(self, X, which, wall_zero_flux):
        """Lifted face terms lift * sgn * (X* - X-) of a 5-variable field on the faces
        normal to axis d of every leaf, for X = which(d) (a tensor [5, K, ...]):
        X* = 1/2 (X- + X+) at conforming faces; at walls X* = X- (gradient pass) or
        X*.n = 0 (flux pass, wall_zero_flux); on hanging faces the central average is
        formed on the mortars, (I_a x I_b) X_coarse with X_fine, the fine side takes it
        there and the coarse side its projection sum_ab (R_a x R_b).  Returns the
        contributions embedded at the face nodes, [3][5, K, ...] (one per axis)."""
        N, K = self.N, self.K
        nf = (N + 1) ** 2
        lift = 2.0 / self.wN / self.h
        out = []
        for d in range(3):
            Xd = which(d)
            delta = {f: torch.zeros(5, K, nf, dtype=F64) for f in (2 * d, 2 * d + 1)}
            sel = self.conf[:, 2] == d
            if bool(sel.any()):
                eM, eP = self.conf[sel, 0], self.conf[sel, 1]
                XL = face_slice(Xd, 2 * d + 1, N)[:, eM]
                XR = face_slice(Xd, 2 * d, N)[:, eP]
                avg = 0.5 * (XL + XR)
                delta[2 * d + 1] = delta[2 * d + 1].index_add(1, eM, avg - XL)      # sgn = +1
                delta[2 * d] = delta[2 * d].index_add(1, eP, -(avg - XR))          # sgn = -1
            for f in (2 * d, 2 * d + 1):
                sgn = 1.0 if f % 2 else -1.0
                sel = self.bnd[:, 1] == f
                if bool(sel.any()) and wall_zero_flux:
                    e = self.bnd[sel, 0]
                    Xw = face_slice(Xd, f, N)[:, e]
                    delta[f] = delta[f].index_add(1, e, sgn * (0.0 - Xw))
                sel = self.hang[:, 1] == f
                if not bool(sel.any()):
                    continue
                fo_ = f ^ 1
                ec = self.hang[sel, 0]
                Xc = face_slice(Xd, f, N)[:, ec]
                proj = torch.zeros_like(Xc)
                for quad in range(4):
                    a, b = quad & 1, quad >> 1
                    ef = self.hang[sel, 2 + quad]
                    Xf = face_slice(Xd, fo_, N)[:, ef]
                    avg = 0.5 * (interp2(self.I[a], self.I[b], Xc, N) + Xf)
                    proj = proj + interp2(self.Rm[a], self.Rm[b], avg, N)
                    delta[fo_] = delta[fo_].index_add(1, ef, -sgn * (avg - Xf))    # n_f = -n_c
                delta[f] = delta[f].index_add(1, ec, sgn * (proj - Xc))
            T = torch.zeros(5, K, N + 1, N + 1, N + 1, dtype=F64)
            for f in (2 * d, 2 * d + 1):
                T = T + face_embed(delta[f] * lift[None, :, d, None], f, N, K)
            out.append(T)
        return out

    def viscous(self, q):
        """Artificial viscosity div(mu grad q') of every perturbation variable (section
        4.3 applies mu = 1.5 m^2/s to the rising bubble; the form is a reading), by the
        two-pass central scheme: sigma_d = (2/h_d) D_d q' + lifted (q* - q-) n_d, then
        R = (2/h_d) D_d (mu sigma_d) + lifted (G* - G-).n; walls carry no diffusive flux."""
        mu = self.phys.mu
        g2 = 2.0 / self.h
        dq = [torch.einsum('im,vekjm->vekji', self.D, q), torch.einsum('jm,vekmi->vekji', self.D, q),
              torch.einsum('km,vemji->vekji', self.D, q)]
        Tq = self._central_face_terms(q, lambda d: q, wall_zero_flux=False)
        sigma = [g2[None, :, d, None, None, None] * dq[d] + Tq[d] for d in range(3)]
        G = [mu * s for s in sigma]
        dG = [torch.einsum('im,vekjm->vekji', self.D, G[0]), torch.einsum('jm,vekmi->vekji', self.D, G[1]),
              torch.einsum('km,vemji->vekji', self.D, G[2])]
        TG = self._central_face_terms(None, lambda d: G[d], wall_zero_flux=True)
        return sum(g2[None, :, d, None, None, None] * dG[d] + TG[d] for d in range(3))


# ----------------------------------------------------------------------------- passive tracer

def tracer_flux_dir(q, C, bg, phys, d):
    """Tracer flux C u_d along axis d (section 2.1: the flux of C = rho c is C U / rho)."""
    rho, u, _, _ = primitives(q, bg, phys)
    return C * u[d]


def tracer_rusanov(qL, CL, bgL, qR, CR, bgR, phys, d, sgn):
    """Tracer part of the Rusanov flux for n = sgn e_d: {C u.n} + 1/2 lambda (C- - C+),
    with lambda the same local maximum wave speed as the Euler system's flux."""
    rhoL, uL, _, PL = primitives(qL, bgL, phys)
    rhoR, uR, _, PR = primitives(qR, bgR, phys)
    lamL = torch.abs(uL[d]) + sound_speed(rhoL, PL, phys.gamma)
    lamR = torch.abs(uR[d]) + sound_speed(rhoR, PR, phys.gamma)
    lam = torch.maximum(lamL, lamR)
    FL = sgn * CL * uL[d]
    FR = sgn * CR * uR[d]
    return 0.5 * (FL + FR) + 0.5 * lam * (CL - CR)


def tracer_rhs(op: Operator, q, C):
    """R_C(q, C): the strong-form dGSEM right-hand side of the tracer equation
    dC/dt + div(C u) = 0 (section 2.1), u = U/rho from the Euler state q, with the
    same Rusanov flux, mirror walls (no tracer flux through a wall) and the same
    hanging-face scheme (mortars or pointwise matching) as the Euler operator.
    C is [K, N+1, N+1, N+1]; so is the result."""
    N, K, ph = op.N, op.K, op.phys
    nf = (N + 1) ** 2
    g2 = 2.0 / op.h
    # volume: -sum_d (2/h_d) D_d (C u_d)
    Fx = tracer_flux_dir(q, C, op.bg, ph, 0)
    Fy = tracer_flux_dir(q, C, op.bg, ph, 1)
    Fz = tracer_flux_dir(q, C, op.bg, ph, 2)
    R = -(g2[:, 0, None, None, None] * torch.einsum('im,ekjm->ekji', op.D, Fx)
          + g2[:, 1, None, None, None] * torch.einsum('jm,ekmi->ekji', op.D, Fy)
          + g2[:, 2, None, None, None] * torch.einsum('km,emji->ekji', op.D, Fz))
    delta = [torch.zeros(K, nf, dtype=F64) for _ in range(6)]
    lift = 2.0 / op.wN / op.h

    def trace(f, elems):
        qt, bgt = op._trace(q, f, elems)
        return qt, face_slice(C[None], f, N)[0][elems], bgt

    for d in range(3):
        sel = op.conf[:, 2] == d
        if not bool(sel.any()):
            continue
        eM, eP = op.conf[sel, 0], op.conf[sel, 1]
        qL, cL, bL = trace(2 * d + 1, eM)
        qR, cR, bR = trace(2 * d, eP)
        Fs = tracer_rusanov(qL, cL, bL, qR, cR, bR, ph, d, 1.0)
        delta[2 * d + 1] = delta[2 * d + 1].index_add(0, eM, Fs - tracer_flux_dir(qL, cL, bL, ph, d))
        delta[2 * d] = delta[2 * d].index_add(0, eP, -Fs + tracer_flux_dir(qR, cR, bR, ph, d))
    for f in range(6):
        sel = op.bnd[:, 1] == f
        if not bool(sel.any()):
            continue
        d, s = f // 2, f % 2
        sgn = 1.0 if s == 1 else -1.0
        e = op.bnd[sel, 0]
        qL, cL, bL = trace(f, e)
        qR = torch.stack([qL[0]] + [(-qL[1 + m] if m == d else qL[1 + m]) for m in range(3)] + [qL[4]])
        Fs = tracer_rusanov(qL, cL, bL, qR, cL, bL, ph, d, sgn)
        delta[f] = delta[f].index_add(0, e, Fs - sgn * tracer_flux_dir(qL, cL, bL, ph, d))
    for f in range(6):
        sel = op.hang[:, 1] == f
        if not bool(sel.any()):
            continue
        d, s = f // 2, f % 2
        sgn = 1.0 if s == 1 else -1.0
        fo_ = 2 * d + (1 - s)
        ec = op.hang[sel, 0]
        qc, cc, bc = trace(f, ec)
        proj = torch.zeros_like(cc)          # mortar: projected flux; pointwise: fine C at coarse nodes
        projq = torch.zeros_like(qc)         # pointwise: fine state at coarse nodes
        for quad in range(4):
            a, b = quad & 1, quad >> 1
            ef = op.hang[sel, 2 + quad]
            qf, cf, bf = trace(fo_, ef)
            qm = interp2(op.I[a], op.I[b], qc, N)
            cm = interp2(op.I[a], op.I[b], cc, N)
            Fs = tracer_rusanov(qm, cm, bf, qf, cf, bf, ph, d, sgn)      # F*.n_c on the mortar
            if op.nonconforming == "mortar":
                proj = proj + interp2(op.Rm[a], op.Rm[b], Fs, N)
            else:
                proj = proj + interp2(op.P[a], op.P[b], cf, N)
                projq = projq + interp2(op.P[a], op.P[b], qf, N)
            delta[fo_] = delta[fo_].index_add(0, ef, -Fs + sgn * tracer_flux_dir(qf, cf, bf, ph, d))
        if op.nonconforming == "pointwise":
            proj = tracer_rusanov(qc, cc, bc, projq, proj, bc, ph, d, sgn)
        delta[f] = delta[f].index_add(0, ec, proj - sgn * tracer_flux_dir(qc, cc, bc, ph, d))
    for f in range(6):
        d = f // 2
        R = R - face_embed((delta[f] * lift[:, d, None])[None], f, N, K)[0]
    return R


def tracer_stage(op: Operator, a, b, dt, qs, C0, Cs):
    """C_out = a C0 + b (Cs + dt R_C(qs, Cs)): the tracer part of one Shu-Osher
    stage, with the Euler stage input qs supplying the velocity."""
    return a * C0 + b * (Cs + dt * tracer_rhs(op, qs, Cs))


def tracer_mass(op: Operator, C):
    """Integral of C (exactly rounded sum of J_e W_n C)."""
    return math.fsum((quad_weights(op) * C).reshape(-1).tolist())


def rhs(mesh, phys, q):
    return Operator(mesh, phys).rhs(q)


def rk_stage(op: Operator, a, b, dt, q0, qs):
    """q_out = a q0 + b (qs + dt R(qs)) (one Shu-Osher stage)."""
    return a * q0 + b * (qs + dt * op.rhs(qs))


SSP_RK3 = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def ssp_rk3_step(op: Operator, dt, q):
    q1 = rk_stage(op, *SSP_RK3[0], dt, q, q)
    q2 = rk_stage(op, *SSP_RK3[1], dt, q, q1)
    return rk_stage(op, *SSP_RK3[2], dt, q, q2)


# ----------------------------------------------------------------------------- budgets

def quad_weights(op: Operator):
    """J_e W_n at every node: (h_x h_y h_z / 8) w_i w_j w_k, tensor [K, N+1, N+1, N+1]."""
    w = _t(op.re.w)
    J = op.h.prod(dim=1) / 8.0
    return J[:, None, None, None] * w[:, None, None] * w[None, :, None] * w[None, None, :]


def budgets(op: Operator, q):
    """(mass', total mass, integral of Theta', energy), each an exactly rounded sum.

    Energy density: P/(gamma - 1) + |U|^2/(2 rho) + rho g z (a reading; the
    paper reports only its relative change)."""
    ph = op.phys
    JW = quad_weights(op)
    rho_b, Th_b, P_b = op.bg
    _, _, Z = node_xyz(op.mesh)
    rho = rho_b + q[0]
    Pp = pressure_perturbation(q[4], Th_b, P_b, ph.gamma)
    P = P_b + Pp
    E = P / (ph.gamma - 1.0) + (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / (2.0 * rho) + rho * ph.g * Z

    def fsum(t):
        return math.fsum(t.detach().reshape(-1).tolist())

    return (fsum(JW * q[0]), fsum(JW * rho), fsum(JW * q[4]), fsum(JW * E))


# ----------------------------------------------------------------------------- indicator

IND_THETA = 0
IND_GRAD_THETA = 1


def indicator(op: Operator, q, kind=IND_THETA):
    """Per-leaf eta: max over nodes of |theta'| (kind 0) or of |grad theta| (kind 1).

    theta' = (Thetabar + Theta')/(rhobar + rho') - Thetabar/rhobar."""
    rho_b, Th_b, _ = op.bg
    theta = (Th_b + q[4]) / (rho_b + q[0])
    if kind == IND_THETA:
        val = torch.abs(theta - Th_b / rho_b)
    else:
        g2 = 2.0 / op.h
        tx = torch.einsum('im,ekjm->ekji', op.D, theta) * g2[:, 0, None, None, None]
        ty = torch.einsum('jm,ekmi->ekji', op.D, theta) * g2[:, 1, None, None, None]
        tz = torch.einsum('km,emji->ekji', op.D, theta) * g2[:, 2, None, None, None]
        val = torch.sqrt(tx * tx + ty * ty + tz * tz)
    return val.reshape(op.K, -1).max(dim=1).values


def flags_from_indicator(mesh: fo.Mesh, eta, thr):
    """+1 where eta > thr and l < Lmax; -1 where eta <= thr and l > 0; else 0."""
    lev = mesh.levels()
    eta = np.asarray(eta)
    fl = np.zeros(mesh.K, dtype=np.int8)
    fl[(eta > thr) & (lev < mesh.desc.max_level)] = 1
    fl[(eta <= thr) & (lev > 0)] = -1
    return fl


# ----------------------------------------------------------------------------- transfer

def _apply3(A, B, C, t):
    """(C (x) B (x) A) on element data [..., k, j, i]: A acts on i, B on j, C on k."""
    t = torch.einsum('im,...kjm->...kji', A, t)
    t = torch.einsum('jm,...kmi->...kji', B, t)
    return torch.einsum('km,...mji->...kji', C, t)


def refine_project(mesh_to: fo.Mesh, q_from):
    """Children get (I_a (x) I_b (x) I_c) of the parent; kept leaves are copied."""
    re = refelem(mesh_to.N)
    I = [_t(re.I[0]), _t(re.I[1])]
    out = []
    for e in range(mesh_to.K):
        src, kind = int(mesh_to.xfer_src[e]), int(mesh_to.xfer_kind[e])
        qp = q_from[:, src]
        if kind == fo.KIND_COPY:
            out.append(qp)
        else:
            a, b, c = kind & 1, (kind >> 1) & 1, (kind >> 2) & 1
            out.append(_apply3(I[a], I[b], I[c], qp))
    return torch.stack(out, dim=1)


def coarsen_project(mesh_to: fo.Mesh, q_from):
    """Parents get sum over children of (R_a (x) R_b (x) R_c) q_child; kept leaves copied."""
    re = refelem(mesh_to.N)
    Rm = [_t(re.R[0]), _t(re.R[1])]
    out = []
    for e in range(mesh_to.K):
        src, kind = int(mesh_to.xfer_src[e]), int(mesh_to.xfer_kind[e])
        if kind == fo.KIND_COPY:
            out.append(q_from[:, src])
        else:
            acc = 0.0
            for c in range(8):
                a, b, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
                acc = acc + _apply3(Rm[a], Rm[b], Rm[cc], q_from[:, src + c])
            out.append(acc)
    return torch.stack(out, dim=1)


def _transfer_adjoint(forward, mesh_to: fo.Mesh, qbar_to, K_from):
    N1 = mesh_to.N + 1
    x = torch.zeros(5, K_from, N1, N1, N1, dtype=torch.float64, requires_grad=True)
    (g,) = torch.autograd.grad(forward(mesh_to, x), x, grad_outputs=qbar_to)
    return g


def refine_project_adjoint(mesh_to: fo.Mesh, qbar_to, K_from):
    """P^T qbar_to for the (linear) refine transfer P onto mesh_to from K_from
    source leaves, in the Euclidean inner product on the DOF vectors, by
    reverse-mode differentiation of ``refine_project``."""
    return _transfer_adjoint(refine_project, mesh_to, qbar_to, K_from)


def coarsen_project_adjoint(mesh_to: fo.Mesh, qbar_to, K_from):
    """P^T qbar_to for the (linear) coarsen transfer onto mesh_to, as above."""
    return _transfer_adjoint(coarsen_project, mesh_to, qbar_to, K_from)


# ----------------------------------------------------------------------------- adjoint and JVP

def rhs_adjoint(op: Operator, q, lam):
    """qbar = (dR/dq)^T lam in the Euclidean inner product on the DOF vector,
    by reverse-mode differentiation of ``Operator.rhs``.  Conventions at the
    non-smooth points follow PyTorch: d|x|/dx = 0 at 0 and a max tie splits
    the derivative 1/2, 1/2."""
    qv = q.detach().clone().requires_grad_(True)
    R = op.rhs(qv)
    (g,) = torch.autograd.grad(R, qv, grad_outputs=lam)
    return g


def rhs_jvp(op: Operator, q, v):
    """J v = (dR/dq) v by forward-mode (dual-number) differentiation."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        qd = fwAD.make_dual(q.detach(), v)
        R = op.rhs(qd)
        return fwAD.unpack_dual(R).tangent


def rk3_step_adjoint(op: Operator, dt, q0, lam3):
    """Reverse of one SSP-RK3 step: given dJ/dq_{n+1} return dJ/dq_n.

    Stages q1 = q0 + dt R(q0); q2 = 3/4 q0 + 1/4 (q1 + dt R(q1));
    q3 = 1/3 q0 + 2/3 (q2 + dt R(q2)); transposed stage by stage."""
    q1 = rk_stage(op, *SSP_RK3[0], dt, q0, q0)
    q2 = rk_stage(op, *SSP_RK3[1], dt, q0, q1)
    lam2 = (2.0 / 3.0) * (lam3 + dt * rhs_adjoint(op, q2, lam3))
    lam1 = 0.25 * (lam2 + dt * rhs_adjoint(op, q1, lam2))
    return (1.0 / 3.0) * lam3 + 0.75 * lam2 + lam1 + dt * rhs_adjoint(op, q0, lam1)


def target_functional(op: Operator, q, box):
    """J = sum_e J_e sum_{n: x_n in box} W_n theta'^2 (inclusive nodal mask)."""
    X, Y, Z = node_xyz(op.mesh)
    (x0, x1), (y0, y1), (z0, z1) = box
    mask = ((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1) & (Z >= z0) & (Z <= z1)).to(F64)
    rho_b, Th_b, _ = op.bg
    thp = (Th_b + q[4]) / (rho_b + q[0]) - Th_b / rho_b
    return (quad_weights(op) * mask * thp * thp).sum()


# ----------------------------------------------------------------------------- initial states

def cosine_bell(r):
    """1/2 (1 + cos(pi r)) for r <= 1, else 0."""
    return torch.where(r <= 1.0, 0.5 * (1.0 + torch.cos(math.pi * torch.clamp(r, max=1.0))),
                       torch.zeros_like(r))


def thermal_state(op: Operator, theta_p):
    """Perturbation state for a theta perturbation at unperturbed hydrostatic
    pressure: Theta' = 0, rho' = -rhobar theta'/(theta0 + theta'), U = 0."""
    rho_b = op.bg[0]
    th0 = op.phys.theta0
    rp = -rho_b * theta_p / (th0 + theta_p)
    z = torch.zeros_like(rp)
    return torch.stack([rp, z, z, z, z])


def bubble_state(op: Operator, dtheta=2.0, radius=250.0, centre=(500.0, 500.0, 350.0)):
    """Cosine-bell warm bubble (sections 4.2 and 4.3, here in 3-D)."""
    X, Y, Z = node_xyz(op.mesh)
    r = torch.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) / radius
    return thermal_state(op, dtheta * cosine_bell(r))


def density_current_state(op: Operator, dtheta=-15.0, xc=0.0, zc=3000.0, rx=4000.0, rz=2000.0):
    """Cold cosine bell, independent of y."""
    X, _, Z = node_xyz(op.mesh)
    r = torch.sqrt(((X - xc) / rx) ** 2 + ((Z - zc) / rz) ** 2)
    return thermal_state(op, dtheta * cosine_bell(r))


def isentropic_vortex(X, Y, t=0.0, beta=5.0, gamma=1.4, centre=(0.0, 0.0), speed=(1.0, 1.0)):
    """Isentropic vortex of section 4.1 with R = P0 = 1 and theta = 1 far away:
    (u, v) = (U_inf, V_inf) + beta/(2 pi) exp((1 - r^2)/2) (-(y - y_c), x - x_c),
    a temperature deficit T = 1 - (gamma - 1) beta^2/(8 gamma pi^2) exp(1 - r^2),
    rho = T^(1/(gamma - 1)), P = rho^gamma (isentropic, so theta = 1 everywhere and
    Theta = rho), translated rigidly at (U_inf, V_inf): the exact solution at time
    t (no periodic images; the perturbation is below 3e-7 at the edge of the
    paper's [-6, 6]^2 domain).  Returns the perturbation state about the constant
    background (rhobar, Thetabar) = (1, 1): (rho', rho u, rho v, 0, Theta').
    Reading: the paper prints the perturbation with a plus sign and calls it the
    potential temperature; with theta = 1 and P = rho^gamma it is read as the
    usual temperature deficit (a plus sign would give no vortex in balance)."""
    xr = X - centre[0] - speed[0] * t
    yr = Y - centre[1] - speed[1] * t
    r2 = xr * xr + yr * yr
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * torch.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    amp = beta / (2.0 * math.pi) * torch.exp(0.5 * (1.0 - r2))
    u = speed[0] - amp * yr
    v = speed[1] + amp * xr
    return torch.stack([rho - 1.0, rho * u, rho * v, torch.zeros_like(rho), rho - 1.0])
