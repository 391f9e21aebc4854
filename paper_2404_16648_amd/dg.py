"""Thin ctypes binding of the C ABI in include/dg.h (argument marshalling only).

Every numerical step runs in the HIP library ``libdgamr.so``; this module only
converts torch tensors to device pointers and streams, checks shapes and turns
status codes into exceptions.  It raises if the library is missing: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdgamr.so")

DG_OK = 0
DG_EINVAL = -1
DG_ENOMEM = -2
DG_EHIP = -3
DG_EUNSUPPORTED = -4
DG_ENONFINITE = -5

DG_PASS_COARSEN = 0
DG_PASS_REFINE = 1
DG_BG_NEUTRAL = 0
DG_BG_CONSTANT = 1
DG_BG_ISOTHERMAL = 2
DG_FP64 = 0
DG_MIXED = 1
DG_NC_MORTAR = 0
DG_NC_POINTWISE = 1
DG_IND_THETA = 0
DG_IND_GRAD_THETA = 1
DG_IND_PPRIME = 2
DG_KIND_COPY = -1
DG_KIND_FAMILY = 8

EXPORTED = [
    "dg_mesh_build", "dg_mesh_free", "dg_mesh_info_get", "dg_mesh_export", "dg_node_coords",
    "dg_init_bell", "dg_rhs", "dg_rk_stage", "dg_refine_project", "dg_coarsen_project",
    "dg_refine_project_adjoint", "dg_coarsen_project_adjoint", "dg_rhs_adjoint", "dg_rk_stage_adjoint", "dg_budgets", "dg_budgets_noalloc", "dg_indicator", "dg_indicator_async", "dg_pass_changes", "dg_flags_after_coarsen", "dg_tracer_rhs", "dg_tracer_stage", "dg_tracer_mass",
    "dg_project_fields", "dg_flags_buffer", "dg_fma_burst", "dg_sphere_mesh_build", "dg_sphere_faces",
    "dg_sphere_geometry", "dg_sphere_volumes", "dg_sphere_refine_project", "dg_sphere_coarsen_project",
    "dg_sphere_adapt_project", "dg_sphere_adapt_project_adjoint", "dg_sphere_face_kinds", "dg_last_error",
]


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dg status {code}: {msg}")
        self.code = code


class ForestDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("max_level", C.c_int32), ("periodic", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("host_only", C.c_int32)]


class SphereDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("n", C.c_int32), ("nz", C.c_int32), ("r_e", C.c_double), ("H", C.c_double),
                ("host_only", C.c_int32), ("max_level", C.c_int32)]


class Phys(C.Structure):
    _fields_ = [("cp", C.c_double), ("cv", C.c_double), ("P0", C.c_double), ("g", C.c_double),
                ("background", C.c_int32), ("precision", C.c_int32),
                ("theta0", C.c_double), ("rho0", C.c_double), ("Theta0", C.c_double),
                ("nonconforming", C.c_int32), ("mu", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [("K", C.c_int64), ("Np", C.c_int64), ("n_conf", C.c_int64), ("n_bnd", C.c_int64),
                ("n_hang", C.c_int64), ("n_refined", C.c_int64), ("n_coarsened", C.c_int64),
                ("N", C.c_int32), ("max_level_present", C.c_int32)]


class MeshTables(C.Structure):
    _fields_ = [("leaf", C.c_void_p), ("conf", C.c_void_p), ("bnd", C.c_void_p), ("hang", C.c_void_p),
                ("xfer_src", C.c_void_p), ("xfer_kind", C.c_void_p)]


class Bell(C.Structure):
    _fields_ = [("dtheta", C.c_double), ("centre", C.c_double * 3), ("radius", C.c_double * 3)]


_lib = None


def lib():
    """Load libdgamr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2404_16648_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.dg_mesh_build.argtypes = [C.POINTER(ForestDesc), P, P, C.c_int32, C.POINTER(P)]
        L.dg_mesh_free.argtypes = [P]
        L.dg_mesh_info_get.argtypes = [P, C.POINTER(MeshInfo)]
        L.dg_mesh_export.argtypes = [P, C.POINTER(MeshTables)]
        L.dg_node_coords.argtypes = [P, P, P]
        L.dg_init_bell.argtypes = [P, C.POINTER(Phys), C.POINTER(Bell), P, P]
        L.dg_rhs.argtypes = [P, C.POINTER(Phys), P, P, P]
        L.dg_rk_stage.argtypes = [P, C.POINTER(Phys), C.c_double, C.c_double, C.c_double, P, P, P, P]
        L.dg_refine_project.argtypes = [P, P, P, P, P]
        L.dg_coarsen_project.argtypes = [P, P, P, P, P]
        L.dg_refine_project_adjoint.argtypes = [P, P, P, P, P]
        L.dg_coarsen_project_adjoint.argtypes = [P, P, P, P, P]
        L.dg_rhs_adjoint.argtypes = [P, C.POINTER(Phys), P, P, P, P]
        L.dg_rk_stage_adjoint.argtypes = [P, C.POINTER(Phys), C.c_double, P, C.c_double, P, C.c_double,
                                          C.c_double, P, P, P, P]
        L.dg_budgets.argtypes = [P, C.POINTER(Phys), P, P, P]
        L.dg_budgets_noalloc.argtypes = [P, C.POINTER(Phys), P, P, P]
        L.dg_fma_burst.argtypes = [C.c_int32, C.c_int32, P, P, P]
        L.dg_flags_buffer.argtypes = [P, P, C.c_int32]
        L.dg_flags_after_coarsen.argtypes = [P, P, P]
        L.dg_tracer_rhs.argtypes = [P, C.POINTER(Phys), P, P, P, P]
        L.dg_tracer_stage.argtypes = [P, C.POINTER(Phys), C.c_double, C.c_double, C.c_double, P, P, P, P, P]
        L.dg_tracer_mass.argtypes = [P, P, P, P]
        L.dg_project_fields.argtypes = [P, P, C.c_int32, P, P, P]
        L.dg_indicator.argtypes = [P, C.POINTER(Phys), P, C.c_int32, C.c_double, P, P, P]
        L.dg_indicator_async.argtypes = [P, C.POINTER(Phys), P, C.c_int32, C.c_double, P, P, P]
        L.dg_pass_changes.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32)]
        L.dg_sphere_mesh_build.argtypes = [C.POINTER(SphereDesc), C.POINTER(P)]
        L.dg_sphere_faces.argtypes = [P, P]
        L.dg_sphere_geometry.argtypes = [P, P, P, P]
        L.dg_sphere_volumes.argtypes = [P, P, P]
        L.dg_sphere_refine_project.argtypes = [P, P, C.POINTER(Phys), P, P, P, P]
        L.dg_sphere_coarsen_project.argtypes = [P, P, C.POINTER(Phys), P, P, P]
        L.dg_sphere_adapt_project.argtypes = [P, P, C.POINTER(Phys), P, P, P, P]
        L.dg_sphere_adapt_project_adjoint.argtypes = [P, P, C.POINTER(Phys), P, P, C.c_double, P, P, P]
        L.dg_sphere_face_kinds.argtypes = [P, P]
        L.dg_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name != "dg_last_error":
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(code):
    if code != DG_OK:
        raise DGError(code, lib().dg_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("field tensors must live on the GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("field tensors must be contiguous float64")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass(frozen=True)
class PhysParams:
    """Gas constants, gravity, background and precision (dg_phys)."""
    cp: float = 1004.67
    cv: float = 717.5
    P0: float = 1.0e5
    g: float = 9.80616
    background: int = DG_BG_NEUTRAL
    precision: int = DG_FP64
    theta0: float = 300.0
    rho0: float = 1.0
    Theta0: float = 300.0
    nonconforming: int = DG_NC_MORTAR
    mu: float = 0.0          # artificial viscosity (m^2/s)

    def c(self):
        return Phys(self.cp, self.cv, self.P0, self.g, self.background, self.precision,
                    self.theta0, self.rho0, self.Theta0, self.nonconforming, self.mu)


class Mesh:
    """Owning handle of a dg_mesh."""

    def __init__(self, handle, prev=None):
        self._h = C.c_void_p(handle)
        self.prev = prev          # keeps the source mesh alive for the projections
        self.shell = bool(getattr(prev, "shell", False))   # a cubed-sphere shell (set by dg_sphere_mesh_build)
        info = MeshInfo()
        _check(lib().dg_mesh_info_get(self._h, C.byref(info)))
        self.info = info

    @property
    def handle(self):
        return self._h

    @property
    def K(self):
        return int(self.info.K)

    @property
    def N(self):
        return int(self.info.N)

    @property
    def Np(self):
        return int(self.info.Np)

    def free(self):
        if self._h is not None and self._h.value:
            lib().dg_mesh_free(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def tables(self):
        """Host copies of the integer tables (numpy int32)."""
        i = self.info
        out = {
            "leaf": np.zeros((i.K, 5), np.int32), "conf": np.zeros((i.n_conf, 3), np.int32),
            "bnd": np.zeros((i.n_bnd, 2), np.int32), "hang": np.zeros((i.n_hang, 6), np.int32),
            "xfer_src": np.zeros(i.K, np.int32), "xfer_kind": np.zeros(i.K, np.int32),
        }
        t = MeshTables(*[C.c_void_p(out[k].ctypes.data) if out[k].size else None
                         for k in ("leaf", "conf", "bnd", "hang", "xfer_src", "xfer_kind")])
        _check(lib().dg_mesh_export(self._h, C.byref(t)))
        return out

    def field(self, device="cuda"):
        import torch
        return torch.zeros(5, self.K, self.Np, dtype=torch.float64, device=device)


def dg_mesh_build(N=None, nroot=None, max_level=0, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                  periodic=(0, 0, 0), prev: Mesh | None = None, flags=None, pass_=DG_PASS_REFINE,
                  host_only=False) -> Mesh:
    out = C.c_void_p()
    if prev is None:
        d = ForestDesc(N, nroot[0], nroot[1], nroot[2], max_level, (C.c_int32 * 3)(*periodic),
                       (C.c_double * 3)(*lo), (C.c_double * 3)(*hi), 1 if host_only else 0)
        _check(lib().dg_mesh_build(C.byref(d), None, None, 0, C.byref(out)))
    else:
        fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        if fl.shape != (prev.K,):
            raise ValueError("flags must have one entry per leaf of prev")
        _check(lib().dg_mesh_build(None, prev.handle, C.c_void_p(fl.ctypes.data), pass_, C.byref(out)))
    return Mesh(out.value, prev)


def dg_sphere_mesh_build(N, n, nz, r_e=6.371e6, H=1.0e4, host_only=False, max_level=0) -> Mesh:
    """Cubed-sphere shell mesh (six panels of n x n elements, nz layers), the root
    level of a forest refinable max_level times."""
    out = C.c_void_p()
    d = SphereDesc(N, n, nz, r_e, H, 1 if host_only else 0, max_level)
    _check(lib().dg_sphere_mesh_build(C.byref(d), C.byref(out)))
    m = Mesh(out.value)
    m.shell = True
    return m


def dg_sphere_faces(mesh: Mesh):
    """Face connectivity of a shell mesh: int32 [K, 6, 3] (neighbour, its face, flip)."""
    nb = np.zeros((mesh.K, 6, 3), np.int32)
    _check(lib().dg_sphere_faces(mesh.handle, C.c_void_p(nb.ctypes.data)))
    return nb


def dg_sphere_geometry(mesh: Mesh):
    """Host geometry of a shell mesh: metric [10, K, Np], fgeo [K, 6, (N+1)^2, 4], c1d [3, K, N+1]."""
    n1 = mesh.N + 1
    metric = np.zeros((10, mesh.K, mesh.Np))
    fgeo = np.zeros((mesh.K, 6, n1 * n1, 4))
    c1d = np.zeros((3, mesh.K, n1))
    _check(lib().dg_sphere_geometry(mesh.handle, C.c_void_p(metric.ctypes.data), C.c_void_p(fgeo.ctypes.data),
                                    C.c_void_p(c1d.ctypes.data)))
    return metric, fgeo, c1d


def dg_sphere_volumes(mesh: Mesh):
    """Spherical-excess volume of every element (float64 [K]) and the totals
    (isoparametric volume sum J W, sum of the spherical-excess volumes)."""
    vol = np.zeros(mesh.K)
    tot = np.zeros(2)
    _check(lib().dg_sphere_volumes(mesh.handle, C.c_void_p(vol.ctypes.data), C.c_void_p(tot.ctypes.data)))
    return vol, (float(tot[0]), float(tot[1]))


def dg_sphere_refine_project(coarse: Mesh, fine: Mesh, phys: PhysParams, q_coarse, q_fine, stream=None,
                             scale=True):
    """Refinement transfer between a shell and its refinement; returns the mass
    scale factor (waiting for the stream), or None with scale=False (enqueue only)."""
    _shape_check(coarse, q_coarse)
    _shape_check(fine, q_fine)
    ph = phys.c()
    s = np.zeros(1)
    _check(lib().dg_sphere_refine_project(coarse.handle, fine.handle, C.byref(ph), _ptr(q_coarse), _ptr(q_fine),
                                          C.c_void_p(s.ctypes.data) if scale else None, _stream(stream)))
    return float(s[0]) if scale else None


def dg_sphere_adapt_project(src: Mesh, dst: Mesh, phys: PhysParams, q_from, q_to, stream=None, scale=True):
    """Transfer of a shell's refine or coarsen pass (dst built from src); returns
    the refinement's mass scale factor (waiting for the stream), or None with
    scale=False (enqueue only)."""
    _shape_check(src, q_from)
    _shape_check(dst, q_to)
    ph = phys.c()
    s = np.zeros(1)
    _check(lib().dg_sphere_adapt_project(src.handle, dst.handle, C.byref(ph), _ptr(q_from), _ptr(q_to),
                                         C.c_void_p(s.ctypes.data) if scale else None, _stream(stream)))
    return float(s[0]) if scale else None


def dg_sphere_adapt_project_adjoint(src: Mesh, dst: Mesh, phys: PhysParams, q_from, q_to, scale, qbar_to, qbar_from,
                                    stream=None):
    """The transpose of the derivative of dg_sphere_adapt_project at q_from (q_to its
    output, scale its factor): qbar_from from qbar_to."""
    _shape_check(dst, qbar_to)
    _shape_check(src, qbar_from)
    if q_from is not None:
        _shape_check(src, q_from)
    if q_to is not None:
        _shape_check(dst, q_to)
    ph = phys.c()
    _check(lib().dg_sphere_adapt_project_adjoint(src.handle, dst.handle, C.byref(ph),
                                                 _ptr(q_from) if q_from is not None else None,
                                                 _ptr(q_to) if q_to is not None else None, float(scale),
                                                 _ptr(qbar_to), _ptr(qbar_from), _stream(stream)))


def dg_sphere_face_kinds(mesh: Mesh):
    """Face kinds of a shell, int32 [K, 6]: 0 wall, 1 conforming, 2 + 4 quadrant fine side, 3 coarse side."""
    k = np.zeros((mesh.K, 6), np.int32)
    _check(lib().dg_sphere_face_kinds(mesh.handle, C.c_void_p(k.ctypes.data)))
    return k


def dg_sphere_coarsen_project(fine: Mesh, coarse: Mesh, phys: PhysParams, q_fine, q_coarse, stream=None):
    """Coarsening transfer from a shell's refinement back to the shell."""
    _shape_check(fine, q_fine)
    _shape_check(coarse, q_coarse)
    ph = phys.c()
    _check(lib().dg_sphere_coarsen_project(fine.handle, coarse.handle, C.byref(ph), _ptr(q_fine), _ptr(q_coarse),
                                           _stream(stream)))


def dg_pass_changes(mesh: Mesh, flags, pass_) -> bool:
    """Whether dg_mesh_build(prev=mesh, flags=flags, pass_=pass_) would change a leaf."""
    fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
    if fl.shape != (mesh.K,):
        raise ValueError("flags must have one entry per leaf")
    ch = C.c_int32(0)
    _check(lib().dg_pass_changes(mesh.handle, C.c_void_p(fl.ctypes.data), pass_, C.byref(ch)))
    return bool(ch.value)


def _shape_check(mesh, *ts):
    for t in ts:
        if t is not None and tuple(t.shape) != (5, mesh.K, mesh.Np):
            raise ValueError(f"field shape {tuple(t.shape)} != (5, {mesh.K}, {mesh.Np})")


def dg_node_coords(mesh: Mesh, xyz, stream=None):
    if tuple(xyz.shape) != (3, mesh.K, mesh.Np):
        raise ValueError("xyz must be [3, K, Np]")
    _check(lib().dg_node_coords(mesh.handle, _ptr(xyz), _stream(stream)))


def dg_init_bell(mesh: Mesh, phys: PhysParams, q, dtheta, centre, radius, stream=None):
    _shape_check(mesh, q)
    b = Bell(dtheta, (C.c_double * 3)(*centre), (C.c_double * 3)(*radius))
    p = phys.c()
    _check(lib().dg_init_bell(mesh.handle, C.byref(p), C.byref(b), _ptr(q), _stream(stream)))


def dg_rhs(mesh: Mesh, phys: PhysParams, q, rhs, stream=None):
    _shape_check(mesh, q, rhs)
    p = phys.c()
    _check(lib().dg_rhs(mesh.handle, C.byref(p), _ptr(q), _ptr(rhs), _stream(stream)))


def dg_rk_stage(mesh: Mesh, phys: PhysParams, a, b, dt, q0, qs, qout, stream=None):
    _shape_check(mesh, q0, qs, qout)
    p = phys.c()
    _check(lib().dg_rk_stage(mesh.handle, C.byref(p), a, b, dt, _ptr(q0), _ptr(qs), _ptr(qout),
                             _stream(stream)))


def dg_refine_project(src: Mesh, dst: Mesh, q_from, q_to, stream=None):
    _shape_check(src, q_from)
    _shape_check(dst, q_to)
    _check(lib().dg_refine_project(src.handle, dst.handle, _ptr(q_from), _ptr(q_to), _stream(stream)))


def dg_coarsen_project(src: Mesh, dst: Mesh, q_from, q_to, stream=None):
    _shape_check(src, q_from)
    _shape_check(dst, q_to)
    _check(lib().dg_coarsen_project(src.handle, dst.handle, _ptr(q_from), _ptr(q_to), _stream(stream)))


def dg_refine_project_adjoint(src: Mesh, dst: Mesh, qbar_to, qbar_from, stream=None):
    """qbar_from := P^T qbar_to, P the refine transfer src -> dst."""
    _shape_check(dst, qbar_to)
    _shape_check(src, qbar_from)
    _check(lib().dg_refine_project_adjoint(src.handle, dst.handle, _ptr(qbar_to), _ptr(qbar_from),
                                           _stream(stream)))


def dg_coarsen_project_adjoint(src: Mesh, dst: Mesh, qbar_to, qbar_from, stream=None):
    """qbar_from := P^T qbar_to, P the coarsen transfer src -> dst."""
    _shape_check(dst, qbar_to)
    _shape_check(src, qbar_from)
    _check(lib().dg_coarsen_project_adjoint(src.handle, dst.handle, _ptr(qbar_to), _ptr(qbar_from),
                                            _stream(stream)))


def _tracer_check(mesh, *ts):
    for t in ts:
        if t is not None and tuple(t.shape) != (mesh.K, mesh.Np):
            raise ValueError(f"tracer shape {tuple(t.shape)} != ({mesh.K}, {mesh.Np})")


def dg_tracer_rhs(mesh: Mesh, phys: PhysParams, q, c, rhs, stream=None):
    """rhs := R_C(q, c), the tracer right-hand side (c, rhs: [K, Np])."""
    _shape_check(mesh, q)
    _tracer_check(mesh, c, rhs)
    p = phys.c()
    _check(lib().dg_tracer_rhs(mesh.handle, C.byref(p), _ptr(q), _ptr(c), _ptr(rhs), _stream(stream)))


def dg_tracer_stage(mesh: Mesh, phys: PhysParams, a, b, dt, qs, c0, cs, cout, stream=None):
    """cout := a c0 + b (cs + dt R_C(qs, cs))."""
    _shape_check(mesh, qs)
    _tracer_check(mesh, c0, cs, cout)
    p = phys.c()
    _check(lib().dg_tracer_stage(mesh.handle, C.byref(p), a, b, dt, _ptr(qs), _ptr(c0), _ptr(cs), _ptr(cout),
                                 _stream(stream)))


def dg_tracer_mass(mesh: Mesh, c, stream=None):
    _tracer_check(mesh, c)
    out = (C.c_double * 1)()
    _check(lib().dg_tracer_mass(mesh.handle, _ptr(c), out, _stream(stream)))
    return out[0]


def dg_project_fields(src: Mesh, dst: Mesh, q_from, q_to, stream=None):
    """Conservative transfer of nvar fields [nvar, K, Np] (or one field [K, Np])."""
    nv = 1 if q_from.dim() == 2 else int(q_from.shape[0])
    for t, m in ((q_from, src), (q_to, dst)):
        shape = (m.K, m.Np) if nv == 1 and t.dim() == 2 else (nv, m.K, m.Np)
        if tuple(t.shape) != shape:
            raise ValueError(f"field shape {tuple(t.shape)} != {shape}")
    _check(lib().dg_project_fields(src.handle, dst.handle, nv, _ptr(q_from), _ptr(q_to), _stream(stream)))


def ssp_rk3_step_tracer(mesh: Mesh, phys: PhysParams, dt, q, q1, q2, c, c1, c2, stream=None, side=None):
    """One SSP-RK3 step of the Euler state and a passive tracer, in place on q and
    c (stage buffers q1, q2, c1, c2).

    Tracer stage k needs the Euler stage input of stage k (for the velocity and
    the wave speed).  On one stream each tracer stage runs before the Euler stage
    that could overwrite its input.  With `side` (another stream) the tracer
    stages run there, beside the Euler stages on `stream` (the two use separate
    mortar workspaces of the mesh and only read its tables): after the first Euler
    stage (which also makes the mesh's device tables and background if this is
    the first call on it), side runs the first two tracer stages while the second
    Euler stage runs, and the third beside the third, which waits for the first
    tracer stage (it overwrites q, which that stage reads).  `stream` waits for
    side at the end, so later work on it is ordered after the whole step.  The
    results are bitwise those of the one-stream order."""
    if side is None:
        dg_tracer_stage(mesh, phys, *SSP_RK3[0], dt, q, c, c, c1, stream)
        dg_rk_stage(mesh, phys, *SSP_RK3[0], dt, q, q, q1, stream)
        dg_tracer_stage(mesh, phys, *SSP_RK3[1], dt, q1, c, c1, c2, stream)
        dg_rk_stage(mesh, phys, *SSP_RK3[1], dt, q, q1, q2, stream)
        dg_tracer_stage(mesh, phys, *SSP_RK3[2], dt, q2, c, c2, c, stream)
        dg_rk_stage(mesh, phys, *SSP_RK3[2], dt, q, q2, q, stream)
        return
    import torch
    main = stream if stream is not None else torch.cuda.current_stream()
    dg_rk_stage(mesh, phys, *SSP_RK3[0], dt, q, q, q1, main)
    side.wait_stream(main)                       # q, c ready and q1 written
    dg_tracer_stage(mesh, phys, *SSP_RK3[0], dt, q, c, c, c1, side)
    t1 = torch.cuda.Event()
    t1.record(side)
    dg_tracer_stage(mesh, phys, *SSP_RK3[1], dt, q1, c, c1, c2, side)
    dg_rk_stage(mesh, phys, *SSP_RK3[1], dt, q, q1, q2, main)
    e2 = torch.cuda.Event()
    e2.record(main)
    side.wait_event(e2)                          # q2 written
    dg_tracer_stage(mesh, phys, *SSP_RK3[2], dt, q2, c, c2, c, side)
    main.wait_event(t1)                          # the first tracer stage has read q
    dg_rk_stage(mesh, phys, *SSP_RK3[2], dt, q, q2, q, main)
    main.wait_stream(side)


def dg_rhs_adjoint(mesh: Mesh, phys: PhysParams, q, lam, qbar, stream=None):
    _shape_check(mesh, q, lam, qbar)
    p = phys.c()
    _check(lib().dg_rhs_adjoint(mesh.handle, C.byref(p), _ptr(q), _ptr(lam), _ptr(qbar), _stream(stream)))


def dg_rk_stage_adjoint(mesh: Mesh, phys: PhysParams, a1, w1, a2, w2, b, dt, q, y, out, stream=None):
    _shape_check(mesh, w1, w2, q, y, out)
    p = phys.c()
    _check(lib().dg_rk_stage_adjoint(mesh.handle, C.byref(p), a1, _ptr(w1), a2, _ptr(w2), b, dt, _ptr(q),
                                     _ptr(y), _ptr(out), _stream(stream)))


def dg_flags_after_coarsen(coarsened: Mesh, flags):
    """Refine-pass flags on `coarsened` from the cycle's flags on the mesh its
    coarsen pass started from (a new array)."""
    fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
    out = np.zeros(coarsened.K, dtype=np.int8)
    _check(lib().dg_flags_after_coarsen(coarsened.handle, C.c_void_p(fl.ctypes.data),
                                        C.c_void_p(out.ctypes.data) if coarsened.K else None))
    return out


def dg_flags_buffer(mesh: Mesh, flags, B):
    """Buffer zone: B rounds of face-neighbour dilation of the +1 flags (returns a new array)."""
    fl = np.ascontiguousarray(np.asarray(flags, dtype=np.int8)).copy()
    if fl.shape != (mesh.K,):
        raise ValueError("flags must have one entry per leaf")
    _check(lib().dg_flags_buffer(mesh.handle, C.c_void_p(fl.ctypes.data), int(B)))
    return fl


def dg_fma_burst(blocks, iters, sink, stream=None):
    """Calibration launch (float64 FMA rate); returns the flops it performs."""
    if tuple(sink.shape) != (256 * blocks,):
        raise ValueError("sink must be [256*blocks]")
    out = C.c_double()
    _check(lib().dg_fma_burst(blocks, iters, _ptr(sink), C.byref(out), _stream(stream)))
    return out.value


def dg_budgets(mesh: Mesh, phys: PhysParams, q, stream=None):
    _shape_check(mesh, q)
    out = (C.c_double * 4)()
    p = phys.c()
    _check(lib().dg_budgets(mesh.handle, C.byref(p), _ptr(q), out, _stream(stream)))
    return tuple(out)


def dg_budgets_noalloc(mesh: Mesh, phys: PhysParams, q, out_dev, stream=None):
    """Budgets into the device float64 tensor out_dev[4], enqueued only (no
    allocation, copy or synchronisation)."""
    import torch
    _shape_check(mesh, q)
    if (not isinstance(out_dev, torch.Tensor) or not out_dev.is_cuda or out_dev.dtype != torch.float64
            or out_dev.numel() < 4 or not out_dev.is_contiguous()):
        raise ValueError("out_dev must be a contiguous float64 GPU tensor of at least 4 entries")
    p = phys.c()
    _check(lib().dg_budgets_noalloc(mesh.handle, C.byref(p), _ptr(q), C.c_void_p(out_dev.data_ptr()),
                                    _stream(stream)))


def dg_indicator(mesh: Mesh, phys: PhysParams, q, kind, thr, eta=None, stream=None):
    _shape_check(mesh, q)
    fl = np.zeros(mesh.K, dtype=np.int8)
    p = phys.c()
    _check(lib().dg_indicator(mesh.handle, C.byref(p), _ptr(q), kind, thr, _ptr(eta),
                              C.c_void_p(fl.ctypes.data) if mesh.K else None, _stream(stream)))
    return fl


def dg_indicator_async(mesh: Mesh, phys: PhysParams, q, kind, thr, flags_dev, eta=None, stream=None):
    """Enqueue the indicator; flags_dev is a device int8 tensor of K entries."""
    import torch
    _shape_check(mesh, q)
    if (not isinstance(flags_dev, torch.Tensor) or not flags_dev.is_cuda or flags_dev.dtype != torch.int8
            or flags_dev.numel() < mesh.K or not flags_dev.is_contiguous()):
        raise ValueError("flags_dev must be a contiguous int8 GPU tensor of at least K entries")
    p = phys.c()
    _check(lib().dg_indicator_async(mesh.handle, C.byref(p), _ptr(q), kind, thr, _ptr(eta),
                                    C.c_void_p(flags_dev.data_ptr()), _stream(stream)))


SSP_RK3 = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def ssp_rk3_step(mesh: Mesh, phys: PhysParams, dt, q, q1, q2, stream=None):
    """One SSP-RK3 step in place on q, using q1, q2 as stage buffers (3 dg_rk_stage calls)."""
    dg_rk_stage(mesh, phys, *SSP_RK3[0], dt, q, q, q1, stream)
    dg_rk_stage(mesh, phys, *SSP_RK3[1], dt, q, q1, q2, stream)
    dg_rk_stage(mesh, phys, *SSP_RK3[2], dt, q, q2, q, stream)


def adapt_meshes(mesh: Mesh, phys: PhysParams, q, kind, thr, stream=None, buffer=0):
    """The two passes of one adaptation cycle from the state q: indicator -> flags
    (-> buffer zone of `buffer` leaves) -> coarsen pass -> refine pass (parents
    made by the coarsen pass are not refined in the same cycle).  Returns
    (mesh_c, mesh_r); a pass that changes no leaf returns its input mesh itself."""
    return adapt_meshes_from_flags(mesh, dg_indicator(mesh, phys, q, kind, thr, stream=stream), buffer)


def adapt_meshes_from_flags(mesh: Mesh, flags, buffer=0):
    """The two forest passes of one adaptation cycle from the indicator's flags
    (host work only); see :func:`adapt_meshes`."""
    if buffer:
        flags = dg_flags_buffer(mesh, flags, buffer)
    # a pass that would change no leaf is not built (its result would equal its input)
    mc = mesh
    if dg_pass_changes(mesh, flags, DG_PASS_COARSEN):
        mc = dg_mesh_build(prev=mesh, flags=flags, pass_=DG_PASS_COARSEN)
        fl2 = dg_flags_after_coarsen(mc, flags)
    else:
        fl2 = np.where(np.asarray(flags) > 0, 1, 0).astype(np.int8)  # the same leaves
    mr = mc
    if dg_pass_changes(mc, fl2, DG_PASS_REFINE):
        mr = dg_mesh_build(prev=mc, flags=fl2, pass_=DG_PASS_REFINE)
    return mc, mr


def adapt_cycle(mesh: Mesh, phys: PhysParams, q, kind, thr, stream=None, buffer=0):
    """One adaptation cycle: the passes of :func:`adapt_meshes`, each followed by
    its conservative projection (host control flow; every arithmetic step runs in
    the library).  Returns (new_mesh, new_q); when neither pass changes a leaf,
    the input mesh and field themselves."""
    return project_cycle(mesh, *adapt_meshes(mesh, phys, q, kind, thr, stream, buffer), q, stream, phys)


def _on(stream):
    """Context in which torch allocates for `stream` (its caching allocator hands a
    block freed there only to later work on the same stream); None: as is."""
    import contextlib
    import torch
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def project_cycle(mesh: Mesh, mc: Mesh, mr: Mesh, q, stream=None, phys: PhysParams | None = None, out_c=None,
                  out_r=None):
    """The projections of one adaptation cycle (mesh -> mc coarsening, mc -> mr
    refinement; a pass that changed nothing is skipped).  Returns (mr, q on mr);
    the new fields are out_c / out_r when given ([5, K, Np] of their meshes, not
    aliasing q), else allocated for `stream`.  A shell takes the transfer of
    section 3.4 (its refinement's scale factor needs phys for the background)."""
    import torch
    if mesh.shell and phys is None:
        raise ValueError("a shell's projections need phys")
    qc = q
    with _on(stream):
        if mc is not mesh:
            qc = out_c if out_c is not None else torch.empty(5, mc.K, mc.Np, dtype=torch.float64, device=q.device)
            if mesh.shell:
                dg_sphere_adapt_project(mesh, mc, phys, q, qc, stream, scale=False)
            else:
                dg_coarsen_project(mesh, mc, q, qc, stream)
        qr = qc
        if mr is not mc:
            qr = out_r if out_r is not None else torch.empty(5, mr.K, mr.Np, dtype=torch.float64, device=q.device)
            if mesh.shell:
                dg_sphere_adapt_project(mc, mr, phys, qc, qr, stream, scale=False)
            else:
                dg_refine_project(mc, mr, qc, qr, stream)
    return mr, qr


class GraphedSteps:
    """`nsteps` SSP-RK3 steps on one mesh captured once as a HIP graph and then
    replayed, for meshes small enough that launch overhead dominates.  The state
    lives in `self.q` (advanced in place by every replay()); the stage buffers are
    owned by the object.  The mesh's device tables, its background and the kernels
    are made ready by a warm-up step on scratch buffers before the capture, so the
    captured calls only launch kernels (no allocation, no memset, no copy)."""

    def __init__(self, mesh: Mesh, phys: PhysParams, dt, q, nsteps):
        import torch
        self.mesh, self.phys, self.dt, self.nsteps = mesh, phys, dt, nsteps
        self.q = q
        self.q1, self.q2 = torch.empty_like(q), torch.empty_like(q)
        w = q.clone()
        ssp_rk3_step(mesh, phys, dt, w, self.q1, self.q2)
        torch.cuda.synchronize()
        del w
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(nsteps):
                ssp_rk3_step(mesh, phys, dt, self.q, self.q1, self.q2)

    def replay(self):
        self.graph.replay()


class AdaptiveStepper:
    """SSP-RK3 steps with an adaptation cycle before every `every`-th step
    (section 3.2: regrid every T steps; indicator and projections on the GPU,
    forest passes on the host), the host part of each cycle overlapped with GPU
    work.  At a cycle the indicator is enqueued, its flags copied to pinned host
    memory behind an event, and the next step is computed at once on the current
    mesh, out of place, while the host waits for the flags and runs the passes.
    If the cycle changes no leaf that step is the result (the same kernels on the
    same inputs as adapting first: bitwise the same state); otherwise it is
    dropped and the step is made again after the projections.  Host control flow
    only: every arithmetic step runs in the library.

    step(events=None) advances one step; with a list, an event pair around the
    three stage launches of the step that is kept is appended to it.  The state is
    `self.q`; the tensor passed in becomes one of the stepper's buffers."""

    def __init__(self, mesh: Mesh, phys: PhysParams, q, dt, every, kind, thr, buffer=0, stream=None):
        import torch
        self.mesh, self.phys, self.q, self.dt = mesh, phys, q, dt
        self.every, self.kind, self.thr, self.buffer = every, kind, thr, buffer
        self.stream = stream
        if stream is not None:
            # the caller's state was made on another stream: the stepper's stream
            # waits for it, and the tensor is marked as used there
            stream.wait_stream(torch.cuda.current_stream())
            q.record_stream(stream)
        self.n = 0           # steps made
        self.cycles = 0      # adaptation cycles run
        self.changed = 0     # cycles that changed the mesh (speculative step dropped)
        # flag buffers (device and pinned host), allocated ahead of the first cycle and
        # grown with the mesh: an allocation inside a cycle would stall it
        self._dev = torch.empty(0, dtype=torch.int8, device=q.device)
        self._host = torch.empty(0, dtype=torch.int8).pin_memory()
        self._reserve(mesh.K)
        # four flat buffers: the state, the speculative step's output and the two
        # stage buffers (the state and the speculation swap when the speculation is
        # kept); a cycle that changes the mesh projects into the speculation's buffer
        # (through a stage buffer when both passes change) and takes the new mesh's
        # fields as views of them, so it allocates nothing unless the mesh outgrows
        # them (then all four are made again with a quarter to spare)
        self._flat = [q.view(-1)] + self._new_flats(3, q.numel() + q.numel() // 4)
        self._roles = [0, 1, 2, 3]   # state, speculation, stage 1, stage 2
        self._views(mesh.K)

    def _new_flats(self, n, cap):
        import torch
        with _on(self.stream):  # allocated for the stream that uses them
            return [torch.empty(cap, dtype=torch.float64, device=self.q.device) for _ in range(n)]

    def _view(self, i, K):
        return self._flat[i][:5 * K * self.mesh.Np].view(5, K, self.mesh.Np)

    def _views(self, K):
        st, sp, a, b = self._roles
        self._spec, self._q1, self._q2 = self._view(sp, K), self._view(a, K), self._view(b, K)

    def _reserve(self, K):
        import torch
        if self._dev.numel() < K:
            with _on(self.stream):
                self._dev = torch.empty(2 * K, dtype=torch.int8, device=self.q.device)
        if self._host.numel() < K:
            self._host = torch.empty(2 * K, dtype=torch.int8).pin_memory()

    def _stages(self, mesh, q, out, events):
        import torch
        q1, q2 = self._q1, self._q2
        if events is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream() if self.stream is None else self.stream)
        dg_rk_stage(mesh, self.phys, *SSP_RK3[0], self.dt, q, q, q1, self.stream)
        dg_rk_stage(mesh, self.phys, *SSP_RK3[1], self.dt, q, q1, q2, self.stream)
        dg_rk_stage(mesh, self.phys, *SSP_RK3[2], self.dt, q, q2, out, self.stream)
        if events is not None:
            e1.record(torch.cuda.current_stream() if self.stream is None else self.stream)
            return e0, e1
        return None

    def step(self, events=None):
        import torch
        due = self.n > 0 and self.every > 0 and self.n % self.every == 0
        mesh, q = self.mesh, self.q
        if not due:
            ev = self._stages(mesh, q, q, events)
        else:
            self.cycles += 1
            K = mesh.K
            self._reserve(max(K, 1))
            dg_indicator_async(mesh, self.phys, q, self.kind, self.thr, self._dev, stream=self.stream)
            host = self._host[:K]
            strm = torch.cuda.current_stream() if self.stream is None else self.stream
            with torch.cuda.stream(strm):  # the copy and its event on the indicator's stream
                host.copy_(self._dev[:K], non_blocking=True)
            ready = torch.cuda.Event()
            ready.record(strm)
            spec = self._spec
            ev = self._stages(mesh, q, spec, events)  # speculative: q itself is kept
            ready.synchronize()
            flags = host.numpy().copy()
            mc, mr = adapt_meshes_from_flags(mesh, flags, self.buffer)
            if mr is mesh:
                self.q, self._spec = spec, q  # the old state's buffer takes the next speculation
                r = self._roles
                self._roles = [r[1], r[0], r[2], r[3]]
            else:
                self.changed += 1
                need = 5 * max(mc.K, mr.K) * mesh.Np
                if min(f.numel() for f in self._flat) < need:
                    # q stays alive (and its buffer in use on the stream) until the
                    # projection below has read it
                    self._flat = self._new_flats(4, need + need // 4)
                    self._roles = [3, 0, 1, 2]
                st, sp, a, b = self._roles
                both = mc is not mesh and mr is not mc
                out_c = self._flat[a][:5 * mc.K * mesh.Np].view(5, mc.K, mesh.Np) if both else None
                out_r = self._flat[sp][:5 * mr.K * mesh.Np].view(5, mr.K, mesh.Np)
                if mr is mc:  # only the coarsen pass changed: its output is the new state
                    out_c, out_r = out_r, None
                mr2, qn = project_cycle(mesh, mc, mr, q, self.stream, self.phys, out_c, out_r)
                mr2.prev = None
                self.mesh, self.q = mr2, qn
                self._roles = [sp, st, a, b]
                self._reserve(mr2.K)
                self._views(mr2.K)
                ev = self._stages(mr2, qn, qn, events)
        if ev is not None:
            events.append(ev)
        self.n += 1


def initial_mesh(N, nroot, max_level, lo, hi, periodic, phys: PhysParams, bell, kind, thr):
    """Uniform level-0 forest, then repeat (cosine-bell IC on the nodes ->
    indicator -> refine pass) until no leaf is flagged (at most max_level
    passes).  Returns (mesh, q) with q the IC on the final mesh."""
    import torch
    m = dg_mesh_build(N, nroot, max_level, lo, hi, periodic)
    for _ in range(max_level + 1):
        q = torch.empty(5, m.K, m.Np, dtype=torch.float64, device="cuda")
        dg_init_bell(m, phys, q, *bell)
        fl = dg_indicator(m, phys, q, kind, thr)
        fl[fl < 0] = 0
        if not (fl > 0).any():
            return m, q
        m = dg_mesh_build(prev=m, flags=fl, pass_=DG_PASS_REFINE)
        m.prev = None
    q = torch.empty(5, m.K, m.Np, dtype=torch.float64, device="cuda")
    dg_init_bell(m, phys, q, *bell)
    return m, q
