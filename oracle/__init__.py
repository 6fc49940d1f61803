"""FP64 CPU oracle for the entropic (KBC) lattice Boltzmann step with moving walls.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1608_04658_amd``) never imports, links or calls it, and it
shares no code with the GPU path: its C source (``elbm_oracle.c``) carries its
own lattice tables and follows the paper's equations with one scalar loop per
node in FP64.

A second library, ``elbm_oracle_adjoint.cpp`` (C++, FP64), is the adjoint of one step: it
restates the step on a generic scalar type and takes exact local Jacobians with forward-mode dual
numbers (``Simulation.adjoint_step``).  It does not call the forward oracle, so the tests check the
two against each other.

This module is a ctypes wrapper (argument marshalling plus the time loop).
Population arrays are float64 numpy arrays of shape (27, nz, ny, nx); the
velocity order is i = 9 (cz+1) + 3 (cy+1) + (cx+1).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "elbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libelbm_oracle.so")
_ADJ_SRC = os.path.join(_HERE, "elbm_oracle_adjoint.cpp")
_ADJ_LIB_PATH = os.path.join(_HERE, "libelbm_oracle_adjoint.so")
_lib = None
_adj_lib = None

NQ = 27


def build(force: bool = True) -> str:
    """Compile the oracle (gcc) and its adjoint (g++): FP64, OpenMP, no FP contraction."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = f"{_LIB_PATH}.{os.getpid()}.tmp"  # per process: concurrent builds do not collide
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    if force or not os.path.exists(_ADJ_LIB_PATH):
        tmp = f"{_ADJ_LIB_PATH}.{os.getpid()}.tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall",
               "-o", tmp, _ADJ_SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _ADJ_LIB_PATH)
    return _LIB_PATH


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("channel", ctypes.c_int32), ("beta", ctypes.c_double), ("rho0", ctypes.c_double),
                ("u_in", ctypes.c_double * 3), ("stream_only", ctypes.c_int32), ("stabiliser", ctypes.c_int32),
                ("central", ctypes.c_int32)]


class Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tracked", ctypes.c_int32), ("p0", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("normal", ctypes.c_double * 3), ("amp", ctypes.c_double),
                ("period", ctypes.c_double), ("dir", ctypes.c_double * 3), ("vel", ctypes.c_double * 3),
                ("omega", ctypes.c_double * 3), ("track_t", ctypes.c_double),
                ("track_c", (ctypes.c_double * 3) * 2), ("track_U", (ctypes.c_double * 3) * 2),
                ("mesh_X", ctypes.POINTER(ctypes.c_double) * 2), ("mesh_V", ctypes.POINTER(ctypes.c_double) * 2),
                ("mesh_tri", ctypes.POINTER(ctypes.c_int32)), ("mesh_nv", ctypes.c_int32), ("mesh_nt", ctypes.c_int32),
                ("mesh_t", ctypes.c_double), ("track_W", (ctypes.c_double * 3) * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("boundary_nodes", ctypes.c_int64), ("links", ctypes.c_int64),
                ("refill_nodes", ctypes.c_int64), ("gamma_guard", ctypes.c_int64),
                ("gamma_min", ctypes.c_double), ("gamma_max", ctypes.c_double), ("exact_fallback", ctypes.c_int64)]


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_feq.argtypes = [ctypes.c_double, _D, _D]
        L.or_collide_ex.argtypes = [_D, ctypes.c_double, _D, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.or_collide_ex.restype = ctypes.c_double
        L.or_collide_central.argtypes = [_D, ctypes.c_double, _D, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.or_collide_central.restype = ctypes.c_double
        L.or_shear_part_central.argtypes = [_D, _D, _D]
        L.or_gamma_exact.argtypes = [_D, ctypes.c_double]
        L.or_gamma_exact.restype = ctypes.c_double
        L.or_H.argtypes = [_D]
        L.or_H.restype = ctypes.c_double
        L.or_shear_part.argtypes = [_D, _D]
        L.or_grad_dist.argtypes = [ctypes.c_double, _D, _D, _D]
        L.or_pressure.argtypes = [ctypes.c_double, _D, _D, ctypes.c_double, _D]
        L.or_beta_from_nu.argtypes = [ctypes.c_double]
        L.or_beta_from_nu.restype = ctypes.c_double
        L.or_kinematics.argtypes = [ctypes.POINTER(Body), ctypes.c_double, _D, _D]
        L.or_q.argtypes = [ctypes.POINTER(Body), _D, _D, ctypes.c_int]
        L.or_q.restype = ctypes.c_double
        L.or_solid_mask.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Body), ctypes.c_int, ctypes.c_double, _U8]
        L.or_grad_u.argtypes = [ctypes.POINTER(Grid), _D, _U8, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.or_macro.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Body), ctypes.c_int, ctypes.c_double, _D, _U8,
                               _D, _D, _D]
        L.or_step.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Body), ctypes.c_int, ctypes.c_double, _D, _U8,
                              _U8, _D, _D, _D, ctypes.POINTER(Stats)]
        L.or_step.restype = ctypes.c_int
        L.or_refill_state.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Body), ctypes.c_int, ctypes.c_double, _D,
                                      _U8, _U8, _D, _D, _D, ctypes.POINTER(ctypes.c_int64)]
        L.or_init_equilibrium.argtypes = [ctypes.c_long, _D, _D, _D]
        L.or_moments.argtypes = [ctypes.c_long, _D, _D, _D]
        L.or_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), _D]
        L.or_max_threads.restype = ctypes.c_int
        L.or_mesh_crossing.argtypes = [_D, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        L.or_mesh_crossing.restype = ctypes.c_int
        L.or_mesh_inside.argtypes = [_D, _I32, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_mesh_inside.restype = ctypes.c_int
        L.or_ray_triangle.argtypes = [_D, _D, _D, _D, _D, _D, _D, _D]
        L.or_ray_triangle.restype = ctypes.c_int
        L.or_closest_on_triangle.argtypes = [_D, _D, _D, _D, _D]
        L.or_closest_on_triangle.restype = ctypes.c_double
        L.or_mesh_closest_velocity.argtypes = [_D, _D, _I32, ctypes.c_int, _D, _D, _D]
        L.or_mesh_link.argtypes = [_D, _D, _I32, ctypes.c_int, _D, ctypes.c_int, _D, _D]
        L.or_mesh_link.restype = ctypes.c_int
        _lib = L
    return _lib


def adj_lib():
    """The FP64 adjoint of the oracle step (elbm_oracle_adjoint.cpp)."""
    global _adj_lib
    if _adj_lib is None:
        if not os.path.exists(_ADJ_LIB_PATH):
            build()
        L = ctypes.CDLL(_ADJ_LIB_PATH)
        L.oa_collide.argtypes = [_D, ctypes.c_double, _D, ctypes.c_int]
        L.oa_collide_vjp.argtypes = [_D, ctypes.c_double, _D, ctypes.c_int, _D, _D, _D]
        L.oa_grad_pressure_vjp.argtypes = [ctypes.c_double, _D, _D, ctypes.c_double, _D, _D, _D, _D, _D]
        L.oa_link_fraction.argtypes = [ctypes.POINTER(Body), _D, _D, ctypes.c_int, _D]
        L.oa_link_fraction.restype = ctypes.c_double
        L.oa_adjoint_step.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Body), ctypes.c_int, ctypes.c_double,
                                      _D, _U8, _U8, _D, _D, _D, _D, _D, _D, _D, _D]
        L.oa_adjoint_step.restype = ctypes.c_int
        _adj_lib = L
    return _adj_lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _i32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I32)


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_U8)


# ----------------------------------------------------------------------------- single-node routines
def lattice():
    c = (ctypes.c_int32 * 81)()
    w = (ctypes.c_double * 27)()
    lib().or_lattice(c, w)
    return np.array(c[:], dtype=np.int64).reshape(27, 3), np.array(w[:])


def beta_from_nu(nu: float) -> float:
    return lib().or_beta_from_nu(nu)


def feq(rho: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(27)
    lib().or_feq(rho, _dp(u), _dp(out))
    return out


def collide(f, beta: float, F=None, gamma_fixed: float = 0.0, central: bool = False):
    """KBC collision of one node (central: the central-moment s). Returns (f_post, gamma, guard_used)."""
    f = np.array(f, dtype=np.float64).copy()
    g = ctypes.c_int(0)
    Fp = _dp(np.ascontiguousarray(F, dtype=np.float64)) if F is not None else None
    fn = lib().or_collide_central if central else lib().or_collide_ex
    gam = fn(_dp(f), beta, Fp, gamma_fixed, ctypes.byref(g))
    return f, gam, bool(g.value)


def shear_part_central(f, u) -> np.ndarray:
    out = np.zeros(27)
    lib().or_shear_part_central(_dp(np.ascontiguousarray(f, dtype=np.float64)),
                                _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(out))
    return out


def gamma_exact(f, beta: float) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().or_gamma_exact(_dp(f), beta)


def H(f) -> float:
    return lib().or_H(_dp(np.ascontiguousarray(f, dtype=np.float64)))


def shear_part(f) -> np.ndarray:
    out = np.zeros(27)
    lib().or_shear_part(_dp(np.ascontiguousarray(f, dtype=np.float64)), _dp(out))
    return out


def grad_dist(rho: float, u, Pi) -> np.ndarray:
    out = np.zeros(27)
    lib().or_grad_dist(rho, _dp(np.ascontiguousarray(u, dtype=np.float64)),
                       _dp(np.ascontiguousarray(np.asarray(Pi, dtype=np.float64).reshape(9))), _dp(out))
    return out


def pressure(rho: float, u, G, beta: float) -> np.ndarray:
    out = np.zeros(9)
    lib().or_pressure(rho, _dp(np.ascontiguousarray(u, dtype=np.float64)),
                      _dp(np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(9))), beta, _dp(out))
    return out.reshape(3, 3)


def collide_adjoint(f, beta: float, gout, F=None, lbgk: bool = False):
    """(df'/df)^T gout and (df'/dF)^T gout of one node's collision, from the adjoint library."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(gout, dtype=np.float64)
    gf, gF = np.zeros(27), np.zeros(3)
    Fp = _dp(np.ascontiguousarray(F, dtype=np.float64)) if F is not None else None
    adj_lib().oa_collide_vjp(_dp(f), beta, Fp, 1 if lbgk else 0, _dp(g), _dp(gf), _dp(gF))
    return gf, gF


def collide_restated(f, beta: float, F=None, lbgk: bool = False):
    """The adjoint library's own restatement of one node's collision (values)."""
    f = np.array(f, dtype=np.float64)
    Fp = _dp(np.ascontiguousarray(F, dtype=np.float64)) if F is not None else None
    adj_lib().oa_collide(_dp(f), beta, Fp, 1 if lbgk else 0)
    return f


def grad_pressure_adjoint(rho: float, u, G, beta: float, gout):
    """Grad's distribution at (rho, u, Pi(rho, u, G)) and its transposed derivative (g_rho, g_u, g_G)."""
    out, gu, gG, gr = np.zeros(27), np.zeros(3), np.zeros(9), np.zeros(1)
    adj_lib().oa_grad_pressure_vjp(rho, _dp(np.ascontiguousarray(u, dtype=np.float64)),
                                   _dp(np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(9))), beta,
                                   _dp(np.ascontiguousarray(gout, dtype=np.float64)), _dp(out), _dp(gr), _dp(gu),
                                   _dp(gG))
    return out, float(gr[0]), gu, gG.reshape(3, 3)


def link_fraction_adjoint(body, c, xb, i: int):
    """(q, dq/dc) of a link of a sphere or plane with centre c, from the adjoint library."""
    g = np.zeros(3)
    q = adj_lib().oa_link_fraction(ctypes.byref(body), _dp(np.asarray(c, dtype=np.float64)),
                                   _dp(np.asarray(xb, dtype=np.float64)), int(i), _dp(g))
    return q, g


# ----------------------------------------------------------------------------- bodies
def make_body(kind="sphere", center=(0, 0, 0), radius=0.0, normal=(0, 0, 0), amp=0.0, period=0.0,
              direction=(0, 0, 0), vel=(0, 0, 0), omega=(0, 0, 0), motion="prescribed", density_ratio=0.0,
              gravity=(0, 0, 0)) -> Body:
    """A body for ``or_step``.  motion="free": a sphere moved by the fluid force, gravity and
    buoyancy (its track is set by ``Simulation`` each step; density_ratio = rho_s / rho_f);
    motion="free_rotating": the same, also turned by the torque (omega = initial angular velocity)."""
    b = Body()
    b.tracked = 1 if motion in ("free", "free_rotating") else 0
    b.kind = 0 if kind == "sphere" else 1
    b.p0[:] = list(map(float, center))
    b.radius = float(radius)
    b.normal[:] = list(map(float, normal))
    b.amp = float(amp)
    b.period = float(period)
    b.dir[:] = list(map(float, direction))
    b.vel[:] = list(map(float, vel))
    b.omega[:] = list(map(float, omega))
    return b


def body_from_spec(spec: dict) -> Body:
    if spec.get("kind") == "mesh":
        b = Body()
        b.kind = 2
        b.tracked = 1
        return b
    return make_body(**spec)


# ----------------------------------------------------------------------------- triangulated bodies
def _mesh_arrays(verts, tris, vels=None):
    X = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
    T = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    V = np.zeros_like(X) if vels is None else np.ascontiguousarray(vels, dtype=np.float64).reshape(-1, 3)
    return X, T, V


def mesh_inside(verts, tris, x, y, z) -> bool:
    X, T, _ = _mesh_arrays(verts, tris)
    return bool(lib().or_mesh_inside(_dp(X), _i32(T), len(T), float(x), float(y), float(z)))


def mesh_crossing(A, B, C, y, z):
    """x of the crossing of the +x ray through (y, z) with triangle ABC, or None."""
    xc = np.zeros(1)
    ok = lib().or_mesh_crossing(_dp(np.asarray(A, float)), _dp(np.asarray(B, float)), _dp(np.asarray(C, float)),
                                float(y), float(z), _dp(xc))
    return float(xc[0]) if ok else None


def mesh_link(verts, tris, vels, xb, i: int):
    """(hit, q, wall velocity) of the link of node xb in direction i."""
    X, T, V = _mesh_arrays(verts, tris, vels)
    q = np.zeros(1)
    uw = np.zeros(3)
    hit = lib().or_mesh_link(_dp(X), _dp(V), _i32(T), len(T), _dp(np.asarray(xb, float)), int(i), _dp(q), _dp(uw))
    return bool(hit), float(q[0]), uw


def mesh_closest_velocity(verts, tris, vels, p):
    """(velocity, squared distance) of the surface point closest to p."""
    X, T, V = _mesh_arrays(verts, tris, vels)
    out = np.zeros(3)
    d2 = np.zeros(1)
    lib().or_mesh_closest_velocity(_dp(X), _dp(V), _i32(T), len(T), _dp(np.asarray(p, float)), _dp(out), _dp(d2))
    return out, float(d2[0])


def closest_on_triangle(p, A, B, C):
    w = np.zeros(3)
    d2 = lib().or_closest_on_triangle(_dp(np.asarray(p, float)), _dp(np.asarray(A, float)),
                                      _dp(np.asarray(B, float)), _dp(np.asarray(C, float)), _dp(w))
    return d2, w


def kinematics(body: Body, t: float):
    c = np.zeros(3)
    U = np.zeros(3)
    lib().or_kinematics(ctypes.byref(body), t, _dp(c), _dp(U))
    return c, U


def q_link(body: Body, t: float, xb, i: int) -> float:
    c, _ = kinematics(body, t)
    return lib().or_q(ctypes.byref(body), _dp(c), _dp(np.asarray(xb, dtype=np.float64)), i)


# ----------------------------------------------------------------------------- simulation
class Simulation:
    """Time loop around ``or_step``.  ``A`` holds the post-collision populations."""

    def __init__(self, shape, nu: float, rho=None, u=None, bodies=(), channel: bool = False,
                 u_in=(0.0, 0.0, 0.0), rho0: float = 1.0, F=None, beta: float | None = None,
                 stream_only: bool = False, A0=None, stabiliser: str = "kbc", central: bool = False):
        nx, ny, nz = shape
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.grid = Grid()
        self.grid.nx, self.grid.ny, self.grid.nz = nx, ny, nz
        self.grid.channel = 1 if channel else 0
        self.grid.beta = beta_from_nu(nu) if beta is None else beta
        self.grid.rho0 = rho0
        self.grid.u_in[:] = list(map(float, u_in))
        self.grid.stream_only = 1 if stream_only else 0
        self.grid.stabiliser = {"kbc": 0, "exact": 1, "lbgk": 2}[stabiliser]
        if central and stabiliser != "kbc":
            raise ValueError("the central-moment variant uses the analytic stabiliser")
        self.grid.central = 1 if central else 0
        self.bodies = (Body * max(1, len(bodies)))(*[body_from_spec(b) if isinstance(b, dict) else b
                                                      for b in bodies])
        self.nb = len(bodies)
        self.t = 0
        # freely moving spheres (two-way coupling, Sec. IV.A): Newton's equations
        #   dx/dt = u,  du/dt = F/m + (1 - rho_f/rho_s) g,  m = rho_s (4/3) pi R^3,
        # explicit Euler with unit time step, F the momentum-exchange force of the last step
        # (zero before the first one):  x(t+1) = x(t) + u(t),  u(t+1) = u(t) + F(t)/m + (1 - 1/ratio) g;
        # a rotating one also  w(t+1) = w(t) + M(t)/I,  I = (2/5) m R^2 (solid sphere), M the torque
        # about its centre of the last step
        self.free = {}
        for k, spec in enumerate(bodies):
            if isinstance(spec, dict) and spec.get("motion") in ("free", "free_rotating"):
                ratio = float(spec["density_ratio"])
                R = float(spec["radius"])
                m = ratio * rho0 * (4.0 / 3.0) * math.pi * R ** 3
                rot = spec.get("motion") == "free_rotating"
                self.free[k] = dict(m=m, I=0.4 * m * R * R, rot=rot,
                                    ab=(1.0 - 1.0 / ratio) * np.asarray(spec.get("gravity", (0, 0, 0)), float),
                                    x=np.asarray(spec["center"], float).copy(),
                                    u=np.asarray(spec.get("vel", (0, 0, 0)), float).copy(), F=np.zeros(3),
                                    w=np.asarray(spec.get("omega", (0, 0, 0)) if rot else (0, 0, 0), float).copy(),
                                    M=np.zeros(3))
        # triangulated bodies (Sec. IV.C): vertex positions and velocities of the current time level
        # and, when mesh_next() was called, of the next one (else the mesh holds still)
        self.meshes = {}
        for k, spec in enumerate(bodies):
            if isinstance(spec, dict) and spec.get("kind") == "mesh":
                X, T, V = _mesh_arrays(spec["verts"], spec["tris"], spec.get("vels"))
                ref = np.asarray(spec["center"], float) if spec.get("center") is not None else X.mean(0)
                self.meshes[k] = dict(T=T, X=[X, X], V=[V, V], ref=[ref, ref], next=False)
        self._set_tracks()
        self.F = None if F is None else np.ascontiguousarray(F, dtype=np.float64).reshape(3, nz, ny, nx)
        self.A = np.zeros((27, nz, ny, nx))
        if u is None:
            u = np.zeros((3, nz, ny, nx))
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, nz, ny, nx)
        rp = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(nz, ny, nx)
        if A0 is not None:
            self.A = np.ascontiguousarray(A0, dtype=np.float64).reshape(27, nz, ny, nx).copy()
        else:
            lib().or_init_equilibrium(self.N, _dp(rp) if rp is not None else None, _dp(u), _dp(self.A))
        self.B = np.zeros_like(self.A)
        self.solid = self.mask(0)
        self.forces = []      # per step: array (nb, 6) for the step producing A^{t+1}
        self.stats = []
        self.frozen_masks = None   # optional list of masks indexed by time level

    def mask(self, t: float) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.zeros((nz, ny, nx), dtype=np.uint8)
        if self.nb:
            lib().or_solid_mask(ctypes.byref(self.grid), self.bodies, self.nb, float(t), _u8(out))
        return out

    def mesh_next(self, k: int, verts, vels, center=None):
        """Vertex positions and velocities of triangulated body k at the next time level."""
        m = self.meshes[k]
        X, _, V = _mesh_arrays(verts, m["T"], vels)
        assert X.shape == m["X"][0].shape
        m["X"][1], m["V"][1] = X, V
        m["ref"][1] = np.asarray(center, float) if center is not None else X.mean(0)
        m["next"] = True

    def _set_tracks(self):
        """Centre and velocity of each free sphere at t and t+1 (explicit Euler); the two mesh
        levels of each triangulated body."""
        for k, m in self.meshes.items():
            b = self.bodies[k]
            if not m["next"]:
                m["X"][1], m["V"][1], m["ref"][1] = m["X"][0], m["V"][0], m["ref"][0]
            for lv in range(2):
                b.mesh_X[lv] = _dp(m["X"][lv])
                b.mesh_V[lv] = _dp(m["V"][lv])
                for a in range(3):
                    b.track_c[lv][a] = m["ref"][lv][a]
                    b.track_U[lv][a] = 0.0
            b.mesh_tri = _i32(m["T"])
            b.mesh_nv = len(m["X"][0])
            b.mesh_nt = len(m["T"])
            b.mesh_t = float(self.t)
            b.track_t = float(self.t)
        for k, fb in self.free.items():
            b = self.bodies[k]
            x1 = fb["x"] + fb["u"]
            u1 = fb["u"] + fb["F"] / fb["m"] + fb["ab"]
            w1 = fb["w"] + fb["M"] / fb["I"] if fb["rot"] else fb["w"]
            b.track_t = float(self.t)
            for a in range(3):
                b.track_c[0][a], b.track_c[1][a] = fb["x"][a], x1[a]
                b.track_U[0][a], b.track_U[1][a] = fb["u"][a], u1[a]
                b.track_W[0][a], b.track_W[1][a] = fb["w"][a], w1[a]

    def body_state(self, k: int):
        """Centre and velocity of free body k at the current time level."""
        return self.free[k]["x"].copy(), self.free[k]["u"].copy()

    def body_spin(self, k: int):
        """Angular velocity of free body k at the current time level."""
        return self.free[k]["w"].copy()

    def step(self, n: int = 1, record_masks: list | None = None):
        for _ in range(n):
            self._set_tracks()
            if self.frozen_masks is not None:
                s1 = self.frozen_masks[self.t + 1]
            else:
                s1 = self.mask(self.t + 1)
            if record_masks is not None:
                if not record_masks:
                    record_masks.append(self.solid.copy())
                record_masks.append(s1.copy())
            forces = np.zeros(max(1, self.nb) * 6)
            st = Stats()
            Fp = _dp(self.F) if self.F is not None else None
            rc = lib().or_step(ctypes.byref(self.grid), self.bodies, self.nb, float(self.t), _dp(self.A),
                               _u8(self.solid), _u8(s1), Fp, _dp(self.B), _dp(forces), ctypes.byref(st))
            if rc != 0:
                raise RuntimeError(f"or_step failed: {rc}")
            self.A, self.B = self.B, self.A
            self.solid = s1
            self.t += 1
            self.forces.append(forces[: 6 * self.nb].reshape(self.nb, 6).copy() if self.nb else np.zeros((0, 6)))
            self.stats.append({k: getattr(st, k) for k, _ in Stats._fields_})
            for m in self.meshes.values():
                m["X"][0], m["V"][0], m["ref"][0] = m["X"][1], m["V"][1], m["ref"][1]
                m["next"] = False
            for k, fb in self.free.items():
                b = self.bodies[k]
                fb["x"] = np.array([b.track_c[1][a] for a in range(3)])
                fb["u"] = np.array([b.track_U[1][a] for a in range(3)])
                fb["w"] = np.array([b.track_W[1][a] for a in range(3)])
                fb["F"] = self.forces[-1][k, :3].copy()
                fb["M"] = self.forces[-1][k, 3:].copy()
        return self

    def adjoint_step(self, lam, w_force=None, solid_t1=None):
        """FP64 adjoint of the step t -> t+1 from the current state (oracle adjoint; masks frozen at
        the current mask and at solid_t1, default the frozen or computed mask of t+1):
        for L = <lam, A^{t+1}> + sum_k w_k . F_k(t+1) returns (dL/dA^t, dL/dF or None, dL/d(amp_k),
        A^{t+1}, forces) -- the last two the adjoint library's own forward values.  The state is
        left unchanged."""
        nx, ny, nz = self.shape
        if solid_t1 is None:
            solid_t1 = self.frozen_masks[self.t + 1] if self.frozen_masks is not None else self.mask(self.t + 1)
        s1 = np.ascontiguousarray(solid_t1, dtype=np.uint8)
        self._set_tracks()
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(27, nz, ny, nx)
        out = np.zeros_like(self.A)
        A1 = np.zeros_like(self.A)
        gF = np.zeros((3, nz, ny, nx)) if self.F is not None else None
        gamp = np.zeros(max(1, self.nb))
        forces = np.zeros(max(1, self.nb) * 3)
        w = None
        if w_force is not None:
            w = np.ascontiguousarray(np.asarray(w_force, dtype=np.float64).reshape(-1))
        rc = adj_lib().oa_adjoint_step(ctypes.byref(self.grid), self.bodies, self.nb, float(self.t), _dp(self.A),
                                       _u8(self.solid), _u8(s1), _dp(self.F) if self.F is not None else None,
                                       _dp(lam), _dp(w) if w is not None else None, _dp(out),
                                       _dp(gF) if gF is not None else None, _dp(gamp), _dp(A1), _dp(forces))
        if rc != 0:
            raise RuntimeError(f"oa_adjoint_step failed: {rc}")
        return out, gF, gamp[: self.nb], A1, forces[: 3 * self.nb].reshape(self.nb, 3)

    def moments(self):
        rho = np.zeros(self.N)
        j = np.zeros(3 * self.N)
        lib().or_moments(self.N, _dp(self.A), _dp(rho), _dp(j))
        nx, ny, nz = self.shape
        return rho.reshape(nz, ny, nx), j.reshape(3, nz, ny, nx)

    def velocity(self):
        """Physical velocity U = (j - F/2)/rho of the stored state (previous-step macroscopic field)."""
        rho, j = self.moments()
        if self.F is not None:
            j = j - 0.5 * self.F
        return rho, j / rho

    def macro(self):
        """Previous-step fields (U^t, R^t) of the current state, as the step uses them."""
        nx, ny, nz = self.shape
        U = np.zeros((3, nz, ny, nx))
        R = np.zeros((nz, ny, nx))
        Fp = _dp(self.F) if self.F is not None else None
        lib().or_macro(ctypes.byref(self.grid), self.bodies, self.nb, float(self.t), _dp(self.A), _u8(self.solid), Fp,
                       _dp(U), _dp(R))
        return U, R

    def refill_state(self, solid_t1: np.ndarray):
        """The current state with the nodes uncovered at t+1 refilled (first phase of a step)."""
        U, R = self.macro()
        Aw = np.zeros_like(self.A)
        cnt = ctypes.c_int64(0)
        lib().or_refill_state(ctypes.byref(self.grid), self.bodies, self.nb, float(self.t), _dp(self.A),
                              _u8(self.solid), _u8(np.ascontiguousarray(solid_t1)), _dp(U), _dp(R), _dp(Aw),
                              ctypes.byref(cnt))
        return Aw, cnt.value, U, R

    def grad_u(self, U: np.ndarray, solid_t1: np.ndarray, x: int, y: int, z: int) -> np.ndarray:
        G = np.zeros(9)
        U = np.ascontiguousarray(U, dtype=np.float64)
        lib().or_grad_u(ctypes.byref(self.grid), _dp(U), _u8(np.ascontiguousarray(solid_t1)), x, y, z, _dp(G))
        return G.reshape(3, 3)


def force_rollout_adjoint(shape, nu, bodies, steps: int, weights, rho=None, u=None, F=None, channel=False,
                          u_in=(0.0, 0.0, 0.0), checkpoint: int = 10, masks=None):
    """FP64 gradient of L = sum_t w_t . F_0(t+1) (the momentum-exchange force on body 0 after the step
    t -> t+1, t = 0..steps-1) over a rollout from the equilibrium of (rho, u), by the oracle adjoint:
    the forward run keeps a checkpoint every `checkpoint` steps (and records the solid masks, or takes
    the given ones, frozen); the reverse sweep recomputes each segment's states and applies
    Simulation.adjoint_step backwards.  Returns (L, dL/dF or None, dL/d(amp_k), masks)."""
    wts = np.asarray(weights, dtype=np.float64).reshape(steps, 3)

    def fresh(A0=None):
        sim = Simulation(shape, nu, rho, u, bodies=bodies, channel=channel, u_in=u_in, F=F, A0=A0)
        if masks is not None:
            sim.frozen_masks = masks
            sim.solid = masks[0].copy()
        return sim

    sim = fresh()
    rec = []
    ckpt = {0: sim.A.copy()}
    for t in range(steps):
        sim.step(1, record_masks=rec if masks is None else None)
        if (t + 1) % checkpoint == 0 and t + 1 < steps:
            ckpt[t + 1] = sim.A.copy()
    mk = masks if masks is not None else {k: m for k, m in enumerate(rec)}
    L = float(sum(wts[t] @ sim.forces[t][0, :3] for t in range(steps)))
    nb = len(bodies)
    w_all = np.zeros((steps, max(1, nb), 3))
    w_all[:, 0, :] = wts
    nx, ny, nz = shape
    lam = np.zeros((27, nz, ny, nx))
    gF = np.zeros((3, nz, ny, nx)) if F is not None else None
    gamp = np.zeros(nb)
    for s0 in sorted(ckpt, reverse=True):
        s1 = min(s0 + checkpoint, steps)
        seg = Simulation(shape, nu, bodies=bodies, channel=channel, u_in=u_in, F=F, A0=ckpt[s0])
        seg.t = s0
        seg.frozen_masks = mk
        seg.solid = mk[s0].copy()
        states = [seg.A.copy()]
        for _ in range(s0, s1 - 1):
            seg.step(1)
            states.append(seg.A.copy())
        for t in reversed(range(s0, s1)):
            back = Simulation(shape, nu, bodies=bodies, channel=channel, u_in=u_in, F=F, A0=states[t - s0])
            back.t = t
            back.frozen_masks = mk
            back.solid = mk[t].copy()
            lam, g, ga, _, _ = back.adjoint_step(lam, w_all[t, :nb])
            if gF is not None:
                gF += g
            gamp += ga
    return L, gF, gamp, mk


def max_threads() -> int:
    return lib().or_max_threads()
