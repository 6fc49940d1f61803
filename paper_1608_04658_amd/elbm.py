"""ctypes binding of the C ABI in ``include/elbm.h`` (argument marshalling only).

Every step of the lattice Boltzmann path runs in ``libelbm.so`` (HIP kernels for gfx950).
PyTorch provides the device memory (the workspace tensor, input and output tensors) and the
stream.  The functions below carry the C names; ``Lattice`` is a small convenience owner of a
context and its workspace.  There is no fallback: if the library is not built or no GPU is
present, loading fails with an exception.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "elbm.h")

STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
LAYOUT_SOA, LAYOUT_ROWS = 0, 1  # storage arrays [27][nz][ny][nx] or [nz][ny][27][nx]
BC_PERIODIC, BC_CHANNEL = 0, 1
BODY_SPHERE, BODY_PLANE, BODY_MESH = 0, 1, 2
MOTION_PRESCRIBED, MOTION_FREE, MOTION_FREE_ROTATING = 0, 1, 2
MAX_BODIES = 8
FLAG_BODY_FORCE, FLAG_STREAM_ONLY, FLAG_NO_FP64, FLAG_ADJOINT, FLAG_EXACT_GAMMA, FLAG_LBGK, FLAG_CENTRAL = \
    1, 2, 4, 8, 16, 32, 64


class ElbmError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("max_bodies", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("force_ring", ctypes.c_int32), ("max_boundary", ctypes.c_int64),
                ("nu", ctypes.c_double), ("rho0", ctypes.c_double), ("u_inlet", ctypes.c_double * 3),
                ("fp64_threshold", ctypes.c_double), ("max_mesh_vertices", ctypes.c_int32),
                ("max_mesh_triangles", ctypes.c_int32)]


class Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("motion", ctypes.c_int32), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("normal", ctypes.c_double * 3), ("amp", ctypes.c_double),
                ("period", ctypes.c_double), ("dir", ctypes.c_double * 3), ("vel", ctypes.c_double * 3),
                ("omega", ctypes.c_double * 3), ("density_ratio", ctypes.c_double),
                ("gravity", ctypes.c_double * 3)]


class Info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("nodes", ctypes.c_int64), ("beta", ctypes.c_double),
                ("pop_bytes", ctypes.c_size_t), ("pop_offset", ctypes.c_size_t), ("flags_offset", ctypes.c_size_t),
                ("storage", ctypes.c_int32), ("nbodies", ctypes.c_int32), ("boundary_nodes", ctypes.c_int64),
                ("fp64_nodes", ctypes.c_int64), ("layout", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("gamma_min", ctypes.c_double), ("gamma_max", ctypes.c_double), ("nonfinite", ctypes.c_int32),
                ("gamma_stats", ctypes.c_int32)]


_lib = None
_VP = ctypes.c_void_p


def load():
    """Load libelbm.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ElbmError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "elbm_workspace_bytes": [P(Params), P(ctypes.c_size_t)],
        "elbm_create": [P(Params), _VP, _VP, ctypes.c_size_t, P(_VP)],
        "elbm_destroy": [_VP],
        "elbm_set_stream": [_VP, _VP],
        "elbm_init_equilibrium": [_VP, _VP, _VP],
        "elbm_write_populations": [_VP, _VP, ctypes.c_int64],
        "elbm_read_populations": [_VP, _VP],
        "elbm_set_geometry": [_VP, P(Body), ctypes.c_int32],
        "elbm_set_mesh": [_VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double),
                          P(ctypes.c_double)],
        "elbm_mesh_next": [_VP, _VP, _VP, P(ctypes.c_double)],
        "elbm_body_state": [_VP, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double)],
        "elbm_body_spin": [_VP, ctypes.c_int32, P(ctypes.c_double)],
        "elbm_set_body_force": [_VP, _VP],
        "elbm_step": [_VP, ctypes.c_int32],
        "elbm_step_into": [_VP, _VP, ctypes.c_uint32],
        "elbm_force": [_VP, ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double)],
        "elbm_force_history": [_VP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P(ctypes.c_double)],
        "elbm_read_flags": [_VP, _VP],
        "elbm_get_info": [_VP, P(Info)],
        "elbm_collide_nodes": [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                               _VP],
        "elbm_save_state": [_VP, _VP],
        "elbm_load_state": [_VP, _VP, ctypes.c_int64],
        "elbm_adjoint_step": [_VP, ctypes.c_int64, _VP, _VP, _VP, P(ctypes.c_double), _VP],
        "elbm_adjoint_param_grad": [_VP, P(ctypes.c_double), ctypes.c_int32],
        "elbm_set_timing": [_VP, ctypes.c_int32],
        "elbm_get_timing": [_VP, P(ctypes.c_double), P(ctypes.c_int64)],
        "elbm_step_periodic_noalloc": [P(Params), _VP, _VP, _VP],
        "elbm_set_diagnostics": [_VP, ctypes.c_int32],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.elbm_last_error.argtypes = [_VP]
    L.elbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def header_symbols() -> list[str]:
    """Entry points declared in include/elbm.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(elbm_[a-z_0-9]+)\s*\(", text)))


def _check(rc: int, ctx=None):
    if rc != 0:
        msg = load().elbm_last_error(ctx).decode(errors="replace")
        raise ElbmError(f"elbm error {rc}: {msg}")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_cuda:
            raise ElbmError("expected a device tensor")
        if not t.is_contiguous():
            raise ElbmError("expected a contiguous tensor")
        return t.data_ptr()
    return int(t)


def _stream_handle(stream=None) -> int:
    if isinstance(stream, int):
        return stream
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_params(shape, nu, storage="f32", channel=False, max_bodies=0, flags=0, force_ring=4096, max_boundary=0,
                rho0=1.0, u_inlet=(0.0, 0.0, 0.0), fp64_threshold=0.0, max_mesh_vertices=0,
                max_mesh_triangles=0) -> Params:
    p = Params()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.bc_x = BC_CHANNEL if channel else BC_PERIODIC
    p.max_bodies = int(max_bodies)
    p.flags = int(flags)
    p.force_ring = int(force_ring)
    p.max_boundary = int(max_boundary)
    p.nu = float(nu)
    p.rho0 = float(rho0)
    p.u_inlet[:] = [float(v) for v in u_inlet]
    p.fp64_threshold = float(fp64_threshold)
    p.max_mesh_vertices = int(max_mesh_vertices)
    p.max_mesh_triangles = int(max_mesh_triangles)
    return p


def make_body(spec: dict) -> Body:
    b = Body()
    b.kind = {"sphere": BODY_SPHERE, "plane": BODY_PLANE, "mesh": BODY_MESH}[spec.get("kind", "sphere")]
    b.center[:] = [float(v) for v in spec.get("center", (0, 0, 0))]
    b.radius = float(spec.get("radius", 0.0))
    b.normal[:] = [float(v) for v in spec.get("normal", (0, 0, 0))]
    b.amp = float(spec.get("amp", 0.0))
    b.period = float(spec.get("period", 0.0))
    b.dir[:] = [float(v) for v in spec.get("direction", (0, 0, 0))]
    b.vel[:] = [float(v) for v in spec.get("vel", (0, 0, 0))]
    b.omega[:] = [float(v) for v in spec.get("omega", (0, 0, 0))]
    b.motion = {"prescribed": MOTION_PRESCRIBED, "free": MOTION_FREE,
                "free_rotating": MOTION_FREE_ROTATING}[spec.get("motion", "prescribed")]
    b.density_ratio = float(spec.get("density_ratio", 0.0))
    b.gravity[:] = [float(v) for v in spec.get("gravity", (0, 0, 0))]
    return b


# ----------------------------------------------------------------------------- C-named wrappers
def elbm_workspace_bytes(params: Params) -> int:
    n = ctypes.c_size_t(0)
    _check(load().elbm_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def elbm_create(params: Params, stream, workspace, ws_bytes: int):
    ctx = _VP()
    _check(load().elbm_create(ctypes.byref(params), stream, _ptr(workspace), ws_bytes, ctypes.byref(ctx)))
    return ctx


def elbm_destroy(ctx):
    _check(load().elbm_destroy(ctx))


def elbm_set_stream(ctx, stream):
    _check(load().elbm_set_stream(ctx, stream), ctx)


def elbm_init_equilibrium(ctx, rho_dev, u_dev):
    _check(load().elbm_init_equilibrium(ctx, _ptr(rho_dev), _ptr(u_dev)), ctx)


def elbm_write_populations(ctx, pop_dev, t: int):
    _check(load().elbm_write_populations(ctx, _ptr(pop_dev), int(t)), ctx)


def elbm_read_populations(ctx, pop_dev):
    _check(load().elbm_read_populations(ctx, _ptr(pop_dev)), ctx)


def elbm_set_geometry(ctx, bodies):
    arr = (Body * max(1, len(bodies)))(*[make_body(b) if isinstance(b, dict) else b for b in bodies])
    _check(load().elbm_set_geometry(ctx, arr, len(bodies)), ctx)


def _d3(v):
    return None if v is None else (ctypes.c_double * 3)(*[float(a) for a in v])


def elbm_set_mesh(ctx, tris_dev, nt: int, verts_dev, vels_dev, nv: int, box_lo, box_hi, center=None):
    _check(load().elbm_set_mesh(ctx, _ptr(tris_dev), int(nt), _ptr(verts_dev), _ptr(vels_dev), int(nv), _d3(box_lo),
                                _d3(box_hi), _d3(center)), ctx)


def elbm_mesh_next(ctx, verts_dev, vels_dev, center=None):
    _check(load().elbm_mesh_next(ctx, _ptr(verts_dev), _ptr(vels_dev), _d3(center)), ctx)


def elbm_body_state(ctx, body: int):
    pos = (ctypes.c_double * 3)()
    vel = (ctypes.c_double * 3)()
    _check(load().elbm_body_state(ctx, int(body), pos, vel), ctx)
    return list(pos), list(vel)


def elbm_body_spin(ctx, body: int):
    w = (ctypes.c_double * 3)()
    _check(load().elbm_body_spin(ctx, int(body), w), ctx)
    return list(w)


def elbm_set_body_force(ctx, F_dev):
    _check(load().elbm_set_body_force(ctx, _ptr(F_dev)), ctx)


def elbm_step(ctx, nsteps: int = 1):
    _check(load().elbm_step(ctx, int(nsteps)), ctx)


STEP_SKIP_FORCE = 1


def elbm_step_into(ctx, pop_next, skip_force: bool = False):
    """One step whose new populations go to the device tensor `pop_next` (27 N elements of the
    storage type), which becomes the current population buffer; skip_force leaves the step's force
    unsummed (its ring slot keeps what it held)."""
    _check(load().elbm_step_into(ctx, _ptr(pop_next), STEP_SKIP_FORCE if skip_force else 0), ctx)


def elbm_force(ctx, body: int, step: int):
    F = (ctypes.c_double * 3)()
    M = (ctypes.c_double * 3)()
    _check(load().elbm_force(ctx, int(body), int(step), F, M), ctx)
    return np.array(F[:]), np.array(M[:])


def elbm_force_history(ctx, body: int, first: int, count: int) -> np.ndarray:
    out = np.zeros((count, 6))
    _check(load().elbm_force_history(ctx, int(body), int(first), int(count),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), ctx)
    return out


def elbm_read_flags(ctx, out_dev):
    _check(load().elbm_read_flags(ctx, _ptr(out_dev)), ctx)


def elbm_get_info(ctx) -> Info:
    info = Info()
    _check(load().elbm_get_info(ctx, ctypes.byref(info)), ctx)
    return info


def elbm_set_diagnostics(ctx, gamma_stats: bool):
    _check(load().elbm_set_diagnostics(ctx, 1 if gamma_stats else 0), ctx)


def elbm_save_state(ctx, pop_dev):
    _check(load().elbm_save_state(ctx, _ptr(pop_dev)), ctx)


def elbm_load_state(ctx, pop_dev, t: int):
    _check(load().elbm_load_state(ctx, _ptr(pop_dev), int(t)), ctx)


def elbm_adjoint_step(ctx, t: int, pop_t_dev, lam_in_dev, lam_out_dev, w_force=None, gF_dev=None):
    w = None
    if w_force is not None:
        arr = np.ascontiguousarray(np.asarray(w_force, dtype=np.float64).reshape(-1))
        w = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(load().elbm_adjoint_step(ctx, int(t), _ptr(pop_t_dev), _ptr(lam_in_dev), _ptr(lam_out_dev), w,
                                    _ptr(gF_dev)), ctx)


def elbm_adjoint_param_grad(ctx, nbodies: int, reset: bool = True) -> np.ndarray:
    out = np.zeros(max(1, nbodies))
    _check(load().elbm_adjoint_param_grad(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          1 if reset else 0), ctx)
    return out[:nbodies]


def elbm_set_timing(ctx, enable: bool):
    _check(load().elbm_set_timing(ctx, 1 if enable else 0), ctx)


def elbm_get_timing(ctx):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(load().elbm_get_timing(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def elbm_last_error(ctx=None) -> str:
    return load().elbm_last_error(ctx).decode(errors="replace")


def elbm_collide_nodes(f_in, f_out, gamma, F, n: int, nu: float, fp64_threshold: float = 0.0, flags: int = 0,
                       stream=None):
    _check(load().elbm_collide_nodes(_ptr(f_in), _ptr(f_out), _ptr(gamma), _ptr(F), int(n), float(nu),
                                     float(fp64_threshold), int(flags), _stream_handle(stream)))


def elbm_step_periodic_noalloc(params: Params, pop_in, pop_out, stream=None):
    _check(load().elbm_step_periodic_noalloc(ctypes.byref(params), _ptr(pop_in), _ptr(pop_out),
                                             _stream_handle(stream)))


# ----------------------------------------------------------------------------- convenience owner
class Lattice:
    """One context plus its torch-allocated workspace on the current device and stream."""

    def __init__(self, shape, nu, storage="f32", channel=False, u_inlet=(0.0, 0.0, 0.0), max_bodies=0, flags=0,
                 force_ring=4096, max_boundary=0, rho0=1.0, fp64_threshold=0.0, stream=None, max_mesh_vertices=0,
                 max_mesh_triangles=0):
        import torch
        self.torch = torch
        self.shape = tuple(int(v) for v in shape)
        self.params = make_params(shape, nu, storage, channel, max_bodies, flags, force_ring, max_boundary, rho0,
                                  u_inlet, fp64_threshold, max_mesh_vertices, max_mesh_triangles)
        self._mesh_keep = None
        nbytes = elbm_workspace_bytes(self.params)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # 256-byte aligned device workspace owned by torch
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        self._off = (-base) % 256
        self.ws_ptr = base + self._off
        self.ws_bytes = nbytes
        self.ctx = elbm_create(self.params, self.stream.cuda_stream, self.ws_ptr, nbytes)
        self._bodyforce = None

    def close(self):
        if self.ctx:
            elbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def N(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def init_equilibrium(self, rho, u):
        torch = self.torch
        nx, ny, nz = self.shape
        u_t = torch.as_tensor(np.asarray(u, dtype=np.float64).reshape(3, nz, ny, nx)).cuda().contiguous()
        r_t = None if rho is None else torch.as_tensor(np.asarray(rho, dtype=np.float64).reshape(nz, ny, nx)).cuda()
        elbm_init_equilibrium(self.ctx, r_t, u_t)
        self.stream.synchronize()

    def write_populations(self, pop, t=0):
        torch = self.torch
        nx, ny, nz = self.shape
        p = torch.as_tensor(np.asarray(pop, dtype=np.float64).reshape(27, nz, ny, nx)).cuda().contiguous()
        elbm_write_populations(self.ctx, p, t)
        self.stream.synchronize()

    def set_bodies(self, bodies):
        elbm_set_geometry(self.ctx, list(bodies))

    def _mesh_tensors(self, verts, vels):
        """Device FP64 [nv, 3] tensors from host arrays, or the given device tensors as they are."""
        torch = self.torch

        def dev(a):
            if a is None:
                return None
            if isinstance(a, torch.Tensor) and a.is_cuda:
                if a.dtype != torch.float64 or not a.is_contiguous() or a.dim() != 2 or a.shape[1] != 3:
                    raise ElbmError("mesh arrays on the device must be contiguous float64 [nv, 3]")
                return a
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)).cuda()
        return dev(verts), dev(vels)

    def set_mesh(self, verts, tris, box_lo, box_hi, vels=None, center=None):
        """Triangulated surface at the current time level (host arrays); then set_bodies with a body
        of kind "mesh" last."""
        X, V = self._mesh_tensors(verts, vels)
        if V is not None and V.shape != X.shape:
            raise ElbmError("vels must have the shape of verts")
        T = self.torch.as_tensor(np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)).cuda()
        elbm_set_mesh(self.ctx, T, T.shape[0], X, V, X.shape[0], box_lo, box_hi, center)
        self._mesh_keep = (T, X, V)
        self._mesh_nv = X.shape[0]

    def mesh_next(self, verts, vels=None, center=None):
        """Vertex positions and velocities of the next time level (before the next step)."""
        X, V = self._mesh_tensors(verts, vels)
        if self._mesh_keep is None or X.shape[0] != self._mesh_nv or (V is not None and V.shape != X.shape):
            raise ElbmError("mesh_next needs the vertex count of set_mesh")
        elbm_mesh_next(self.ctx, X, V, center)
        self._mesh_keep = (self._mesh_keep[0], X, V)

    def body_state(self, k: int):
        """Position and velocity of body k at the current time level (numpy arrays)."""
        import numpy as np
        pos, vel = elbm_body_state(self.ctx, k)
        return np.array(pos), np.array(vel)

    def body_spin(self, k: int):
        """Angular velocity of body k at the current time level (numpy array)."""
        return np.array(elbm_body_spin(self.ctx, k))

    def set_body_force(self, F):
        torch = self.torch
        nx, ny, nz = self.shape
        if F is None:
            self._bodyforce = None
            elbm_set_body_force(self.ctx, None)
            return
        Ft = torch.as_tensor(np.asarray(F, dtype=np.float32).reshape(3, nz, ny, nx)).cuda().contiguous()
        self._bodyforce = Ft
        elbm_set_body_force(self.ctx, Ft)

    def step(self, n=1):
        elbm_step(self.ctx, n)

    def populations(self):
        """Current populations as a float64 device tensor (27, nz, ny, nx)."""
        nx, ny, nz = self.shape
        out = self.torch.empty((27, nz, ny, nx), dtype=self.torch.float64, device="cuda")
        elbm_read_populations(self.ctx, out)
        self.stream.synchronize()
        return out

    def flags(self):
        nx, ny, nz = self.shape
        out = self.torch.empty((nz, ny, nx), dtype=self.torch.uint8, device="cuda")
        elbm_read_flags(self.ctx, out)
        self.stream.synchronize()
        return out

    def force(self, body, step):
        return elbm_force(self.ctx, body, step)

    def force_history(self, body, first, count):
        return elbm_force_history(self.ctx, body, first, count)

    def info(self) -> Info:
        return elbm_get_info(self.ctx)

    def state_tensor(self):
        """A new device tensor holding a copy of the current populations in storage format and
        layout (flat, 27 N elements; `storage_shape` gives their arrangement)."""
        torch = self.torch
        dt = {0: torch.float32, 1: torch.float16, 2: torch.int16}[self.params.storage]
        out = torch.empty(27 * self.N, dtype=dt, device="cuda")
        elbm_save_state(self.ctx, out)
        return out

    def load_state(self, state, t):
        elbm_load_state(self.ctx, state, t)

    def storage_shape(self):
        """Shape of the storage arrays in memory order: (27, nz, ny, nx) or (nz, ny, 27, nx)."""
        nx, ny, nz = self.shape
        return (27, nz, ny, nx) if self.info().layout == LAYOUT_SOA else (nz, ny, 27, nx)

    def population_view(self):
        """Zero-copy view of the current population storage in the workspace, indexed
        [i, z, y, x] whatever the layout (a permuted view for the row-interleaved one)."""
        torch = self.torch
        info = self.info()
        dt = {0: torch.float32, 1: torch.float16, 2: torch.int16}[info.storage]
        es = 4 if info.storage == 0 else 2
        if info.pop_offset == 2 ** 64 - 1:
            raise ElbmError("the current populations are in a caller's buffer (elbm_step_into)")
        start = self._off + info.pop_offset
        raw = self._ws[start:start + 27 * self.N * es].view(dt)
        v = raw.view(self.storage_shape())
        return v if info.layout == LAYOUT_SOA else v.permute(2, 0, 1, 3)
