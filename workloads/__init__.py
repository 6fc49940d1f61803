"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This module holds none of the lattice Boltzmann method's arithmetic: it only
builds macroscopic initial fields (density, velocity), body-force fields and
body/geometry descriptions, all in float64 numpy arrays of layout
(component, nz, ny, nx) with x fastest.  Each side turns them into populations
with its own code.

Workloads (sizes, viscosities and step counts of the benchmark configurations):

* ``tg32``      -- 32^3 periodic box, 3-D Taylor-Green vortex, u0 = 0.05, nu = 1e-3, 100 steps.
* ``turb256``   -- 256^3 periodic box, seeded divergence-free field with energy
                   spectrum E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 4, rms 0.04, nu = 0.00815, 1000 steps.
* ``sphere384`` -- 384x192x192 channel, inlet 0.03, sphere R = 12 oscillating in y
                   with amplitude 8 and period 2000, nu = 0.0072, 4000 steps.
* ``turb512``   -- 512^3 periodic box, same recipe with k0 = 8 (seed 1609), 500 steps.
* ``adj128``    -- 128x64x64 channel, inlet 0.03, sphere R = 8 oscillating in y
                   (amplitude 4, period 2000), body force uniform in [-1e-6, 1e-6], nu = 0.0048.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.fft


def node_coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def taylor_green_3d(n: int, u0: float):
    """u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz, w = 0, k = 2 pi / n, rho = 1."""
    x, y, z = node_coords((n, n, n))
    k = 2.0 * math.pi / n
    u = np.zeros((3, n, n, n))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    return np.ones((n, n, n)), u


def taylor_green_2d(nx: int, ny: int, nz: int, u0: float):
    """z-invariant 2-D vortex array: u = u0 sin kx cos ky, v = -u0 cos kx sin ky (nx == ny)."""
    x, y, _ = node_coords((nx, ny, nz))
    kx = 2.0 * math.pi / nx
    ky = 2.0 * math.pi / ny
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(kx * x) * np.cos(ky * y)
    u[1] = -u0 * np.cos(kx * x) * np.sin(ky * y)
    return np.ones((nz, ny, nx)), u


def shear_wave(nx: int, ny: int, nz: int, u0: float, mode: int = 1):
    """u_x = u0 sin(2 pi mode y / ny), all else at rest, rho = 1."""
    _, y, _ = node_coords((nx, ny, nz))
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(2.0 * math.pi * mode * y / ny)
    return np.ones((nz, ny, nx)), u


def uniform_flow(shape, u):
    nx, ny, nz = shape
    out = np.zeros((3, nz, ny, nx))
    for a in range(3):
        out[a] = u[a]
    return np.ones((nz, ny, nx)), out


def turbulence(n: int, k0: float, urms: float, seed: int):
    """Seeded divergence-free random field on an n^3 periodic box.

    Complex Gaussian Fourier amplitudes (numpy default_rng(seed)), projected onto
    the divergence-free subspace, rescaled per integer shell |k| (rounded) to the
    spectrum E(k) ~ k^4 exp(-2 (k/k0)^2), transformed back and scaled to a
    per-component rms of ``urms``.  rho = 1.
    """
    rng = np.random.default_rng(seed)
    kf = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(kf, kf, kr, indexing="ij")
    shp = KX.shape
    a = [(rng.standard_normal(shp, dtype=np.float64) + 1j * rng.standard_normal(shp, dtype=np.float64))
         for _ in range(3)]
    k2 = KX * KX + KY * KY + KZ * KZ
    k2s = np.where(k2 == 0, 1.0, k2)
    kdota = (KX * a[0] + KY * a[1] + KZ * a[2]) / k2s
    a[0] = a[0] - KX * kdota
    a[1] = a[1] - KY * kdota
    a[2] = a[2] - KZ * kdota
    del kdota
    kmag = np.sqrt(k2)
    shell = np.rint(kmag).astype(np.int64)
    nsh = int(shell.max()) + 1
    # energy currently in each shell (rfft half-space: weight 2 for kx > 0 planes, 1 otherwise)
    wgt = np.where(KX > 0, 2.0, 1.0)
    e = (np.abs(a[0]) ** 2 + np.abs(a[1]) ** 2 + np.abs(a[2]) ** 2) * wgt
    e_shell = np.bincount(shell.ravel(), weights=e.ravel(), minlength=nsh)
    ks = np.arange(nsh, dtype=np.float64)
    target = ks ** 4 * np.exp(-2.0 * (ks / k0) ** 2)
    target[0] = 0.0
    scale = np.sqrt(np.divide(target, e_shell, out=np.zeros_like(target), where=e_shell > 0))
    fac = scale[shell]
    del e, wgt, shell, kmag, k2, k2s
    u = np.empty((3, n, n, n))
    for c in range(3):
        u[c] = scipy.fft.irfftn(a[c] * fac, s=(n, n, n), axes=(0, 1, 2), workers=-1)
    a = None
    rms = math.sqrt(float(np.mean(u * u)) )
    u *= urms / rms
    return np.ones((n, n, n)), u


def turbulence_device(n: int, k0: float, urms: float, seed: int, device="cuda"):
    """Same recipe as ``turbulence`` drawn on a torch device (torch.Generator seeded with ``seed``;
    a different random stream from numpy's).  Used for the largest boxes, where the host FFT is slow.
    Returns float64 torch tensors (rho, u) on ``device``."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    kf = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    kr = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    KZ, KY, KX = torch.meshgrid(kf, kf, kr, indexing="ij")
    shp = KX.shape
    a = [torch.complex(torch.randn(shp, generator=g, device=device, dtype=torch.float64),
                       torch.randn(shp, generator=g, device=device, dtype=torch.float64)) for _ in range(3)]
    k2 = KX * KX + KY * KY + KZ * KZ
    k2s = torch.where(k2 == 0, torch.ones_like(k2), k2)
    kdota = (KX * a[0] + KY * a[1] + KZ * a[2]) / k2s
    a = [a[0] - KX * kdota, a[1] - KY * kdota, a[2] - KZ * kdota]
    del kdota
    shell = torch.round(torch.sqrt(k2)).to(torch.int64)
    nsh = int(shell.max().item()) + 1
    wgt = torch.where(KX > 0, 2.0, 1.0)
    e = (a[0].abs() ** 2 + a[1].abs() ** 2 + a[2].abs() ** 2) * wgt
    e_shell = torch.bincount(shell.reshape(-1), weights=e.reshape(-1), minlength=nsh)
    ks = torch.arange(nsh, device=device, dtype=torch.float64)
    target = ks ** 4 * torch.exp(-2.0 * (ks / k0) ** 2)
    target[0] = 0.0
    scale = torch.where(e_shell > 0, torch.sqrt(target / torch.where(e_shell > 0, e_shell, 1.0)), 0.0)
    fac = scale[shell]
    del e, wgt, k2, k2s, KX, KY, KZ
    u = torch.empty((3, n, n, n), device=device, dtype=torch.float64)
    for c in range(3):
        u[c] = torch.fft.irfftn(a[c] * fac, s=(n, n, n), dim=(0, 1, 2))
    del a, fac, shell
    u *= urms / torch.sqrt(torch.mean(u * u))
    return torch.ones((n, n, n), device=device, dtype=torch.float64), u


def body_force(shape, seed: int, amp: float):
    """Per-node body-force field, each component uniform in [-amp, amp]."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3, nz, ny, nx))


def sphere(center, radius, amp=0.0, period=0.0, direction=(0.0, 1.0, 0.0), vel=(0.0, 0.0, 0.0),
           omega=(0.0, 0.0, 0.0)) -> dict:
    return dict(kind="sphere", center=tuple(map(float, center)), radius=float(radius), amp=float(amp),
                period=float(period), direction=tuple(map(float, direction)), vel=tuple(map(float, vel)),
                omega=tuple(map(float, omega)))


def free_sphere(center, radius, density_ratio, gravity=(0.0, 0.0, 0.0), vel=(0.0, 0.0, 0.0), omega=None) -> dict:
    """A sphere moved by the fluid force, gravity and buoyancy (two-way coupling); center and vel
    are its state at the time level at which it is set.  With omega (its angular velocity then) the
    sphere also turns under the fluid torque."""
    d = dict(kind="sphere", center=tuple(map(float, center)), radius=float(radius), vel=tuple(map(float, vel)),
             motion="free", density_ratio=float(density_ratio), gravity=tuple(map(float, gravity)))
    if omega is not None:
        d["motion"] = "free_rotating"
        d["omega"] = tuple(map(float, omega))
    return d


def plane(point, normal, vel=(0.0, 0.0, 0.0)) -> dict:
    return dict(kind="plane", center=tuple(map(float, point)), normal=tuple(map(float, normal)),
                vel=tuple(map(float, vel)))


# ----------------------------------------------------------------------------- named workloads
def taylor_microscale_nu(n: int, k0: float, urms: float, re_lambda: float) -> float:
    """nu = u' lambda / Re_lambda with lambda = n / (pi k0) for the k^4 exp(-2 (k/k0)^2) spectrum."""
    lam = n / (math.pi * k0)
    return urms * lam / re_lambda


WORKLOADS = {
    "tg32": dict(shape=(32, 32, 32), nu=1e-3, steps=100, channel=False, kind="taylor_green", u0=0.05),
    "turb256": dict(shape=(256, 256, 256), nu=taylor_microscale_nu(256, 4, 0.04, 100.0), steps=1000,
                    channel=False, kind="turbulence", k0=4.0, urms=0.04, seed=1608),
    "sphere384": dict(shape=(384, 192, 192), nu=0.0072, steps=4000, channel=True, u_in=(0.03, 0.0, 0.0),
                      bodies=[sphere((96, 96, 96), 12, amp=8, period=2000)]),
    "turb512": dict(shape=(512, 512, 512), nu=taylor_microscale_nu(512, 8, 0.04, 100.0), steps=500,
                    channel=False, kind="turbulence", k0=8.0, urms=0.04, seed=1609),
    "adj128": dict(shape=(128, 64, 64), nu=0.0048, steps=301, channel=True, u_in=(0.03, 0.0, 0.0),
                   bodies=[sphere((32, 32, 32), 8, amp=4, period=2000)], force_seed=1610, force_amp=1e-6,
                   loss_window=(100, 300), checkpoint=20),
}


def initial_field(name: str, shape=None):
    w = WORKLOADS[name]
    shape = shape or w["shape"]
    if w.get("kind") == "taylor_green":
        return taylor_green_3d(shape[0], w["u0"])
    if w.get("kind") == "turbulence":
        return turbulence(shape[0], w["k0"], w["urms"], w["seed"])
    return uniform_flow(shape, w.get("u_in", (0.0, 0.0, 0.0)))
