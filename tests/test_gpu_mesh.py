"""Triangulated bodies on the GPU against the oracle (the deforming geometries of Sec. IV.C):
solid masks bit for bit (including rays through triangle edges and vertices), then whole steps of a
resting box in a channel, a rigidly oscillating sphere mesh and the deforming swimmer.  Measured up to
5.9e-8 on the fluid populations, 6.1e-7 on the force and 3.0e-6 on the torque (relative to the largest
component); bounds 1e-6, 1e-5 and 3e-5."""
import numpy as np
import pytest

import workloads as WL
from workloads import meshes as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def E(torch_cuda):
    from paper_1608_04658_amd import elbm
    elbm.load()
    return elbm


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("kind", ["box_between_planes", "box_on_nodes", "octahedron", "icosphere"])
def test_mesh_mask_bit_exact(E, oracle_mod, kind):
    O = oracle_mod
    shape = (22, 20, 21)
    if kind == "box_between_planes":
        v, t = M.box_mesh((4.3, 5.6, 4.1), (14.6, 13.2, 15.9))
    elif kind == "box_on_nodes":
        v, t = M.box_mesh((4.0, 5.0, 4.0), (14.0, 13.0, 15.0))
    elif kind == "octahedron":
        v, t = M.octahedron_mesh((11.0, 9.0, 10.0), 5.0)
    else:
        v, t = M.icosphere_mesh((10.7, 9.6, 10.2), 5.3, 3)
    lo, hi = v.min(0) - 0.5, v.max(0) + 0.5
    lat = E.Lattice(shape, 0.1, max_bodies=1, max_mesh_vertices=len(v), max_mesh_triangles=len(t))
    rho, u = WL.uniform_flow(shape, (0.0, 0.0, 0.0))
    lat.init_equilibrium(rho, u)
    _say(f"mask {kind}: {len(t)} triangles")
    lat.set_mesh(v, t, lo, hi)
    lat.set_bodies([dict(kind="mesh")])
    got = (lat.flags().cpu().numpy() & 1) > 0
    ref = O.Simulation(shape, 0.1, bodies=[dict(kind="mesh", verts=v, tris=t)]).solid > 0
    _say(f"mask {kind}: {int(ref.sum())} solid nodes, {int((got != ref).sum())} differ")
    assert ref.sum() > 0
    assert np.array_equal(got, ref)


def _compare(E, lat, s, label, steps):
    fluid = s.solid == 0
    got_flags = (lat.flags().cpu().numpy() & 1) > 0
    assert np.array_equal(got_flags, s.solid > 0), "masks differ"
    err = np.max(np.abs(lat.populations().cpu().numpy()[:, fluid] - s.A[:, fluid]))
    F = lat.force_history(0, 1, steps)
    Fo = np.array([f[0] for f in s.forces])
    ef = np.max(np.abs(F[:, :3] - Fo[:, :3])) / np.max(np.abs(Fo[:, :3]))
    em = np.max(np.abs(F[:, 3:] - Fo[:, 3:])) / max(np.max(np.abs(Fo[:, 3:])), 1e-12)
    _say(f"{label}: max|df| = {err:.3e}, force rel {ef:.2e}, torque rel {em:.2e}, "
         f"refills {sum(st['refill_nodes'] for st in s.stats)}")
    assert err <= 1e-6
    assert ef <= 1e-5
    assert em <= 3e-5


def test_resting_box_in_channel(E, oracle_mod):
    O = oracle_mod
    shape, nu, u_in, steps = (40, 20, 20), 0.01, (0.03, 0.0, 0.0), 25
    v, t = M.box_mesh((14.3, 6.6, 7.2), (21.7, 13.1, 12.9))
    rho, u = WL.uniform_flow(shape, u_in)
    lat = E.Lattice(shape, nu, channel=True, u_inlet=u_in, max_bodies=1, max_mesh_vertices=len(v),
                    max_mesh_triangles=len(t))
    lat.init_equilibrium(rho, u)
    c = (18.0, 9.85, 10.05)
    lat.set_mesh(v, t, v.min(0) - 0.5, v.max(0) + 0.5, center=c)
    lat.set_bodies([dict(kind="mesh")])
    lat.step(steps)
    s = O.Simulation(shape, nu, rho, u, bodies=[dict(kind="mesh", verts=v, tris=t, center=c)], channel=True,
                     u_in=u_in).step(steps)
    _compare(E, lat, s, "resting box", steps)


def test_oscillating_sphere_mesh(E, oracle_mod):
    """A level-3 sphere mesh moved rigidly along y (amplitude 1.5, period 40) in a channel."""
    O = oracle_mod
    shape, nu, u_in, steps = (40, 20, 20), 0.01, (0.03, 0.0, 0.0), 30
    body = WL.sphere((15.3, 10.2, 9.8), 4.0, amp=1.5, period=40.0, direction=(0.0, 1.0, 0.0))
    v0, t = M.icosphere_mesh((0.0, 0.0, 0.0), 4.0, 3)
    ob = O.body_from_spec(body)

    def level(k):
        c, U = O.kinematics(ob, float(k))
        return v0 + c, np.tile(U, (len(v0), 1)), c
    rho, u = WL.uniform_flow(shape, u_in)
    lat = E.Lattice(shape, nu, channel=True, u_inlet=u_in, max_bodies=1, max_mesh_vertices=len(v0),
                    max_mesh_triangles=len(t))
    lat.init_equilibrium(rho, u)
    X, V, c = level(0)
    lo, hi = np.array([10.8, 4.2, 5.3]), np.array([19.8, 15.9, 14.3])
    lat.set_mesh(X, t, lo, hi, vels=V, center=c)
    lat.set_bodies([dict(kind="mesh")])
    s = O.Simulation(shape, nu, rho, u, bodies=[dict(kind="mesh", verts=X, tris=t, vels=V, center=c)], channel=True,
                     u_in=u_in)
    for k in range(steps):
        X, V, c = level(k + 1)
        lat.mesh_next(X, V, center=c)
        lat.step(1)
        s.mesh_next(0, X, V, center=c)
        s.step(1)
    _compare(E, lat, s, "oscillating sphere mesh", steps)


def test_deforming_swimmer(E, oracle_mod):
    """The swimmer of Sec. IV.C (L = 32, undulation period 400, started at full amplitude) held in
    place in a channel, deforming every step."""
    O = oracle_mod
    shape, nu, u_in, steps = (56, 24, 24), 0.01, (0.02, 0.0, 0.0), 30
    L, T, t0, head = 32.0, 400.0, 400.0, (12.0, 11.7, 12.3)
    kw = dict(n_seg=80, n_theta=12)
    X, t, V = M.swimmer_mesh(head, L, T, t0, **kw)
    rho, u = WL.uniform_flow(shape, u_in)
    lat = E.Lattice(shape, nu, channel=True, u_inlet=u_in, max_bodies=1, max_mesh_vertices=len(X),
                    max_mesh_triangles=len(t))
    lat.init_equilibrium(rho, u)
    lo = np.array([head[0] - 1.0, head[1] - 6.0, head[2] - 4.0])
    hi = np.array([head[0] + L + 1.0, head[1] + 6.0, head[2] + 4.0])
    c = np.array([head[0] + 0.5 * L, head[1], head[2]])
    lat.set_mesh(X, t, lo, hi, vels=V, center=c)
    lat.set_bodies([dict(kind="mesh")])
    s = O.Simulation(shape, nu, rho, u, bodies=[dict(kind="mesh", verts=X, tris=t, vels=V, center=c)], channel=True,
                     u_in=u_in)
    _say(f"swimmer: {len(t)} triangles, {int((s.solid > 0).sum())} solid nodes at t = 0")
    for k in range(steps):
        X, _, V = M.swimmer_mesh(head, L, T, t0 + k + 1, **kw)
        lat.mesh_next(X, V, center=c)
        lat.step(1)
        s.mesh_next(0, X, V, center=c)
        s.step(1)
    _compare(E, lat, s, "deforming swimmer", steps)


def test_mesh_errors_are_reported(E):
    shape = (20, 20, 20)
    v, t = M.box_mesh((5.5, 5.5, 5.5), (12.5, 12.5, 12.5))
    rho, u = WL.uniform_flow(shape, (0.0, 0.0, 0.0))
    lat = E.Lattice(shape, 0.1, max_bodies=1, max_mesh_vertices=len(v), max_mesh_triangles=len(t))
    lat.init_equilibrium(rho, u)
    with pytest.raises(E.ElbmError, match="faces"):
        lat.set_mesh(v, t, (1.0, 5.0, 5.0), (13.0, 13.0, 13.0))
    with pytest.raises(E.ElbmError, match="elbm_set_mesh"):
        lat.set_bodies([dict(kind="mesh")])
    lat.set_mesh(v, t, (5.0, 5.0, 5.0), (13.0, 13.0, 13.0))
    lat.set_bodies([dict(kind="mesh")])
    lat.step(1)
    lat.force_history(0, 1, 1)
    # a vertex outside the declared box (it stays inside the lattice): reported, nothing faults
    far = v.copy()
    far[0] = (18.5, 18.5, 18.5)  # beyond the cell grid around the box (one cell of margin)
    lat.mesh_next(far)
    lat.step(1)
    with pytest.raises(E.ElbmError, match="declared box"):
        lat.force_history(0, 1, 2)
    # a vertex index out of range: replaced by 0 on the device and reported
    bad = t.copy()
    bad[3, 1] = len(v) + 7
    lat2 = E.Lattice(shape, 0.1, max_bodies=1, max_mesh_vertices=len(v), max_mesh_triangles=len(t))
    lat2.init_equilibrium(rho, u)
    lat2.set_mesh(v, bad, (5.0, 5.0, 5.0), (13.0, 13.0, 13.0))
    lat2.set_bodies([dict(kind="mesh")])
    lat2.step(1)
    with pytest.raises(E.ElbmError, match="vertex index"):
        lat2.force_history(0, 1, 1)
