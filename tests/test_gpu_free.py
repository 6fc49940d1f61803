"""Free-moving spheres (two-way coupling, Sec. IV.A) on the GPU: the library's trajectory, forces and
populations against the FP64 oracle (same Euler recurrence, integrated independently in the
oracle's driver).  The paper's Galilean-invariance check of the coupling (the settling sphere) is in
test_gpu_settling.py."""
import numpy as np
import pytest

import workloads as WL

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


@pytest.mark.parametrize("channel", [False, True])
def test_free_sphere_parity(E, oracle_mod, channel):
    O = oracle_mod
    shape = (40, 24, 24)
    nu, steps = 0.03, 120
    body = WL.free_sphere((15.3, 11.6, 11.2), 4.0, 1.5, gravity=(6e-5, 1.5e-5, -5e-6), vel=(0.002, 0.0, 0.0))
    _say(f"case: free sphere parity channel={channel}")
    rho, u = WL.uniform_flow(shape, (0.0, 0.0, 0.0))
    lat = E.Lattice(shape, nu, channel=channel, u_inlet=(0.0, 0.0, 0.0), max_bodies=1)
    lat.init_equilibrium(rho, u)
    lat.set_bodies([body])
    s = O.Simulation(shape, nu, rho, u, bodies=[body], channel=channel, u_in=(0.0, 0.0, 0.0))
    gx, gu, ox, ou = [], [], [], []
    for t in range(steps):
        lat.step(1)
        s.step(1)
        x, v = lat.body_state(0)
        gx.append(x)
        gu.append(v)
        x, v = s.body_state(0)
        ox.append(x)
        ou.append(v)
    gx, gu, ox, ou = map(np.array, (gx, gu, ox, ou))
    F = lat.force_history(0, 1, steps)[:, :3]
    Fo = np.array([f[0, :3] for f in s.forces])
    ex = np.max(np.abs(gx - ox))
    eu = np.max(np.abs(gu - ou)) / np.max(np.abs(ou))
    eF = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    assert np.array_equal(lat.flags().cpu().numpy() & 1, (s.solid > 0).astype(np.uint8))
    fluid = s.solid == 0  # the populations of solid nodes are not part of the state
    ef = np.max(np.abs(lat.populations().cpu().numpy()[:, fluid] - s.A[:, fluid]))
    _say(f"free sphere channel={channel}: travel {ox[-1] - ox[0]}, max|dx| {ex:.2e}, velocity rel {eu:.2e}, "
         f"force rel {eF:.2e}, max|df| {ef:.2e}")
    # measured: position 4.7e-8, velocity 8.2e-7, force 2.9e-6, populations 1.8e-8
    assert ex <= 1e-6
    assert eu <= 1e-5
    assert eF <= 3e-5
    assert ef <= 1e-6


def test_free_rotating_sphere_parity(E, oracle_mod):
    """A sphere released with a spin and settling off-axis in a channel stream (lift, drag and
    torque all nonzero): position, velocity, angular velocity, forces, torques and populations."""
    O = oracle_mod
    shape, nu, steps, u_in = (40, 24, 24), 0.03, 100, (0.01, 0.0, 0.0)
    body = WL.free_sphere((16.3, 11.6, 11.2), 4.0, 2.0, gravity=(0.0, 3e-5, 0.0), vel=(0.0, 0.0, 0.0),
                          omega=(0.001, -0.002, 0.004))
    _say("case: free rotating sphere parity")
    rho, u = WL.uniform_flow(shape, u_in)
    lat = E.Lattice(shape, nu, channel=True, u_inlet=u_in, max_bodies=1)
    lat.init_equilibrium(rho, u)
    lat.set_bodies([body])
    s = O.Simulation(shape, nu, rho, u, bodies=[body], channel=True, u_in=u_in)
    g, o = [], []
    for t in range(steps):
        lat.step(1)
        s.step(1)
        g.append(np.concatenate([*lat.body_state(0), lat.body_spin(0)]))
        o.append(np.concatenate([*s.body_state(0), s.body_spin(0)]))
    g, o = np.array(g), np.array(o)
    ex = np.max(np.abs(g[:, :3] - o[:, :3]))
    eu = np.max(np.abs(g[:, 3:6] - o[:, 3:6])) / np.max(np.abs(o[:, 3:6]))
    ew = np.max(np.abs(g[:, 6:] - o[:, 6:])) / np.max(np.abs(o[:, 6:]))
    F = lat.force_history(0, 1, steps)
    Fo = np.array([f[0] for f in s.forces])
    eF = np.max(np.abs(F[:, :3] - Fo[:, :3])) / np.max(np.abs(Fo[:, :3]))
    eM = np.max(np.abs(F[:, 3:] - Fo[:, 3:])) / np.max(np.abs(Fo[:, 3:]))
    fluid = s.solid == 0
    ef = np.max(np.abs(lat.populations().cpu().numpy()[:, fluid] - s.A[:, fluid]))
    _say(f"free rotating sphere: spin {o[0, 6:]} -> {o[-1, 6:]}, max|dx| {ex:.2e}, velocity rel {eu:.2e}, "
         f"spin rel {ew:.2e}, force rel {eF:.2e}, torque rel {eM:.2e}, max|df| {ef:.2e}")
    assert np.max(np.abs(o[-1, 6:] - o[0, 6:])) > 1e-5  # the torque did turn it
    # measured: position 2.7e-7, velocity 1.9e-6, spin 1.7e-7, force 1.5e-6, torque 4.3e-7,
    # populations 2.8e-8
    assert ex <= 1e-6
    assert eu <= 2e-5
    assert ew <= 2e-6
    assert eF <= 2e-5
    assert eM <= 5e-6
    assert ef <= 1e-6


def test_free_sphere_leaving_the_domain_is_an_error(E):
    """A free sphere must stay 3 nodes inside every face: the step that would take it closer fails."""
    lat = E.Lattice((32, 24, 24), 0.05, max_bodies=1)
    rho, u = WL.uniform_flow((32, 24, 24), (0.0, 0.0, 0.0))
    lat.init_equilibrium(rho, u)
    lat.set_bodies([WL.free_sphere((8.0, 12.0, 12.0), 4.0, 50.0, vel=(-0.3, 0.0, 0.0))])
    lat.step(2)  # centre 8 -> 7.7 -> 7.4: still 3 nodes inside
    with pytest.raises(E.ElbmError, match="free body"):
        lat.step(10)
