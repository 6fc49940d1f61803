"""Rotating bodies and the torque of the momentum exchange (Sec. IV.A, wall velocity U + Omega x r):
a sphere spinning slowly about z in a periodic box of fluid initially at rest approaches the Stokes
torque -8 pi rho nu R^3 Omega (within 8 %: staircase surface at R = 4 and periodic images), with no
net force and no torque about x or y (symmetry of the node set about the centre); reversing Omega
reverses the torque exactly (mirror symmetry)."""
import numpy as np

import workloads as WL


def test_slowly_rotating_sphere_has_stokes_torque(oracle_mod):
    O = oracle_mod
    nu, R, om = 0.1, 4.0, 2e-4
    s = O.Simulation((32, 32, 32), nu, bodies=[WL.sphere((15.5, 15.5, 15.5), R, omega=(0.0, 0.0, om))])
    s.step(400)
    f = s.forces[-1][0]
    stokes = -8.0 * np.pi * nu * R ** 3 * om
    assert np.max(np.abs(f[:5])) < 1e-12
    assert abs(f[5] / stokes - 1.0) < 0.08
    assert f[5] < 0.0


def test_torque_is_odd_in_the_rotation_rate(oracle_mod):
    O = oracle_mod
    out = []
    for om in (3e-4, -3e-4):
        s = O.Simulation((24, 24, 24), 0.05, bodies=[WL.sphere((11.5, 11.5, 11.5), 3.5, omega=(0.0, 0.0, om))])
        s.step(30)
        out.append(np.array([f[0, 5] for f in s.forces]))
    assert np.max(np.abs(out[0] + out[1])) <= 1e-12 * np.max(np.abs(out[0]))
