"""Pins of the oracle's freely rotating sphere (two-way coupling with the torque: I dw/dt = M,
explicit Euler with unit step, I = (2/5) m R^2; Sec. IV.A's Newton equations with the rotational
one the swimmer case of Sec. IV.C also integrates).  Pinned by what mechanics fixes: the state
follows the Euler recurrence with the torques the steps report (the first update keeps the initial
spin, no torque yet); a sphere spinning about an axis through the centre of a box symmetric about
it feels no net force and stays put; and its spin decays at the rate the Stokes torque -8 pi rho nu
R^3 w gives, 15 nu rho/(rho_s R^2), within the box effect the prescribed-rotation pin measures
(-4.6 % of the torque at R = 4 in a 32^3 box)."""
import math

import numpy as np

import workloads as WL

SHAPE = (32, 32, 32)
CENTRE = (15.5, 15.5, 15.5)  # midway between lattice planes: the node set is symmetric about it


def _spin_run(O, steps, nu=0.1, R=4.0, ratio=20.0, w0=(0.0, 0.0, 0.002)):
    s = O.Simulation(SHAPE, nu, bodies=[WL.free_sphere(CENTRE, R, ratio, omega=w0)])
    ws, xs = [], []
    for _ in range(steps):
        ws.append(s.body_spin(0))
        xs.append(s.body_state(0)[0])
        s.step(1)
    ws.append(s.body_spin(0))
    xs.append(s.body_state(0)[0])
    return s, np.array(ws), np.array(xs)


def test_spin_follows_the_euler_recurrence(oracle_mod):
    O = oracle_mod
    R, ratio = 4.0, 20.0
    s, ws, _ = _spin_run(O, 12, R=R, ratio=ratio)
    m = ratio * (4.0 / 3.0) * math.pi * R ** 3
    I = 0.4 * m * R * R
    assert np.array_equal(ws[1], ws[0])  # no torque before the first step
    for k in range(1, 12):
        M = s.forces[k - 1][0, 3:]
        assert np.max(np.abs(ws[k + 1] - (ws[k] + M / I))) == 0.0


def test_symmetric_spin_exerts_no_force(oracle_mod):
    s, ws, xs = _spin_run(oracle_mod, 30)
    assert np.max(np.abs(xs - xs[0])) == 0.0
    F = np.array([f[0, :3] for f in s.forces])
    M = np.array([f[0, 3:] for f in s.forces])
    assert np.max(np.abs(F)) < 1e-12 * max(1.0, np.max(np.abs(M)))
    assert np.max(np.abs(M[:, :2])) < 1e-12  # torque only about the spin axis
    assert np.all(M[1:, 2] < 0)  # it opposes the spin


def test_spin_decays_at_the_stokes_rate(oracle_mod):
    nu, R, ratio = 0.1, 4.0, 20.0
    _, ws, _ = _spin_run(oracle_mod, 120, nu=nu, R=R, ratio=ratio)
    rate = -(math.log(ws[120, 2]) - math.log(ws[60, 2])) / 60.0
    theory = 15.0 * nu / (ratio * R * R)
    print(f"spin-down rate {rate:.5f}, Stokes {theory:.5f} ({rate / theory - 1:+.3f})")
    assert abs(rate / theory - 1.0) < 0.08
