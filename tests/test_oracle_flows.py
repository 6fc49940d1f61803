"""Pins of the oracle's full time step (Secs. II and III) against exact solutions,
closed forms and brute force: streaming as an index permutation, viscous decay
at the Chapman-Enskog viscosity, Couette and Poiseuille flow between walls, the
momentum balance that fixes the momentum-exchange force, the target values of
the moving-wall rule on a flat wall, refill moments, link fractions q and the
finite-difference stencil."""
import math

import numpy as np
import pytest

import workloads as WL


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


@pytest.fixture(scope="module")
def lat(O):
    c, w = O.lattice()
    return c, w


def test_streaming_is_exact_permutation(O, lat):
    """Pull streaming (eq. kineticEq, left-hand side): f_i(x, t+1) = A_i(x - c_i), periodic."""
    c, _ = lat
    nx, ny, nz = 7, 5, 4
    rng = np.random.default_rng(0)
    A0 = rng.integers(0, 1000, size=(27, nz, ny, nx)).astype(np.float64)
    s = O.Simulation((nx, ny, nz), 0.1, A0=A0, stream_only=True)
    s.step(1)
    for i in range(27):
        want = np.roll(A0[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(s.A[i], want)
    s.step(nx * ny * nz)  # lcm-free check: after nx*ny*nz steps every shift wraps around
    for i in range(27):
        k = nx * ny * nz + 1
        want = np.roll(A0[i], shift=(c[i, 2] * k, c[i, 1] * k, c[i, 0] * k), axis=(0, 1, 2))
        assert np.array_equal(s.A[i], want)


def _fit_rate(ts, amps):
    p = np.polyfit(ts, np.log(amps), 1)
    return -p[0]


def test_taylor_green_2d_decays_at_the_chapman_enskog_viscosity(O):
    """z-invariant Taylor-Green vortex: exact Navier-Stokes solution with amplitude
    ~ exp(-2 nu k^2 t); nu from beta by the relation of Sec. II."""
    n = 32
    nu = 0.02
    rho, u = WL.taylor_green_2d(n, n, 1, 1e-3)
    s = O.Simulation((n, n, 1), nu, rho, u)
    k = 2 * math.pi / n
    prof = u[0] / 1e-3
    ts, amps = [], []
    for t in range(0, 400):
        s.step(1)
        if s.t >= 100 and s.t % 20 == 0:
            _, U = s.velocity()
            ts.append(s.t)
            amps.append(np.sum(U[0] * prof) / np.sum(prof * prof))
    rate = _fit_rate(ts, amps)
    assert abs(rate / (2 * nu * k * k) - 1) < 0.01


def test_shear_wave_decays_at_the_chapman_enskog_viscosity(O):
    n = 24
    for nu in (0.01, 0.1):
        rho, u = WL.shear_wave(2, n, 1, 1e-4)
        s = O.Simulation((2, n, 1), nu, rho, u)
        k = 2 * math.pi / n
        prof = u[0] / 1e-4
        ts, amps = [], []
        for t in range(300):
            s.step(1)
            if s.t >= 60 and s.t % 10 == 0:
                _, U = s.velocity()
                ts.append(s.t)
                amps.append(np.sum(U[0] * prof) / np.sum(prof * prof))
        rate = _fit_rate(ts, amps)
        assert abs(rate / (nu * k * k) - 1) < 0.01


def test_bulk_flow_stays_divergence_free_and_isotropic(O):
    """3-D Taylor-Green on 16^3 for 50 steps: mass conserved to round-off, mean momentum zero."""
    rho, u = WL.taylor_green_3d(16, 0.05)
    s = O.Simulation((16, 16, 16), 1e-3, rho, u)
    m0 = s.moments()[0].sum()
    s.step(50)
    r, j = s.moments()
    assert abs(r.sum() - m0) < 1e-10
    assert np.max(np.abs(j.sum(axis=(1, 2, 3)))) < 1e-12


def _channel_walls(ny, y_lo, y_hi, u_top=(0.0, 0.0, 0.0)):
    """Two plane walls: solid below y_lo and above y_hi (normals point into the fluid)."""
    return [WL.plane((0, y_lo, 0), (0, 1, 0)), WL.plane((0, y_hi, 0), (0, -1, 0), vel=u_top)]


@pytest.mark.parametrize("y_lo,y_hi", [(0.5, 18.5), (0.3, 18.8)])
def test_couette_profile_is_linear(O, y_lo, y_hi):
    """Moving-wall Grad rule (Sec. III) between a resting and a sliding plane: the steady
    solution is the linear profile through the wall positions, for any link fraction q."""
    ny = 20
    U = 0.01
    bodies = _channel_walls(ny, y_lo, y_hi, u_top=(U, 0, 0))
    _, y, _ = WL.node_coords((2, ny, 1))
    u = np.zeros((3, 1, ny, 2))
    u[0] = np.clip(U * (y - y_lo) / (y_hi - y_lo), 0, U)
    s = O.Simulation((2, ny, 1), 1.0 / 6.0, np.ones((1, ny, 2)), u, bodies=bodies)
    s.step(3000)
    _, Uf = s.velocity()
    fluid = s.solid[0, :, 0] == 0
    ys = np.arange(ny)[fluid]
    exact = U * (ys - y_lo) / (y_hi - y_lo)
    got = Uf[0, 0, fluid, 0]
    assert np.max(np.abs(got - exact)) < 1e-6 * U
    assert np.max(np.abs(Uf[1:, 0, fluid, :])) < 1e-9


def test_poiseuille_profile_and_wall_force_balance(O):
    """Body-force-driven channel: parabolic steady profile, and at steady state the
    momentum-exchange force on the walls equals the total body force on the fluid."""
    ny = 20
    g = 1e-6
    nu = 1.0 / 6.0
    bodies = _channel_walls(ny, 0.5, 18.5)
    F = np.zeros((3, 1, ny, 2))
    F[0] = g
    s = O.Simulation((2, ny, 1), nu, bodies=bodies, F=F)
    s.step(6000)
    _, Uf = s.velocity()
    fluid = s.solid[0, :, 0] == 0
    ys = np.arange(ny)[fluid]
    exact = g / (2 * nu) * (ys - 0.5) * (18.5 - ys)
    got = Uf[0, 0, fluid, 0]
    assert np.max(np.abs(got - exact)) / exact.max() < 0.01
    total_body_force = g * 2 * fluid.sum()
    fwall = s.forces[-1][:, 0].sum()
    assert abs(fwall / total_body_force - 1) < 1e-6
    # each wall also carries the static pressure c_s^2 rho per unit area (2 nodes here),
    # equal and opposite on the two walls
    fy = s.forces[-1][:, 1]
    assert abs(abs(fy[0]) - 2.0 / 3.0) < 1e-3 and abs(fy.sum()) < 1e-12
    assert np.max(np.abs(s.forces[-1][:, 2])) < 1e-14


def test_rest_state_with_body_is_exact_fixed_point(O, lat):
    """Fluid at rest around a resting sphere: f = W everywhere is preserved exactly and the
    momentum-exchange force vanishes (equal link counts in opposite directions)."""
    c, w = lat
    s = O.Simulation((16, 16, 16), 0.05, bodies=[WL.sphere((7.3, 8.1, 7.7), 4.2)])
    s.step(3)
    fluid = s.solid == 0
    for i in range(27):
        assert np.max(np.abs(s.A[i][fluid] - w[i])) < 1e-15
    assert np.max(np.abs(s.forces[-1][0, :3])) < 1e-13


def test_flat_wall_target_values(O, lat):
    """Sec. III on a flat wall moving along its normal: after one step from rest the node next to
    the wall holds the Grad populations at rho_tgt = 1 + rho0 u_w.n (bounce-back density plus the
    displacement term), u_tgt = (q u_f + u_w)/(1+q) with u_f = 0, and Pi^eq (zero gradient)."""
    c, w = lat
    V = 1e-3
    ny = 12
    body = WL.plane((0, 0.5, 0), (0, 1, 0), vel=(0.0, V, 0.0))
    s = O.Simulation((2, ny, 1), 0.05, bodies=[body])
    s.step(1)
    q = 1.0 - (0.5 + V)          # wall at y = 0.5 + V at t = 1, node y = 1
    uw = np.array([0.0, V, 0.0])
    ut = uw / (1 + q)            # u_f = 0 (fluid at rest)
    rt = 1.0 + V                 # rho_stat = 1 at rest, rho_dyn = rho0 u_w.n
    Pi = rt / 3.0 * np.eye(3) + rt * np.outer(ut, ut)
    fs = O.grad_dist(rt, ut, Pi)
    D = c[:, 1] == 1
    f_pre = np.where(D, fs, w)
    r, j = s.moments()
    assert abs(r[0, 1, 0] - f_pre.sum()) < 1e-15
    assert np.allclose(j[:, 0, 1, 0], c.T @ f_pre, atol=1e-16)
    # closed form of the displacement term on a flat wall: sum_Dbar 6 W_i c_i.u_w = u_w.n
    assert abs(np.sum(6 * w[D] * (c[D] @ uw)) - V) < 1e-18


def test_link_fraction_matches_brute_force_ray_march(O, lat):
    c, _ = lat
    body = O.make_body("sphere", center=(6.37, 5.81, 6.12), radius=3.3)
    cen = np.array([6.37, 5.81, 6.12])
    inside = lambda p: np.sum((p - cen) ** 2) < 3.3 ** 2
    count = 0
    for x in range(13):
        for y in range(12):
            for z in range(13):
                xb = np.array([x, y, z], dtype=float)
                if inside(xb):
                    continue
                for i in range(27):
                    if i == 13 or not inside(xb - c[i]):
                        continue
                    lo, hi = 0.0, 1.0  # bisection on the segment xb - s c_i
                    for _ in range(200):
                        m = 0.5 * (lo + hi)
                        if inside(xb - m * c[i]):
                            hi = m
                        else:
                            lo = m
                    assert abs(O.q_link(body, 0.0, xb, i) - 0.5 * (lo + hi)) < 1e-12
                    count += 1
    assert count > 100
    plane = O.make_body("plane", center=(0, 2.25, 0), normal=(0, 1, 0))
    for i in range(27):
        if c[i, 1] == 1:
            assert abs(O.q_link(plane, 0.0, (3.0, 3.0, 1.0), i) - 0.75) < 1e-15


def test_solid_mask_matches_brute_force(O):
    b = WL.sphere((9.37, 8.5, 7.25), 5.5, amp=2.0, period=37.0, direction=(0.0, 1.0, 0.0))
    s = O.Simulation((20, 18, 16), 0.1, bodies=[b])
    x, y, z = WL.node_coords((20, 18, 16))
    for t in (0, 3, 11, 20):
        cy = 8.5 + (2.0 * math.sin(((2.0 * math.pi) * t) / 37.0)) * 1.0
        d2 = (x - 9.37) * (x - 9.37) + (y - cy) * (y - cy) + (z - 7.25) * (z - 7.25)
        assert np.array_equal(s.mask(t) > 0, d2 < 5.5 * 5.5)


def test_refill_sets_density_average_and_wall_velocity(O, lat):
    """Sec. III refill: an uncovered node gets Grad's distribution with the wall velocity, a local
    density average and the pressure tensor, so its populations carry exactly those moments."""
    c, _ = lat
    cc = c.astype(float)
    rng = np.random.default_rng(3)
    n = 18
    b = WL.sphere((7.0, 9.0, 9.0), 4.0, vel=(0.3, 0.0, 0.0), omega=(0.0, 0.0, 0.02))
    rho, u = WL.taylor_green_3d(n, 0.02)
    rho = rho + 0.01 * rng.standard_normal(rho.shape)
    s = O.Simulation((n, n, n), 0.05, rho, u, bodies=[b])
    bb = O.body_from_spec(b)
    checked = 0
    for step in range(4):
        s1 = s.mask(s.t + 1)
        Aw, cnt, U, R = s.refill_state(s1)
        r_prev, _ = s.moments()
        cen, Ub = O.kinematics(bb, s.t + 1)
        refill = np.argwhere((s.solid > 0) & (s1 == 0))
        assert cnt == len(refill)
        for z, y, x in refill:
            vals = []
            for i in range(27):
                if i == 13:
                    continue
                zz, yy, xx = (z + c[i, 2]) % n, (y + c[i, 1]) % n, (x + c[i, 0]) % n
                if s.solid[zz, yy, xx] == 0 and s1[zz, yy, xx] == 0:
                    vals.append(r_prev[zz, yy, xx])
            ravg = np.mean(vals) if vals else 1.0
            uw = Ub + np.cross([0.0, 0.0, 0.02], np.array([x, y, z], float) - cen)
            f = Aw[:, z, y, x]
            G = s.grad_u(U, s1, x, y, z)
            Pi = O.pressure(ravg, uw, G, s.grid.beta)
            assert abs(f.sum() - ravg) < 1e-14
            assert np.allclose(cc.T @ f, ravg * uw, atol=1e-15)
            assert np.allclose(np.einsum("i,ia,ib->ab", f, cc, cc), Pi, atol=1e-14)
            checked += 1
        s.step(1)
    assert checked > 10


def test_refilled_populations_stream_to_the_neighbours(O, lat):
    """The refill comes before streaming: in a stream-only step the neighbours of an uncovered node
    receive its refilled populations unchanged."""
    c, _ = lat
    n = 16
    b = WL.sphere((6.5, 8.2, 8.1), 3.5, vel=(0.4, 0.0, 0.0))
    rho, u = WL.uniform_flow((n, n, n), (0.02, 0.0, 0.0))
    s = O.Simulation((n, n, n), 0.05, rho, u, bodies=[b], stream_only=True)
    s.step(2)
    s1 = s.mask(s.t + 1)
    Aw, cnt, _, _ = s.refill_state(s1)
    assert cnt > 0
    s.step(1)
    hits = 0
    s0 = s.mask(s.t - 1)   # refill nodes of the step just taken: solid at its start, fluid at its end
    for z, y, x in np.argwhere((s0 > 0) & (s1 == 0)):
        for i in range(27):
            zz, yy, xx = (z + c[i, 2]) % n, (y + c[i, 1]) % n, (x + c[i, 0]) % n
            if s1[zz, yy, xx] == 0:
                assert s.A[i, zz, yy, xx] == Aw[i, z, y, x]
                hits += 1
    assert hits > 20


def test_finite_difference_stencil(O):
    """Velocity gradient of Sec. III: central where possible, else 2nd-order one-sided,
    else 1st-order; exact on quadratic (resp. linear) fields."""
    n = 12
    x, y, z = WL.node_coords((n, n, n))
    a = np.array([0.3, -0.2, 0.1])
    U = np.stack([1e-3 * (x - 5) ** 2 + 2e-3 * y, 1e-3 * (y - 4) * (z - 3), -1e-3 * (z - 6) ** 2 + 1e-3 * x])
    dU = lambda px, py, pz: np.array([[2e-3 * (px - 5), 2e-3, 0.0], [0.0, 1e-3 * (pz - 3), 1e-3 * (py - 4)],
                                      [1e-3, 0.0, -2e-3 * (pz - 6)]])
    s = O.Simulation((n, n, n), 0.1)
    solid = np.zeros((n, n, n), np.uint8)
    p = (6, 6, 6)
    assert np.allclose(s.grad_u(U, solid, *p), dU(*p), atol=1e-15)
    solid[6, 6, 5] = 1     # x-1 unusable -> forward 2nd order in x
    solid[6, 7, 6] = 1     # y+1 unusable -> backward 2nd order in y
    solid[7, 6, 6] = 1     # z+1 unusable ...
    solid[4, 6, 6] = 1     # ... and z-2 unusable -> backward 1st order in z (exact only for linear)
    G = s.grad_u(U, solid, *p)
    assert np.allclose(G[:, 0], dU(*p)[:, 0], atol=1e-15)
    assert np.allclose(G[:, 1], dU(*p)[:, 1], atol=1e-15)
    want_z = U[:, 6, 6, 6] - U[:, 5, 6, 6]
    assert np.allclose(G[:, 2], want_z, atol=1e-15)
    solid[5, 6, 6] = 1     # no z neighbour at all -> 0
    assert np.allclose(s.grad_u(U, solid, *p)[:, 2], 0.0)


def test_body_force_drives_uniform_momentum(O):
    n = 6
    F = np.zeros((3, n, n, n))
    F[0] = 2e-5
    F[2] = -1e-5
    s = O.Simulation((n, n, n), 0.05, F=F)
    r0, j0 = s.moments()
    s.step(3)
    r, j = s.moments()
    assert abs(r.sum() - r0.sum()) < 1e-12
    assert np.allclose(j.sum(axis=(1, 2, 3)) - j0.sum(axis=(1, 2, 3)), 3 * F.sum(axis=(1, 2, 3)), atol=1e-15)


def test_channel_keeps_uniform_inflow_and_sphere_drag_points_downstream(O):
    shape = (24, 12, 12)
    rho, u = WL.uniform_flow(shape, (0.03, 0.0, 0.0))
    s = O.Simulation(shape, 0.02, rho, u, channel=True, u_in=(0.03, 0.0, 0.0))
    s.step(40)
    _, U = s.velocity()
    assert np.max(np.abs(U[0] - 0.03)) < 2e-4
    assert np.max(np.abs(U[1:])) < 2e-4
    s2 = O.Simulation(shape, 0.02, rho, u, channel=True, u_in=(0.03, 0.0, 0.0),
                      bodies=[WL.sphere((8.2, 6.1, 5.9), 3.0)])
    s2.step(40)
    fx = np.array([f[0, 0] for f in s2.forces[-10:]])
    assert np.all(fx > 0)


def test_channel_outlet_copies_the_upstream_streamed_value(O, lat):
    """Outlet column x = nx-1: a population entering from outside (c_x = -1) takes the value
    streamed into the upstream neighbour, A_i(nx-1, y - c_y, z - c_z); elsewhere pull streaming."""
    c, _ = lat
    nx, ny, nz = 6, 5, 4
    rng = np.random.default_rng(1)
    A0 = rng.integers(1, 1000, size=(27, nz, ny, nx)).astype(np.float64)
    s = O.Simulation((nx, ny, nz), 0.1, A0=A0, stream_only=True, channel=True)
    s.step(1)
    for i in range(27):
        want = np.roll(A0[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        if c[i, 0] == -1:
            want[:, :, nx - 1] = np.roll(A0[i][:, :, nx - 1], shift=(c[i, 2], c[i, 1]), axis=(0, 1))
        xs = slice(1, nx) if c[i, 0] == 1 else slice(0, nx)   # x = 0 with c_x = +1 is rebuilt (inlet)
        assert np.array_equal(s.A[i][:, :, xs], want[:, :, xs])


def test_channel_inlet_is_a_moving_wall_half_a_cell_upstream(O):
    """Inlet face as the moving-wall rule at x = -1/2 (q = 1/2) with velocity u_in: sliding it
    along y against a resting plane at x = x_w gives the linear Couette profile."""
    nx = 20
    V = 0.01
    xw = nx - 1.5
    s = O.Simulation((nx, 2, 1), 1.0 / 6.0, channel=True, u_in=(0.0, V, 0.0),
                     bodies=[WL.plane((xw, 0, 0), (-1, 0, 0))])
    s.step(3000)
    _, Uf = s.velocity()
    xs = np.arange(nx - 1)
    exact = V * (xw - xs) / (xw + 0.5)
    assert np.max(np.abs(Uf[1, 0, 0, : nx - 1] - exact)) < 1e-6 * V
    assert np.max(np.abs(Uf[0, 0, 0, : nx - 1])) < 1e-9
    assert s.forces[-1].shape == (1, 6)   # the inlet is not a body: only the plane is reported
