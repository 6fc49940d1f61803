"""Pins of the FP64 CPU adjoint (oracle/elbm_oracle_adjoint.cpp) against the forward oracle
(oracle/elbm_oracle.c), which it does not call.

The adjoint of one step t -> t+1 gives dL/dA^t, dL/dF and dL/d(amp) of
    L = <lam, A^{t+1}> + w . F_body(t+1)
with the solid masks of both time levels frozen.  What pins it:
  * its own forward values (it restates the step) equal the forward oracle's A^{t+1} and force;
  * each node-local piece -- the KBC collision (Sec. II, eqs. kineticEq, kbc_relax, the analytic
    stabiliser), Grad's distribution with the pressure tensor (eqs. grad, pressure, pressure2), the
    link fraction of Sec. III -- against central differences of the forward oracle's routines;
  * the whole step against central differences of the forward oracle's step: inner products with
    random directions, directions confined to the places where the step is not a plain pull (the
    inlet face, the outlet copy, the walls' bounce-back entries, the nodes a moving body uncovers,
    the nodes it covers), single entries of dL/dA^t, and dL/dF at 16 seeded nodes x 3 components;
  * a closed form: with streaming alone and no bodies the step is a permutation, whose adjoint is the
    inverse permutation (bit-exact).
Differences are central, with Richardson extrapolation over steps h and 2h where the stabiliser's
curvature matters (states carry relative noise 1e-3, so <dh|dh> is small and a step has to stay far
below the noise: h = 1e-8 on populations of order 1e-2).  Bounds are a few times the measured
agreement (stated per test), far below any dropped term, wrong sign or transposed index."""
import numpy as np
import pytest
from scipy.ndimage import binary_dilation

import workloads as WL

SMALL = dict(shape=(40, 20, 20), nu=0.02, channel=True, u_in=(0.03, 0.0, 0.0),
             body=WL.sphere((16.3, 10.2, 9.9), 4.0, amp=2.0, period=60.0, direction=(0, 1, 0)))


def _say(msg):
    print(msg, flush=True)


def _states(O, n, seed, noise=1e-2):
    """n post-collision-like states: an entropic equilibrium at random rho, u, times (1 + noise)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rho = 1.0 + 0.05 * rng.standard_normal()
        u = rng.uniform(-0.08, 0.08, 3)
        out.append(O.feq(rho, u) * (1.0 + noise * rng.standard_normal(27)))
    return out


def _rich(fun, h):
    """Central difference with Richardson extrapolation: (4 D(h) - D(2h)) / 3."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(2 * h) - fun(-2 * h)) / (4 * h)
    return (4 * d1 - d2) / 3


# ----------------------------------------------------------------------------- node-local pieces
@pytest.mark.parametrize("variant", ["kbc", "kbc_force", "lbgk"])
def test_collision_jacobian_matches_oracle_differences(oracle_mod, variant):
    """Full 27 x 27 (+3 for the body force) Jacobian of the collision, row by row from the adjoint,
    against central differences of the forward oracle's or_collide_ex.  Measured max error 2e-9 of
    the largest entry (Richardson, h = 1e-6 on populations ~ 0.03); bound 1e-7."""
    O = oracle_mod
    beta = O.beta_from_nu(0.01)
    lbgk = variant == "lbgk"
    rng = np.random.default_rng(7)
    worst = 0.0
    for f in _states(O, 6, 11):
        F = rng.uniform(-1e-4, 1e-4, 3) if variant == "kbc_force" else None
        J = np.zeros((27, 27))
        JF = np.zeros((27, 3))
        for r in range(27):
            e = np.zeros(27)
            e[r] = 1.0
            gf, gF = O.collide_adjoint(f, beta, e, F=F, lbgk=lbgk)
            J[r] = gf
            JF[r] = gF
        fd = np.zeros((27, 27))
        gam = 2.0 if lbgk else 0.0
        for c in range(27):
            def fun(h, c=c):
                g = f.copy()
                g[c] += h
                return O.collide(g, beta, F=F, gamma_fixed=gam)[0]
            fd[:, c] = _rich(fun, 1e-6)
        err = np.max(np.abs(J - fd)) / np.max(np.abs(fd))
        worst = max(worst, err)
        if F is not None:
            fdF = np.zeros((27, 3))
            for c in range(3):
                def funF(h, c=c):
                    G = F.copy()
                    G[c] += h
                    return O.collide(f, beta, F=G)[0]
                fdF[:, c] = _rich(funF, 1e-6)
            errF = np.max(np.abs(JF - fdF)) / np.max(np.abs(fdF))
            worst = max(worst, errF)
    _say(f"collision Jacobian ({variant}): max error {worst:.2e} of the largest entry")
    assert worst <= 1e-7


def test_collision_restatement_equals_oracle(oracle_mod):
    """The adjoint library's own collision gives the forward oracle's post-collision state."""
    O = oracle_mod
    beta = O.beta_from_nu(0.004)
    rng = np.random.default_rng(3)
    worst = 0.0
    for f in _states(O, 50, 5):
        F = rng.uniform(-1e-4, 1e-4, 3)
        for FF in (None, F):
            a = O.collide(f, beta, F=FF)[0]
            b = O.collide_restated(f, beta, F=FF)
            worst = max(worst, np.max(np.abs(a - b)))
    _say(f"restated collision vs oracle: max |df| {worst:.1e}")
    assert worst <= 1e-16


def test_collision_adjoint_at_the_guard_is_the_lbgk_one(oracle_mod):
    """Where <dh|dh> <= 1e-30 the stabiliser is gamma = 2 (the reading of the oracle), a constant: the
    adjoint there is that of the LBGK collision."""
    O = oracle_mod
    beta = O.beta_from_nu(0.01)
    c, w = O.lattice()
    fe = O.feq(1.02, [0.03, -0.01, 0.02])
    f = fe + 1e-3 * np.where(c[:, 2] == 0, c[:, 0] * c[:, 1], 0)   # a pure shear mode: h = h_eq
    _, gam, guard = O.collide(f, beta)
    assert guard
    rng = np.random.default_rng(1)
    g = rng.standard_normal(27)
    a = O.collide_adjoint(f, beta, g)[0]
    b = O.collide_adjoint(f, beta, g, lbgk=True)[0]
    assert np.array_equal(a, b)


def test_grad_pressure_adjoint_matches_oracle_differences(oracle_mod):
    """Grad's distribution at the pressure tensor of eqs. pressure/pressure2: values equal to the
    forward oracle's, derivatives in rho, u and the velocity gradient against its central differences
    (the map is polynomial of degree 3: measured 3e-11, bound 1e-9 of the largest entry)."""
    O = oracle_mod
    rng = np.random.default_rng(2)
    beta = O.beta_from_nu(0.0048)
    worst = 0.0
    for _ in range(10):
        rho = 1.0 + 0.02 * rng.standard_normal()
        u = rng.uniform(-0.05, 0.05, 3)
        G = rng.uniform(-0.01, 0.01, (3, 3))
        ref = O.grad_dist(rho, u, O.pressure(rho, u, G, beta))
        gout = rng.standard_normal(27)
        out, gr, gu, gG = O.grad_pressure_adjoint(rho, u, G, beta, gout)
        assert np.max(np.abs(out - ref)) <= 1e-16

        def f_of(r, uu, GG):
            return gout @ O.grad_dist(r, uu, O.pressure(r, uu, GG, beta))
        h = 1e-5
        fd_r = (f_of(rho + h, u, G) - f_of(rho - h, u, G)) / (2 * h)
        worst = max(worst, abs(fd_r - gr) / max(1.0, abs(fd_r)))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (f_of(rho, u + e, G) - f_of(rho, u - e, G)) / (2 * h)
            worst = max(worst, abs(fd - gu[a]) / max(1.0, abs(fd)))
        for a in range(3):
            for b in range(3):
                E = np.zeros((3, 3))
                E[a, b] = h
                fd = (f_of(rho, u, G + E) - f_of(rho, u, G - E)) / (2 * h)
                worst = max(worst, abs(fd - gG[a, b]) / max(1.0, abs(fd)))
    _say(f"Grad/pressure adjoint: max error {worst:.1e}")
    assert worst <= 1e-9


def test_link_fraction_derivative_matches_oracle_differences(oracle_mod):
    """dq/dc (the body centre) of the link fraction of Sec. III for spheres and planes, against central
    differences of the forward oracle's or_q (measured 3e-10; bound 1e-8); q itself equal."""
    O = oracle_mod
    rng = np.random.default_rng(4)
    R = 4.3
    nrm = np.array([0.6, 0.0, 0.8])
    sph = O.make_body("sphere", center=(0, 0, 0), radius=R)
    pl = O.make_body("plane", center=(0, 0, 0), normal=tuple(nrm))
    c, _ = O.lattice()

    def inside(body, cb, p):
        return np.sum((p - cb) ** 2) < R * R if body is sph else nrm @ (p - cb) < 0

    worst = 0.0
    for body in (sph, pl):
        n = 0
        while n < 100:
            i = int(rng.integers(27))
            cb = rng.uniform(-0.5, 0.5, 3)
            d = rng.standard_normal(3)
            xb = np.rint(cb + (R + rng.uniform(0, 1.5)) * d / np.linalg.norm(d)) if body is sph else \
                np.rint(cb + rng.uniform(-3, 3, 3))
            if i == 13 or inside(body, cb, xb) or not inside(body, cb, xb - c[i]):
                continue
            n += 1
            xbc = np.ascontiguousarray(xb, dtype=np.float64)
            q0 = O.lib().or_q(body, O._dp(np.ascontiguousarray(cb)), O._dp(xbc), i)
            q, g = O.link_fraction_adjoint(body, cb, xb, i)
            assert abs(q - q0) <= 1e-15
            for a in range(3):
                def fun(h, a=a):
                    cc = cb.copy()
                    cc[a] += h
                    return O.lib().or_q(body, O._dp(cc), O._dp(xbc), i)
                fd = _rich(fun, 1e-6)
                worst = max(worst, abs(fd - g[a]) / max(1.0, abs(fd)))
    _say(f"link fraction derivative: max error {worst:.1e}")
    assert worst <= 1e-8


# ----------------------------------------------------------------------------- whole step
def _small_case(O, t0, seed):
    cfg = SMALL
    nx, ny, nz = cfg["shape"]
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1e-5, 1e-5, size=(3, nz, ny, nx))
    rho, u = WL.uniform_flow(cfg["shape"], cfg["u_in"])
    s = O.Simulation(cfg["shape"], cfg["nu"], rho, u, bodies=[cfg["body"]], channel=True, u_in=cfg["u_in"], F=F)
    masks = []
    s.step(t0 + 1, record_masks=masks)
    masks = dict(enumerate(masks))
    s2 = O.Simulation(cfg["shape"], cfg["nu"], rho, u, bodies=[cfg["body"]], channel=True, u_in=cfg["u_in"], F=F)
    s2.step(t0)
    A = s2.A * (1.0 + 1e-3 * rng.standard_normal(s2.A.shape))

    def make(Ax, Fx, amp):
        body = dict(cfg["body"])
        body["amp"] = amp
        sim = O.Simulation(cfg["shape"], cfg["nu"], A0=Ax, bodies=[body], channel=True, u_in=cfg["u_in"], F=Fx)
        sim.t = t0
        sim.solid = masks[t0].copy()
        sim.frozen_masks = masks
        return sim
    return dict(A=A, F=F, masks=masks, make=make, amp=cfg["body"]["amp"], rng=rng)


@pytest.fixture(scope="module", params=[7, 28])
def small(request, oracle_mod):
    O = oracle_mod
    t0 = request.param
    c = _small_case(O, t0, 100 + t0)
    rng = c["rng"]
    c["t0"] = t0
    c["lam"] = rng.standard_normal(c["A"].shape)
    c["w"] = np.array([0.7, -0.3, 0.2])
    sim = c["make"](c["A"], c["F"], c["amp"])
    c["adj"] = sim.adjoint_step(c["lam"], c["w"])
    s_t, s_t1 = c["masks"][t0], c["masks"][t0 + 1]
    c["refill"] = (s_t > 0) & (s_t1 == 0)
    c["covered"] = (s_t == 0) & (s_t1 > 0)
    _say(f"t0={t0}: {int(c['refill'].sum())} refill nodes, {int(c['covered'].sum())} covered nodes")
    assert c["refill"].sum() > 0 and c["covered"].sum() > 0
    return c


def _L(c, Ax, Fx, amp):
    r = c["make"](Ax, Fx, amp).step(1)
    return r.A, r.forces[-1][0, :3]


def _dir_deriv(c, dA=None, dF=None, damp=0.0, h=1e-8, rich=True):
    """Central difference of L along (dA, dF, damp); the differences of A^{t+1} and of the force are
    formed before the inner products, so rounding stays at the level of the differences."""
    def fun(s):
        A = c["A"] + s * dA if dA is not None else c["A"]
        F = c["F"] + s * dF if dF is not None else c["F"]
        return _L(c, A, F, c["amp"] + s * damp)

    def D1(hh):
        Ap, fp = fun(hh)
        Am, fm = fun(-hh)
        return (np.sum(c["lam"] * (Ap - Am)) + c["w"] @ (fp - fm)) / (2 * hh)
    d1 = D1(h)
    if not rich:
        return d1
    return (4 * d1 - D1(2 * h)) / 3


def test_step_forward_values_equal_the_oracle_step(small, oracle_mod):
    """The adjoint library's restated step: A^{t+1} and the body force equal or_step's (the step that
    is differentiated is the oracle's)."""
    _, _, _, A1, forces = small["adj"]
    r = small["make"](small["A"], small["F"], small["amp"]).step(1)
    dA = np.max(np.abs(A1 - r.A))
    dF = np.max(np.abs(forces[0] - r.forces[-1][0, :3])) / np.max(np.abs(r.forces[-1][0, :3]))
    _say(f"t0={small['t0']}: restated step vs or_step: max|dA| {dA:.1e}, force rel {dF:.1e}")
    assert dA <= 1e-15 and dF <= 1e-13


def test_step_adjoint_random_direction(small):
    """<dL/dA^t, dA> for a random dA against the oracle's central differences (Richardson, h = 1e-8):
    measured 3e-8 relative; bound 1e-6."""
    lo = small["adj"][0]
    dA = small["rng"].standard_normal(small["A"].shape)
    fd = _dir_deriv(small, dA=dA)
    ad = float(np.sum(lo * dA))
    _say(f"t0={small['t0']}: random dA: FD {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(fd):.1e}")
    assert abs(fd - ad) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("where", ["inlet", "outlet", "walls", "refill", "covered"])
def test_step_adjoint_local_directions(small, where):
    """Directions confined to one kind of irregular place, so that an error there cannot hide under
    the bulk: the inlet face x <= 1, the outlet x >= nx-2 (the outlet copy pulls one entry twice), the
    fluid nodes next to the body and their bounce-back entries, the nodes the body uncovers (their
    refill reads R^t and U^t of neighbours), the nodes it covers.  Bound 1e-6 relative (measured
    <= 4e-8), or 1e-9 absolute where the derivative vanishes."""
    c = small
    s_t, s_t1 = c["masks"][c["t0"]], c["masks"][c["t0"] + 1]
    nz, ny, nx = s_t.shape
    sel = np.zeros_like(s_t, dtype=bool)
    if where == "inlet":
        sel[:, :, :2] = True
    elif where == "outlet":
        sel[:, :, nx - 2:] = True
    elif where == "walls":
        solid = (s_t1 > 0)
        sel = binary_dilation(solid, iterations=1) & ~solid
    elif where == "refill":
        sel = binary_dilation(c["refill"], iterations=2)
    else:
        sel = binary_dilation(c["covered"], iterations=1)
    dA = c["rng"].standard_normal(c["A"].shape) * sel[None]
    fd = _dir_deriv(c, dA=dA)
    ad = float(np.sum(c["adj"][0] * dA))
    _say(f"t0={c['t0']} {where}: {int(sel.sum())} nodes: FD {fd:.10e} adjoint {ad:.10e}")
    assert abs(fd - ad) <= max(1e-6 * abs(fd), 1e-9)


def test_step_adjoint_single_entries(small):
    """Single entries of dL/dA^t at places chosen to cover every rule: refill nodes and their
    neighbours, bounce-back entries of wall nodes, the inlet face, the outlet entries pulled twice,
    nodes solid at t+1, plain bulk nodes.  Each against the oracle's central difference in that
    entry alone (Richardson, h = 1e-7: the rounding of the summed body force, about 1e-15, limits
    the difference quotient to ~1e-8 at h = 1e-8 and below).  Measured max 1.1e-8 absolute on
    entries of order 0.1-3; bound 1e-7 absolute + 1e-6 relative."""
    c = small
    lo = c["adj"][0]
    s_t, s_t1 = c["masks"][c["t0"]], c["masks"][c["t0"] + 1]
    nz, ny, nx = s_t.shape
    rng = np.random.default_rng(c["t0"])
    picks = []
    ref = np.argwhere(binary_dilation(c["refill"], iterations=1))
    wall = np.argwhere(binary_dilation(s_t1 > 0, iterations=1) & (s_t1 == 0))
    for arr, k in ((ref, 6), (wall, 6)):
        for idx in rng.choice(len(arr), size=k, replace=False):
            picks.append((int(rng.integers(27)), *map(int, arr[idx])))
    for _ in range(3):
        picks.append((int(rng.choice([0, 3, 6, 9, 12, 15, 18, 21, 24])), int(rng.integers(nz)), int(rng.integers(ny)), 0))
        picks.append((int(rng.choice([0, 3, 6, 9, 12, 15, 18, 21, 24])), int(rng.integers(nz)), int(rng.integers(ny)), nx - 1))
        picks.append((int(rng.integers(27)), int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(24, 34))))
    solid = np.argwhere(s_t1 > 0)
    picks.append((int(rng.integers(27)), *map(int, solid[len(solid) // 2])))
    worst = 0.0
    for (i, z, y, x) in picks:
        dA = np.zeros_like(c["A"])
        dA[i, z, y, x] = 1.0
        fd = _dir_deriv(c, dA=dA, h=1e-7)
        err = abs(fd - lo[i, z, y, x])
        worst = max(worst, err / (1e-7 + 1e-6 * abs(fd)))
        _say(f"  entry {(i, z, y, x)}: FD {fd:.10e} adjoint {lo[i, z, y, x]:.10e} error {err:.1e}")
    _say(f"t0={c['t0']}: {len(picks)} single entries, worst error / bound = {worst:.2e}")
    assert worst <= 1.0


def test_step_adjoint_body_force(small):
    """<dL/dF, v> for a random direction (the body force enters smoothly: h = 0.1 on |v| <= 1e-6,
    measured 3e-10 relative, bound 1e-7), and dL/dF at 16 seeded nodes x 3 components, each against the
    oracle's central difference in that component alone (measured <= 1e-6 relative at these nodes'
    magnitudes; bound 1e-5 relative + 1e-9 absolute)."""
    c = small
    gF = c["adj"][1]
    rng = np.random.default_rng(1610)
    v = rng.uniform(-1e-6, 1e-6, c["F"].shape)
    fd = _dir_deriv(c, dF=v, h=0.1, rich=False)
    ad = float(np.sum(gF * v))
    _say(f"t0={c['t0']}: <dL/dF, v>: FD {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(fd):.1e}")
    assert abs(fd - ad) <= 1e-7 * abs(fd)
    s_t1 = c["masks"][c["t0"] + 1]
    fluid = np.argwhere(s_t1 == 0)
    worst = 0.0
    for idx in rng.choice(len(fluid), size=16, replace=False):
        z, y, x = map(int, fluid[idx])
        for a in range(3):
            e = np.zeros_like(c["F"])
            e[a, z, y, x] = 1.0
            fd = _dir_deriv(c, dF=e, h=1e-7)
            worst = max(worst, abs(fd - gF[a, z, y, x]) / (1e-9 + 1e-5 * abs(fd)))
    _say(f"t0={c['t0']}: dL/dF at 16 nodes x 3: worst error / bound {worst:.2e}")
    assert worst <= 1.0


def test_step_adjoint_amplitude(small):
    """dL/d(amp) (through the link fractions, wall velocities, rho_dyn, refill velocity and the rigid
    U^t of nodes solid at t) against the oracle's central difference with the masks frozen (Richardson,
    h = 1e-5): measured 3e-10 relative; bound 1e-7."""
    c = small
    g = c["adj"][2][0]
    fd = _dir_deriv(c, damp=1.0, h=1e-5)
    _say(f"t0={c['t0']}: dL/d(amp): FD {fd:.10e} adjoint {g:.10e} rel {abs(fd - g) / abs(fd):.1e}")
    assert abs(fd - g) <= 1e-7 * abs(fd)


def test_stream_only_adjoint_is_the_inverse_permutation(oracle_mod):
    """Streaming alone on a periodic box: A^{t+1}_i(x) = A^t_i(x - c_i), a permutation, so
    dL/dA^t_i(x) = lam_i(x + c_i) exactly."""
    O = oracle_mod
    shape = (7, 5, 4)
    nx, ny, nz = shape
    rng = np.random.default_rng(9)
    A = O.lattice()[1][:, None, None, None] * (1 + 0.1 * rng.standard_normal((27, nz, ny, nx)))
    s = O.Simulation(shape, 0.1, A0=A, stream_only=True)
    lam = rng.standard_normal((27, nz, ny, nx))
    lo = s.adjoint_step(lam)[0]
    c, _ = O.lattice()
    want = np.stack([np.roll(lam[i], shift=(-c[i, 2], -c[i, 1], -c[i, 0]), axis=(0, 1, 2)) for i in range(27)])
    assert np.array_equal(lo, want)


def test_periodic_plane_and_rotating_sphere_lbgk(oracle_mod):
    """A periodic box with a moving plane wall and an oscillating, rotating sphere, LBGK collision:
    random-direction inner products for A, F and both amplitudes (measured <= 5e-9 relative; bound
    1e-6)."""
    O = oracle_mod
    shape = (24, 18, 16)
    nx, ny, nz = shape
    bodies = [dict(kind="plane", center=(0, 3.3, 0), normal=(0, 1, 0), amp=0.7, period=40.0,
                   direction=(0, 1, 0)),
              WL.sphere((12.2, 10.1, 7.9), 3.2, amp=1.5, period=50.0, direction=(1, 0, 0), omega=(0.0, 0.0, 0.004))]
    rng = np.random.default_rng(12)
    F = rng.uniform(-1e-5, 1e-5, size=(3, nz, ny, nx))
    rho, u = WL.uniform_flow(shape, (0.02, 0.0, 0.01))
    t0 = 9
    s = O.Simulation(shape, 0.02, rho, u, bodies=bodies, F=F, stabiliser="lbgk")
    masks = []
    s.step(t0 + 1, record_masks=masks)
    masks = dict(enumerate(masks))
    s0 = O.Simulation(shape, 0.02, rho, u, bodies=bodies, F=F, stabiliser="lbgk")
    s0.step(t0)
    A = s0.A * (1 + 1e-3 * rng.standard_normal(s0.A.shape))
    assert int(((masks[t0] > 0) & (masks[t0 + 1] == 0)).sum()) > 0

    def make(Ax, Fx, amps):
        bs = [dict(b, amp=a) for b, a in zip(bodies, amps)]
        sim = O.Simulation(shape, 0.02, A0=Ax, bodies=bs, F=Fx, stabiliser="lbgk")
        sim.t = t0
        sim.solid = masks[t0].copy()
        sim.frozen_masks = masks
        return sim
    amps = np.array([b["amp"] for b in bodies])
    lam = rng.standard_normal(A.shape)
    w = np.array([[0.2, 0.9, -0.1], [0.5, 0.3, 0.4]])
    lo, gF, gamp, _, _ = make(A, F, amps).adjoint_step(lam, w)

    def D(dA, dF, da, h):
        def L(s):
            r = make(A + s * dA, F + s * dF, amps + s * da).step(1)
            return r.A, r.forces[-1][:, :3]
        Ap, fp = L(h)
        Am, fm = L(-h)
        return (np.sum(lam * (Ap - Am)) + np.sum(w * (fp - fm))) / (2 * h)
    z = np.zeros_like(A)
    zF = np.zeros_like(F)
    dA = rng.standard_normal(A.shape)
    fd = (4 * D(dA, zF, 0 * amps, 1e-8) - D(dA, zF, 0 * amps, 2e-8)) / 3
    ad = float(np.sum(lo * dA))
    _say(f"periodic bodies, LBGK: dA FD {fd:.10e} adjoint {ad:.10e}")
    assert abs(fd - ad) <= 1e-6 * abs(fd)
    v = rng.uniform(-1e-6, 1e-6, F.shape)
    fd = D(z, v, 0 * amps, 0.1)
    ad = float(np.sum(gF * v))
    _say(f"periodic bodies, LBGK: dF FD {fd:.10e} adjoint {ad:.10e}")
    assert abs(fd - ad) <= 1e-6 * abs(fd)
    for k in range(2):
        e = np.zeros(2)
        e[k] = 1.0
        fd = (4 * D(z, zF, e, 1e-5) - D(z, zF, e, 2e-5)) / 3
        _say(f"periodic bodies, LBGK: d/d(amp_{k}) FD {fd:.10e} adjoint {gamp[k]:.10e}")
        assert abs(fd - gamp[k]) <= 1e-6 * abs(fd)
