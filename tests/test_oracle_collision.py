"""Pins of the oracle's single-node routines against what the paper and the
mathematics fix independently of the oracle's own formulas (Sec. II):
equilibrium as a constrained entropy minimiser, conservation, the fixed point,
H-decrease, the LBGK limit, the exact stabiliser of eq. gamma_min, and the
k/s/h moment split."""
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


@pytest.fixture(scope="module")
def lat(O):
    c, w = O.lattice()
    return c.astype(np.float64), w


def test_lattice_is_d3q27(lat):
    c, w = lat
    # all 27 velocities of {-1,0,1}^3, tensor-product weights, isotropy up to 4th order, c_s^2 = 1/3
    assert sorted(map(tuple, c.astype(int))) == sorted(itertools.product((-1, 0, 1), repeat=3))
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-15)
    # 4th-order isotropy: sum w c_a c_b c_c c_d = c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(T4, iso, atol=1e-15)
    for i in range(27):
        assert np.all(c[26 - i] == -c[i])


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.1, (0.05, -0.03, 0.02)), (0.93, (0.2, 0.1, -0.15)),
                                   (1.0, (0.0, 0.3, 0.0))])
def test_equilibrium_is_constrained_entropy_minimiser(O, lat, rho, u):
    """eq. feq_min: compare with an independent numerical solution of the minimisation
    (Newton on the convex dual: f_i = W_i exp(l0 + l.c_i) with the 4 constraints)."""
    c, w = lat
    u = np.array(u)
    j = rho * u

    A = np.c_[np.ones(27), c]
    lam = np.zeros(4)
    for _ in range(60):  # Newton on the dual; Jacobian sum_i f_i A_i A_i^T
        f_num = w * np.exp(A @ lam)
        g = A.T @ f_num - np.concatenate(([rho], j))
        lam -= np.linalg.solve(A.T @ (f_num[:, None] * A), g)
    f_num = w * np.exp(A @ lam)
    assert np.max(np.abs(A.T @ f_num - np.concatenate(([rho], j)))) < 1e-14
    f = O.feq(rho, u)
    assert np.max(np.abs(f - f_num)) < 1e-13
    # constraints and the stationarity condition ln(f/W) in span{1, c}
    assert abs(f.sum() - rho) < 1e-14
    assert np.allclose(c.T @ f, j, atol=1e-14)
    A = np.c_[np.ones(27), c]
    coef, *_ = np.linalg.lstsq(A, np.log(f / w), rcond=None)
    assert np.max(np.abs(A @ coef - np.log(f / w))) < 1e-13
    # a perturbation inside the constraint set raises H
    rng = np.random.default_rng(7)
    P = np.eye(27) - A @ np.linalg.pinv(A)
    for _ in range(20):
        d = P @ rng.standard_normal(27) * 1e-4
        assert O.H(f + d) > O.H(f)


def test_equilibrium_differs_from_polynomial_at_third_order(O, lat):
    c, w = lat
    for s in (0.02, 0.04):
        u = np.array([1.0, 0.7, -0.4]) * s
        cu = c @ u
        fpoly = w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
        diff = np.max(np.abs(O.feq(1.0, u) - fpoly))
        assert diff < 2.0 * s ** 3 and diff > 0.01 * s ** 3


def _random_state(O, rng, eps, umax=0.08):
    u = rng.uniform(-umax, umax, 3)
    f0 = O.feq(rng.uniform(0.9, 1.1), u)
    return f0 * (1.0 + eps * rng.standard_normal(27))


def test_collision_conserves_mass_and_momentum(O, lat):
    c, _ = lat
    rng = np.random.default_rng(1)
    for k in range(300):
        f = _random_state(O, rng, 0.05)
        beta = rng.uniform(0.5, 0.999)
        f2, gam, _ = O.collide(f, beta)
        assert abs(f2.sum() - f.sum()) < 1e-14
        assert np.allclose(c.T @ f2, c.T @ f, atol=1e-15)


def test_axis_factors_of_the_equilibrium_multiply_to_a_square(O, lat):
    """eq. feq_min factorises over the axes, feq_i = rho prod_a phi(c_ia; u_a), with
    phi(0) = (2/3)(2 - s) and phi(+1) phi(-1) = ((2 - s)/6)^2, s = sqrt(1 + 3u^2) (since
    (2u + s)(s - 2u) = 1 - u^2).  The GPU collision takes all three reciprocal weights of an axis
    from 1/(2 - s) through this product; here it is checked on the oracle's equilibrium, whose y and
    z factors at rest are 2/3."""
    c, _ = lat
    idx = {k: int(np.flatnonzero((c == (k, 0, 0)).all(axis=1))[0]) for k in (-1, 0, 1)}
    for u in np.linspace(-0.45, 0.45, 19):
        f = O.feq(1.0, np.array([u, 0.0, 0.0]))
        phi = {k: f[idx[k]] / (2.0 / 3.0) ** 2 for k in idx}
        s = np.sqrt(1.0 + 3.0 * u * u)
        assert abs(phi[1] * phi[-1] / ((2.0 - s) / 6.0) ** 2 - 1.0) < 1e-13
        assert abs(phi[0] / ((2.0 / 3.0) * (2.0 - s)) - 1.0) < 1e-13


def test_equilibrium_is_fixed_point(O):
    for u in ((0.0, 0.0, 0.0), (0.04, -0.02, 0.01)):
        f = O.feq(1.05, np.array(u))
        f2, gam, guard = O.collide(f, 0.97)
        assert np.max(np.abs(f2 - f)) < 1e-15


def test_H_does_not_increase(O):
    """Discrete H-theorem (Sec. II): with the analytic stabiliser H(f') <= H(f)."""
    rng = np.random.default_rng(2)
    worst = -np.inf
    for k in range(2000):
        f = _random_state(O, rng, rng.choice([1e-3, 1e-2, 3e-2]))
        beta = rng.uniform(0.5, 0.999)
        f2, gam, _ = O.collide(f, beta)
        dH = O.H(f2) - O.H(f)
        worst = max(worst, dH)
    assert worst <= 1e-15


def test_quadratic_entropy_decrease_is_exact(O, lat):
    """For the quadratic entropy Q = <df|df>/2 the analytic gamma minimises Q(f') along
    gamma; the minimum is (1-2 beta)^2 (<ds|ds> - a^2/b)/2 <= Q(f)."""
    c, w = lat
    rng = np.random.default_rng(3)
    for k in range(200):
        f = _random_state(O, rng, 0.02)
        beta = rng.uniform(0.5, 0.999)
        rho = f.sum()
        u = c.T @ f / rho
        fe = O.feq(rho, u)
        f2, gam, _ = O.collide(f, beta)
        fe2 = O.feq(f2.sum(), c.T @ f2 / f2.sum())
        Q1 = 0.5 * np.sum((f - fe) ** 2 / fe)
        Q2 = 0.5 * np.sum((f2 - fe2) ** 2 / fe2)
        assert Q2 <= Q1 + 1e-18
        # gamma is the argmin: nearby fixed gammas do not do better
        for dg in (-1e-3, 1e-3):
            f3, _, _ = O.collide(f, beta, gamma_fixed=gam + dg)
            Q3 = 0.5 * np.sum((f3 - fe2) ** 2 / fe2)
            assert Q3 >= Q2 - 1e-18


def test_fixed_gamma_two_is_lbgk(O, lat):
    """gamma = 2 turns the mirror state into LBGK: f' = f + 2 beta (feq - f) (Sec. II)."""
    c, _ = lat
    rng = np.random.default_rng(4)
    for k in range(50):
        f = _random_state(O, rng, 0.03)
        beta = rng.uniform(0.5, 0.999)
        fe = O.feq(f.sum(), c.T @ f / f.sum())
        f2, _, _ = O.collide(f, beta, gamma_fixed=2.0)
        assert np.max(np.abs(f2 - (f + 2 * beta * (fe - f)))) < 1e-15


def test_gamma_is_two_on_chapman_enskog_states(O, lat):
    """Near-equilibrium (Chapman-Enskog) states df = eps W Q:S at u = 0 with a traceless
    (incompressible) strain S give gamma = 2, i.e. the stabiliser reduces to LBGK relaxation
    near equilibrium.  (<df|dh> = (2/27) eps^2 (tr S)^2, so a trace moves gamma off 2.)"""
    c, w = lat
    rng = np.random.default_rng(5)
    for k in range(20):
        S = rng.standard_normal((3, 3))
        S = S + S.T
        S -= np.trace(S) / 3.0 * np.eye(3)
        Qs = np.einsum("ia,ib,ab->i", c, c, S) - np.trace(S) / 3.0
        for eps in (1e-4, 1e-6):
            f = w * (1.0 + eps * Qs)
            beta = rng.uniform(0.6, 0.999)
            _, gam, _ = O.collide(f, beta)
            assert abs(gam - 2.0) < 1e-8
    S = np.diag([1.0, 0.5, 0.2])
    f = w * (1.0 + 1e-5 * (np.einsum("ia,ib,ab->i", c, c, S) - np.trace(S) / 3.0))
    assert abs(O.collide(f, 0.9)[1] - 2.0) > 1e-3


def test_exact_stabiliser_agrees_to_first_order(O):
    """eq. gamma_min vs its analytic approximation: the difference vanishes linearly with the
    distance from equilibrium."""
    rng = np.random.default_rng(6)
    for k in range(10):
        u = rng.uniform(-0.05, 0.05, 3)
        base = O.feq(1.0, u)
        r = rng.standard_normal(27)
        beta = 0.95
        d = []
        for eps in (1e-2, 1e-3):
            f = base * (1 + eps * r)
            ga = O.collide(f, beta)[1]
            ge = O.gamma_exact(f, beta)
            assert np.isfinite(ge)
            d.append(abs(ga - ge))
        assert d[1] < 0.2 * d[0] + 1e-9
        assert d[0] < 0.05 * abs(ga)


def test_exact_stabiliser_minimises_H(O):
    rng = np.random.default_rng(8)
    for k in range(20):
        f = _random_state(O, rng, 0.02)
        beta = 0.9
        ge = O.gamma_exact(f, beta)
        Hs = [O.H(O.collide(f, beta, gamma_fixed=ge + d)[0]) for d in (-1e-3, 0.0, 1e-3)]
        assert Hs[1] <= Hs[0] and Hs[1] <= Hs[2]


def _moments_all(f, c):
    out = {}
    for p, q, r in itertools.product(range(3), repeat=3):
        out[(p, q, r)] = np.sum(f * c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** r)
    return out


def test_shear_part_carries_exactly_the_deviatoric_stress(O, lat):
    """s (Sec. II): the deviatoric stress of f and no other raw moment."""
    c, _ = lat
    rng = np.random.default_rng(9)
    f = rng.standard_normal(27)
    s = O.shear_part(f)
    Mf = _moments_all(f, c)
    Ms = _moments_all(s, c)
    T = Mf[(2, 0, 0)] + Mf[(0, 2, 0)] + Mf[(0, 0, 2)]
    want = {(2, 0, 0): Mf[(2, 0, 0)] - T / 3, (0, 2, 0): Mf[(0, 2, 0)] - T / 3, (0, 0, 2): Mf[(0, 0, 2)] - T / 3,
            (1, 1, 0): Mf[(1, 1, 0)], (1, 0, 1): Mf[(1, 0, 1)], (0, 1, 1): Mf[(0, 1, 1)]}
    for key, val in Ms.items():
        assert abs(val - want.get(key, 0.0)) < 1e-12, key
    # the 27 raw moments determine a population set: the map is invertible
    M = np.array([[c[i, 0] ** p * c[i, 1] ** q * c[i, 2] ** r for i in range(27)]
                  for p, q, r in itertools.product(range(3), repeat=3)])
    assert np.linalg.matrix_rank(M) == 27


def test_post_collision_moments_relax_as_stated(O, lat):
    """Deviatoric stress relaxes with 2 beta (shear viscosity) and the stress trace with
    gamma beta (bulk viscosity), Chapman-Enskog relations of Sec. II."""
    c, _ = lat
    rng = np.random.default_rng(10)
    for k in range(20):
        f = _random_state(O, rng, 0.02)
        beta = rng.uniform(0.6, 0.99)
        rho = f.sum()
        fe = O.feq(rho, c.T @ f / rho)
        f2, gam, _ = O.collide(f, beta)
        M1, Me, M2 = _moments_all(f, c), _moments_all(fe, c), _moments_all(f2, c)
        for key in ((1, 1, 0), (1, 0, 1), (0, 1, 1)):
            assert abs((M2[key] - Me[key]) - (1 - 2 * beta) * (M1[key] - Me[key])) < 1e-14
        tr = lambda M: M[(2, 0, 0)] + M[(0, 2, 0)] + M[(0, 0, 2)]
        assert abs((tr(M2) - tr(Me)) - (1 - beta * gam) * (tr(M1) - tr(Me))) < 1e-13
        dev = lambda M: M[(2, 0, 0)] - M[(0, 0, 2)]
        assert abs((dev(M2) - dev(Me)) - (1 - 2 * beta) * (dev(M1) - dev(Me))) < 1e-14


def test_body_force_adds_exact_momentum(O, lat):
    c, _ = lat
    rng = np.random.default_rng(11)
    for k in range(20):
        f = _random_state(O, rng, 0.02)
        F = rng.uniform(-1e-3, 1e-3, 3)
        f2, _, _ = O.collide(f, 0.9, F=F)
        assert abs(f2.sum() - f.sum()) < 1e-14
        assert np.allclose(c.T @ f2, c.T @ f + F, atol=1e-15)


def test_beta_from_viscosity(O):
    # nu = c_s^2 (1/(2 beta) - 1/2)
    for nu in (1e-3, 0.0048, 0.0072, 0.00815, 0.1):
        b = O.beta_from_nu(nu)
        assert abs((1.0 / 3.0) * (0.5 / b - 0.5) - nu) < 1e-15
