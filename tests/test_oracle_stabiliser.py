"""Stabiliser variants of the oracle step (the rows after the hot path): gamma = 2 makes a step the
plain LBGK update f' = f + 2 beta (feq - f) of the pulled populations; the exact stabiliser applies, at
every node, the collision with the root of eq. gamma_min of that node's pulled populations."""
import numpy as np

import workloads as WL


def _random_state(O, shape, seed, eps=2e-2):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.standard_normal((nz, ny, nx))
    u = 0.04 * rng.standard_normal((3, nz, ny, nx))
    s = O.Simulation(shape, 0.05, rho, u)
    return s.A * (1.0 + eps * rng.standard_normal(s.A.shape))


def _pulled(O, A):
    c, _ = O.lattice()
    return np.stack([np.roll(A[i], shift=(int(c[i, 2]), int(c[i, 1]), int(c[i, 0])), axis=(0, 1, 2))
                     for i in range(27)])


def test_lbgk_step_is_bgk_relaxation(oracle_mod):
    O = oracle_mod
    shape, nu = (8, 6, 5), 0.05
    A = _random_state(O, shape, 3)
    beta = O.beta_from_nu(nu)
    got = O.Simulation(shape, nu, A0=A, stabiliser="lbgk").step(1).A
    f = _pulled(O, A).reshape(27, -1)
    c, _ = O.lattice()
    rho = f.sum(0)
    u = (c.T @ f) / rho
    ref = np.empty_like(f)
    for n in range(f.shape[1]):
        feq = O.feq(rho[n], u[:, n])
        ref[:, n] = f[:, n] + 2.0 * beta * (feq - f[:, n])
    assert np.max(np.abs(got.reshape(27, -1) - ref)) < 1e-14


def test_exact_step_uses_each_nodes_exact_root(oracle_mod):
    O = oracle_mod
    shape, nu = (6, 5, 4), 0.01
    A = _random_state(O, shape, 4)
    beta = O.beta_from_nu(nu)
    got = O.Simulation(shape, nu, A0=A, stabiliser="exact").step(1).A.reshape(27, -1)
    f = _pulled(O, A).reshape(27, -1)
    for n in range(f.shape[1]):
        ge = O.gamma_exact(f[:, n], beta)
        assert np.isfinite(ge) and ge > 0.0
        ref, gam, _ = O.collide(f[:, n], beta, gamma_fixed=ge)
        assert np.max(np.abs(got[:, n] - ref)) < 1e-15
        # and it is not the analytic stabiliser (they differ at second order in the deviation)
        _, ga, _ = O.collide(f[:, n], beta)
        assert abs(ge - ga) > 1e-9 * abs(ga)
