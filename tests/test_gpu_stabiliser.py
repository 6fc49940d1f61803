"""Collision variants on the GPU against the oracle: the exact root of eq. gamma_min (bracketed
Newton from the analytic value, FP32 with the FP64 recomputation rule), gamma = 2 (LBGK), and the
central-moment shear part (analytic stabiliser), on single collisions, on 100 steps of the 32^3
Taylor-Green workload, and at moving walls."""
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


def _flag(E, mode):
    return {"exact": E.FLAG_EXACT_GAMMA, "lbgk": E.FLAG_LBGK, "central": E.FLAG_CENTRAL}[mode]


def _oracle_kw(mode):
    return dict(stabiliser="kbc", central=True) if mode == "central" else dict(stabiliser=mode)


@pytest.mark.parametrize("mode", ["exact", "lbgk", "central"])
def test_collision_variants_match_oracle(E, oracle_mod, torch_cuda, mode):
    O = oracle_mod
    torch = torch_cuda
    rng = np.random.default_rng(6)
    n = 4096
    states = []
    for k in range(n):
        u = rng.uniform(-0.08, 0.08, 3)
        f = O.feq(rng.uniform(0.9, 1.1), u)
        eps = [1e-4, 1e-3, 1e-2, 3e-2][k % 4]
        states.append(f * (1 + eps * rng.standard_normal(27)))
    S = np.array(states).astype(np.float32).astype(np.float64)
    nu = 0.004
    beta = O.beta_from_nu(nu)
    fin = torch.tensor(S.T.copy(), dtype=torch.float32, device="cuda")
    fout = torch.empty_like(fin)
    gam = torch.empty(n, dtype=torch.float32, device="cuda")
    E.elbm_collide_nodes(fin, fout, gam, None, n, nu, 0.0, _flag(E, mode))
    torch.cuda.synchronize()
    got = fout.cpu().numpy().T.astype(np.float64)
    g = gam.cpu().numpy().astype(np.float64)
    ref, gref = [], []
    for st in S:
        gf = O.gamma_exact(st, beta) if mode == "exact" else (2.0 if mode == "lbgk" else 0.0)
        r, gm, _ = O.collide(st, beta, gamma_fixed=gf, central=(mode == "central"))
        ref.append(r)
        gref.append(gm)
    ref, gref = np.array(ref), np.array(gref)
    err = np.max(np.abs(got - ref))
    # gamma is ill-conditioned where the deviation is tiny: compare it on the larger deviations
    big = np.array([k % 4 >= 2 for k in range(n)])
    gerr = np.max(np.abs(g[big] - gref[big]) / np.abs(gref[big]))
    _say(f"{mode}: collide max|df| = {err:.3e}, gamma rel (eps >= 1e-2) {gerr:.2e}")
    assert err < 1e-6
    assert gerr < 1e-3


@pytest.mark.parametrize("mode", ["exact", "lbgk", "central"])
def test_taylor_green_variants(E, oracle_mod, mode):
    O = oracle_mod
    w = WL.WORKLOADS["tg32"]
    rho, u = WL.initial_field("tg32")
    lat = E.Lattice(w["shape"], w["nu"], flags=_flag(E, mode))
    lat.init_equilibrium(rho, u)
    lat.step(w["steps"])
    got = lat.populations().cpu().numpy()
    ref = O.Simulation(w["shape"], w["nu"], rho, u, **_oracle_kw(mode)).step(w["steps"]).A
    err = np.max(np.abs(got - ref))
    _say(f"tg32 {mode}: max|df| = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("mode", ["exact", "lbgk", "central"])
def test_moving_wall_variants(E, oracle_mod, mode):
    """Wall kernel path: an oscillating sphere in a small channel, 30 steps.  Measured up to 7.5e-8 on
    the populations and 9e-8 on the force; bounds 1e-6 and 1e-5."""
    O = oracle_mod
    shape, nu = (40, 20, 20), 0.01
    body = WL.sphere((15.3, 10.2, 9.8), 4.0, amp=1.5, period=40.0, direction=(0.0, 1.0, 0.0))
    rho, u = WL.uniform_flow(shape, (0.03, 0.0, 0.0))
    lat = E.Lattice(shape, nu, channel=True, u_inlet=(0.03, 0.0, 0.0), max_bodies=1, flags=_flag(E, mode))
    lat.init_equilibrium(rho, u)
    lat.set_bodies([body])
    lat.step(30)
    s = O.Simulation(shape, nu, rho, u, bodies=[body], channel=True, u_in=(0.03, 0.0, 0.0),
                     **_oracle_kw(mode)).step(30)
    fluid = s.solid == 0
    err = np.max(np.abs(lat.populations().cpu().numpy()[:, fluid] - s.A[:, fluid]))
    F = lat.force_history(0, 1, 30)[:, :3]
    Fo = np.array([f[0, :3] for f in s.forces])
    ef = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    _say(f"moving wall {mode}: max|df| = {err:.3e}, force rel {ef:.2e}")
    assert err <= 1e-6
    assert ef <= 1e-5
