"""Failure detection and diagnostics of the library (no counterpart in the paper; the test on the
state is the domain of the entropic equilibrium of Sec. II, eq. feq_min): a non-finite population,
or a node whose velocity leaves the domain where every feq_i > 0, is reported by elbm_get_info and
turned into ELBM_ENONFINITE by elbm_force; the recorded gamma range equals the oracle's; a boundary
list that overflows its capacity is reported as ELBM_ENOSPACE.  The faulty states are ordinary data
written through elbm_write_populations: every kernel treats them as numbers."""
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


def _noisy_equilibrium(O, shape, seed):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    c, w = O.lattice()
    return w[:, None, None, None] * (1.0 + 0.02 * rng.standard_normal((27, nz, ny, nx)))


def test_healthy_state_is_not_flagged(E, oracle_mod):
    shape = (16, 16, 8)
    _say("case: healthy state")
    lat = E.Lattice(shape, 0.01)
    lat.write_populations(_noisy_equilibrium(oracle_mod, shape, 1), 0)
    lat.step(3)
    assert lat.info().nonfinite == 0


@pytest.mark.parametrize("fault", ["nan", "inf", "velocity"])
def test_failed_state_is_reported(E, oracle_mod, fault):
    """One node of a periodic box gets a NaN population, an infinite one, or populations whose
    velocity is u_x = 1.2 (outside |u| < 1, where the equilibrium has non-positive members)."""
    shape = (16, 16, 8)
    _say(f"case: failed state ({fault})")
    A = _noisy_equilibrium(oracle_mod, shape, 2)
    c, w = oracle_mod.lattice()
    if fault == "nan":
        A[5, 3, 4, 5] = np.nan
    elif fault == "inf":
        A[14, 3, 4, 5] = np.inf
    else:
        f = w.copy()
        f[c[:, 0] == 1] += 1.2 / 9.0   # j_x = 1.2 with rho = 1 + 1.2
        f[13] -= 1.2                   # ... brought back to rho = 1
        A[:, 3, 4, 5] = f
    lat = E.Lattice(shape, 0.01)
    lat.write_populations(A, 0)
    assert lat.info().nonfinite == 0   # cleared when the populations are set
    lat.step(1)
    nf = lat.info().nonfinite
    _say(f"{fault}: nonfinite = {nf}")
    assert nf & 1


def test_failed_state_makes_force_fail(E, oracle_mod):
    """With a body in the channel, the force read-back of a step that met a failed state returns
    ELBM_ENONFINITE."""
    shape = (32, 16, 16)
    _say("case: force read-back after a failed state")
    rho, u = WL.uniform_flow(shape, (0.02, 0.0, 0.0))
    lat = E.Lattice(shape, 0.02, channel=True, u_inlet=(0.02, 0.0, 0.0), max_bodies=1)
    lat.init_equilibrium(rho, u)
    lat.set_bodies([WL.sphere((14.0, 8.0, 8.0), 3.0)])
    lat.step(2)
    lat.force(0, 2)   # healthy so far
    A = lat.populations().cpu().numpy()
    A[4, 2, 3, 25] = np.nan
    lat.write_populations(A, 2)
    lat.step(1)
    with pytest.raises(E.ElbmError, match="elbm error -5"):
        lat.force(0, 3)


def test_gamma_range_matches_oracle(E, oracle_mod):
    """The recorded range of the stabiliser over one step equals the oracle's (FP32 arithmetic on the
    GPU: bound 1e-4 relative)."""
    O = oracle_mod
    shape, nu = (16, 16, 16), 0.005
    rho, u = WL.taylor_green_3d(16, 0.05)
    rng = np.random.default_rng(4)
    A0 = O.Simulation(shape, nu, rho, u).A * (1.0 + 1e-2 * rng.standard_normal((27, 16, 16, 16)))
    _say("case: gamma range")
    lat = E.Lattice(shape, nu)
    lat.write_populations(A0, 0)
    E.elbm_set_diagnostics(lat.ctx, True)
    lat.step(1)
    info = lat.info()
    s = O.Simulation(shape, nu, A0=A0).step(1)
    gmin, gmax = s.stats[-1]["gamma_min"], s.stats[-1]["gamma_max"]
    _say(f"gamma range: gpu [{info.gamma_min:.6f}, {info.gamma_max:.6f}] oracle [{gmin:.6f}, {gmax:.6f}]")
    assert info.gamma_stats == 1
    assert abs(info.gamma_min - gmin) <= 1e-4 * abs(gmin) and abs(info.gamma_max - gmax) <= 1e-4 * abs(gmax)
    info2 = lat.info()   # the range restarts after each read
    assert info2.gamma_min == 0.0 and info2.gamma_max == 0.0


def test_boundary_list_overflow_is_reported(E, torch_cuda):
    """A channel whose inlet face alone (16 x 16 nodes) exceeds max_boundary fails at creation with
    ELBM_ENOSPACE; a moving sphere whose boundary nodes exceed the remaining capacity makes
    elbm_get_info report ELBM_ENOSPACE after the step (the list writes stop at the capacity)."""
    _say("case: boundary list overflow")
    with pytest.raises(E.ElbmError, match="elbm error -2"):
        E.Lattice((32, 16, 16), 0.02, channel=True, u_inlet=(0.02, 0, 0), max_bodies=1, max_boundary=100)
    lat = E.Lattice((32, 16, 16), 0.02, channel=True, u_inlet=(0.02, 0, 0), max_bodies=1, max_boundary=16 * 16 + 20)
    rho, u = WL.uniform_flow((32, 16, 16), (0.02, 0.0, 0.0))
    lat.init_equilibrium(rho, u)
    lat.set_bodies([WL.sphere((14.0, 8.0, 8.0), 4.0, amp=1.0, period=40.0)])
    lat.step(1)
    with pytest.raises(E.ElbmError, match="elbm error -2"):
        lat.info()
