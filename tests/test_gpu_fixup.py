"""The FP64 recomputation of nodes whose <dh|dh> is small against the threshold while their shear
part is not (the rule of the reading on the stabiliser's ill-conditioned ratio), in both forms of
the fix-up kernel, against the FP64 oracle.  The state: W + a pure shear mode (eps c_x c_y on the
xy edges, inside s), a higher-order mode correlated with it (delta c_x c_y (3 c_z^2 - 2): no mass,
momentum or second moments, so inside h), and random noise per population and node (exercises the
pull indexing); with the threshold at 1e-4 every node is queued in the first step, gamma ~ 17.
16^3 keeps the queue within the lane form's limit (one node per 32 lanes), 32^3 goes beyond it
(one node per thread).  The FP32-only result (recomputation off) is printed for comparison."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LANE_FORM_MAX = 8192  # queue lengths the fix-up kernel serves one node per 32 lanes


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


def _state(O, n, seed):
    c, w = O.lattice()
    eps, delta, noise = 1e-2, 1e-4, 1e-5
    mode_s = np.where(c[:, 2] == 0, c[:, 0] * c[:, 1], 0).astype(float)
    mode_h = (c[:, 0] * c[:, 1] * (3 * c[:, 2] ** 2 - 2)).astype(float)
    rng = np.random.default_rng(seed)
    A0 = (w + eps * mode_s + delta * mode_h)[:, None, None, None] + noise * rng.uniform(-1, 1, (27, n, n, n))
    return A0


@pytest.mark.parametrize("n, form", [(16, "lanes"), (32, "threads")])
def test_fixup_forms_match_oracle(E, oracle_mod, n, form):
    O = oracle_mod
    shape, nu, steps, thr = (n, n, n), 0.01, 1, 1e-4  # the collision amplifies h: one step
    A0 = _state(O, n, 31 + n)
    assert A0.min() > 0
    ref = O.Simulation(shape, nu, A0=A0).step(steps).A
    _say(f"case: fix-up {form} {shape}")
    lat = E.Lattice(shape, nu, fp64_threshold=thr)
    lat.write_populations(A0, 0)
    counts = []
    for _ in range(steps):
        lat.step(1)
        counts.append(lat.info().fp64_nodes)
    err = np.max(np.abs(lat.populations().cpu().numpy() - ref))
    lat32 = E.Lattice(shape, nu, fp64_threshold=thr, flags=E.FLAG_NO_FP64)
    lat32.write_populations(A0, 0)
    lat32.step(steps)
    err32 = np.max(np.abs(lat32.populations().cpu().numpy() - ref))
    _say(f"fix-up {form} {shape}: queued per step {counts} of {n ** 3}, max|df| {err:.3e} (FP32 only: {err32:.3e})")
    if form == "lanes":
        assert 0 < min(counts) and max(counts) <= LANE_FORM_MAX
    else:
        assert min(counts) > LANE_FORM_MAX
    assert err <= 1e-7
