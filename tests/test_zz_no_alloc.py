"""The allocation-free periodic step (elbm_step_periodic_noalloc, its FP64 queue in a static device
array) against elbm_step on a context (the same kernels, the queue in the caller's workspace):
bit-identical storage, on two calls in a row, the second on a smaller lattice.  The states are the
equilibrium weights plus a shear mode, a correlated higher-order mode and per-node noise, with the
FP64 threshold at 1e-4, so that every node of the first step enters the FP64 queue (the first
lattice's queue goes past the fix-up kernel's lane-form limit, the second's stays within it)."""
import numpy as np
import pytest

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


def _state(shape, seed):
    nx, ny, nz = shape
    i = np.arange(27)
    c = np.stack([i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1], axis=1)
    w1 = np.where(c == 0, 2.0 / 3.0, 1.0 / 6.0)
    w = w1[:, 0] * w1[:, 1] * w1[:, 2]
    mode_s = np.where(c[:, 2] == 0, c[:, 0] * c[:, 1], 0).astype(float)
    mode_h = (c[:, 0] * c[:, 1] * (3 * c[:, 2] ** 2 - 2)).astype(float)
    rng = np.random.default_rng(seed)
    return (w + 1e-2 * mode_s + 1e-4 * mode_h)[:, None, None, None] + 1e-5 * rng.uniform(-1, 1, (27, nz, ny, nx))


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_noalloc_step_matches_context_step(E, torch_cuda, storage):
    torch = torch_cuda
    for shape, seed in (((64, 32, 24), 5), ((16, 16, 8), 6)):  # the second call is smaller
        _say(f"case: allocation-free step {storage} {shape}")
        nu, thr = 0.01, 1e-4
        lat = E.Lattice(shape, nu, storage=storage, fp64_threshold=thr)
        lat.write_populations(_state(shape, seed), 0)
        pin = lat.state_tensor()
        lat.step(1)
        queued = lat.info().fp64_nodes
        want = lat.state_tensor()
        pout = torch.full_like(pin, 7)
        params = E.make_params(shape, nu, storage=storage, fp64_threshold=thr)
        E.elbm_step_periodic_noalloc(params, pin, pout)
        torch.cuda.synchronize()
        same = bool(torch.equal(pout, want))
        _say(f"{storage} {shape}: FP64 queue {queued} of {lat.N} nodes, identical to elbm_step: {same}")
        assert queued == lat.N
        assert same
        lat.close()
