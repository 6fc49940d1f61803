"""elbm_step_into (the step that stores A^{t+1} in a caller's buffer, used by the checkpointed reverse
sweep) against elbm_step: with an oscillating sphere in a channel (nodes covered and uncovered in
the steps stepped into buffers), the forces of every step and the populations of every fluid node
at every level agree bit for bit; the borrowed buffer is reported and released as documented; a
recompute from a saved level with ELBM_STEP_SKIP_FORCE reproduces the states and leaves the recorded
forces in place; bad destinations and flags are rejected on the host."""
import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu

SHAPE = (48, 24, 24)
BODY = WL.sphere((16.2, 12.1, 11.8), 4.0, amp=2.0, period=24.0, direction=(0, 1, 0))


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


def _lattice(E, storage):
    rho, u = WL.uniform_flow(SHAPE, (0.03, 0.0, 0.0))
    lat = E.Lattice(SHAPE, 0.02, storage=storage, channel=True, u_inlet=(0.03, 0.0, 0.0), max_bodies=1,
                    force_ring=16)
    lat.init_equilibrium(rho, u)
    lat.set_bodies([BODY])
    return lat


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_step_into_matches_step(E, torch_cuda, storage):
    torch = torch_cuda
    _say(f"case: elbm_step_into vs elbm_step, {SHAPE}, {storage}")
    steps, into = 10, range(3, 8)   # levels 3..7 are produced by elbm_step_into
    ref = _lattice(E, storage)
    states, fluid = {}, {}
    for t in range(steps):
        ref.step(1)
        states[t + 1] = ref.state_tensor()
        fluid[t + 1] = (ref.flags() & 1) == 0
    f_ref = ref.force_history(0, 1, steps)
    lat = _lattice(E, storage)
    bufs = {}
    for t in range(steps):
        if t + 1 in into:
            bufs[t + 1] = torch.full_like(states[1], 0)
            E.elbm_step_into(lat.ctx, bufs[t + 1])
            assert lat.info().pop_offset == 2 ** 64 - 1
            with pytest.raises(E.ElbmError):
                lat.population_view()
        else:
            lat.step(1)
            lat.population_view()   # the workspace holds the populations again
    f = lat.force_history(0, 1, steps)
    torch.cuda.synchronize()
    shp = lat.storage_shape()
    for k in range(1, steps + 1):
        got = bufs[k] if k in bufs else (lat.state_tensor() if k == steps else None)
        if got is None:
            continue
        a = got.view(shp).cpu().numpy()
        b = states[k].view(shp).cpu().numpy()
        m = fluid[k].cpu().numpy()
        if shp[0] == 27:
            diff = int(np.count_nonzero(a[:, m] != b[:, m]))
        else:
            diff = int(np.count_nonzero((a != b) & m[:, :, None, :]))
        _say(f"level {k}: {diff} differing fluid entries")
        assert diff == 0
    uncovered = sum(int(((~fluid[k - 1]) & fluid[k]).sum()) for k in into)
    covered = sum(int((fluid[k - 1] & ~fluid[k]).sum()) for k in into)
    _say(f"forces of {steps} steps identical; {uncovered} uncovered, {covered} covered nodes in the steps into buffers")
    assert np.array_equal(f, f_ref), np.max(np.abs(f - f_ref))
    assert uncovered > 0 and covered > 0


def test_recompute_without_force_sums(E, torch_cuda):
    """Levels 1..8 by elbm_step (forces recorded), then the state of level 3 loaded back and levels
    4..7 recomputed into buffers with the force sums skipped: the populations of every fluid node
    bit-identical, the force history unchanged."""
    torch = torch_cuda
    _say("case: recompute with ELBM_STEP_SKIP_FORCE")
    lat = _lattice(E, "f32")
    states, fluid = {}, {}
    for t in range(8):
        lat.step(1)
        states[t + 1] = lat.state_tensor()
        fluid[t + 1] = ((lat.flags() & 1) == 0).cpu().numpy()
    f_ref = lat.force_history(0, 1, 8)
    lat.load_state(states[3], 3)
    bufs = [torch.zeros_like(states[1]) for _ in range(4)]
    for k in range(4):
        E.elbm_step_into(lat.ctx, bufs[k], skip_force=True)
    torch.cuda.synchronize()
    shp = lat.storage_shape()
    for k in range(4):
        a = bufs[k].view(shp).cpu().numpy()
        b = states[4 + k].view(shp).cpu().numpy()
        diff = int(np.count_nonzero((a != b) & fluid[4 + k][:, :, None, :]))
        _say(f"recomputed level {4 + k}: {diff} differing fluid entries")
        assert diff == 0
    f = lat.force_history(0, 1, 7)   # the lattice is back at level 7
    assert np.array_equal(f, f_ref[:7])


def test_step_into_rejects_bad_destinations(E, torch_cuda):
    torch = torch_cuda
    _say("case: elbm_step_into argument checks")
    lat = _lattice(E, "f16")
    cur = lat.population_view().data_ptr()   # start of the current population buffer
    with pytest.raises(E.ElbmError, match="elbm error -1"):
        E.elbm_step_into(lat.ctx, cur + 64)                  # overlaps the current populations
    big = torch.empty(27 * lat.N + 8, dtype=torch.float16, device="cuda")
    with pytest.raises(E.ElbmError, match="elbm error -1"):
        E.elbm_step_into(lat.ctx, big[1:])                   # 2-byte aligned
    with pytest.raises(E.ElbmError, match="elbm error -1"):
        E.elbm_step_into(lat.ctx, None)
    ok = torch.empty(27 * lat.N, dtype=torch.float16, device="cuda")
    assert E.load().elbm_step_into(lat.ctx, ok.data_ptr(), 6) == -1   # unknown flag bits: ELBM_EINVAL
    assert lat.info().t == 0
    free = E.Lattice(SHAPE, 0.02, channel=True, u_inlet=(0.03, 0.0, 0.0), max_bodies=1)
    rho, u = WL.uniform_flow(SHAPE, (0.0, 0.0, 0.0))
    free.init_equilibrium(rho, u)
    free.set_bodies([WL.free_sphere((16.0, 12.0, 12.0), 4.0, 2.0)])
    buf = torch.empty(27 * free.N, dtype=torch.float32, device="cuda")
    with pytest.raises(E.ElbmError, match="free bodies"):
        E.elbm_step_into(free.ctx, buf, skip_force=True)
