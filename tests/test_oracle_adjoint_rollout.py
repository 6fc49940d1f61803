"""The oracle adjoint over a rollout (oracle.force_rollout_adjoint: checkpointed reverse sweep of
Simulation.adjoint_step) against central differences of oracle rollouts with the masks of the
nominal run frozen: the differentiable workload's structure (oscillating sphere in a channel, a
seeded body-force field, loss = mean drag over a window) at a size the CPU suite affords.

Per-node checks of dL/dF at 16 seeded nodes x 3 components, each by perturbing that one component
(steps 1e-7 on components of order 1e-6, in FP64; an FP32 rollout could not resolve the resulting
change of the loss), the inner product with a direction v uniform in [-1e-6, 1e-6] at the
workload's step h = 1e-3, and dL/d(amp) at the converged step 1e-5 (Richardson) -- the workload's
stated step 1e-3 is reported beside it, not gated: the stabiliser responds nonlinearly at nodes whose
<dh|dh> is tiny, and the difference quotient at 1e-3 has not converged."""
import numpy as np
import pytest

import workloads as WL

CFG = dict(shape=(36, 18, 18), nu=0.02, channel=True, u_in=(0.03, 0.0, 0.0), steps=30, window=(10, 30),
           body=WL.sphere((14.2, 9.1, 8.8), 3.5, amp=2.0, period=100.0, direction=(0, 1, 0)))


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def case(oracle_mod):
    O = oracle_mod
    c = CFG
    steps = c["steps"]
    F = WL.body_force(c["shape"], 1610, 1e-6)
    rho, u = WL.uniform_flow(c["shape"], c["u_in"])
    w = np.zeros((steps, 3))
    n = c["window"][1] - c["window"][0] + 1
    w[c["window"][0] - 1:c["window"][1], 0] = 1.0 / n
    L, gF, gamp, masks = O.force_rollout_adjoint(c["shape"], c["nu"], [c["body"]], steps, w, rho=rho, u=u, F=F,
                                                 channel=True, u_in=c["u_in"], checkpoint=7)
    refills = sum(int(((masks[t] > 0) & (masks[t + 1] == 0)).sum()) for t in range(steps))
    _say(f"rollout: L = {L:.10e}, {refills} refills over {steps} steps")
    assert refills > 0

    def loss(amp=c["body"]["amp"], Fx=F):
        body = dict(c["body"], amp=amp)
        s = O.Simulation(c["shape"], c["nu"], rho, u, bodies=[body], channel=True, u_in=c["u_in"], F=Fx)
        s.frozen_masks = masks
        s.solid = masks[0].copy()
        s.step(steps)
        return float(sum(w[t] @ s.forces[t][0, :3] for t in range(steps)))
    assert abs(loss() - L) <= 1e-14 * abs(L)
    return dict(L=L, gF=gF, gamp=gamp[0], F=F, loss=loss, amp=c["body"]["amp"])


def test_rollout_amplitude_gradient(case):
    """dL/d(amp) against the converged central difference (Richardson over 1e-5, 2e-5): measured
    7e-10 relative; bound 1e-7.  The workload's step 1e-3 is printed beside it."""
    amp, loss = case["amp"], case["loss"]

    def cd(h):
        return (loss(amp=amp + h) - loss(amp=amp - h)) / (2 * h)
    fd = (4 * cd(1e-5) - cd(2e-5)) / 3
    fd3 = cd(1e-3)
    g = case["gamp"]
    _say(f"dL/d(amp): adjoint {g:.10e}  FD(1e-5, Richardson) {fd:.10e} rel {abs(g - fd) / abs(fd):.1e}  "
         f"FD(1e-3) {fd3:.10e} rel {abs(g - fd3) / abs(fd):.1e}")
    assert abs(g - fd) <= 1e-7 * abs(fd)


def test_rollout_body_force_direction(case):
    """<dL/dF, v>, v uniform in [-1e-6, 1e-6] (seed 1611), at the workload's step h = 1e-3: measured
    2e-9 relative; bound 1e-6."""
    rng = np.random.default_rng(1611)
    v = rng.uniform(-1e-6, 1e-6, case["F"].shape)
    h = 1e-3
    fd = (case["loss"](Fx=case["F"] + h * v) - case["loss"](Fx=case["F"] - h * v)) / (2 * h)
    g = float(np.sum(case["gF"] * v))
    _say(f"<dL/dF, v>: adjoint {g:.10e} FD {fd:.10e} rel {abs(g - fd) / abs(fd):.1e}")
    assert abs(g - fd) <= 1e-6 * abs(fd)


def test_rollout_body_force_per_node(case):
    """dL/dF at 16 seeded fluid nodes x 3 components, each against the FP64 central difference in that
    component alone (Richardson over steps 1e-7 and 2e-7 on components of order 1e-6: larger steps
    have not converged -- near-equilibrium nodes make the stabiliser respond nonlinearly -- and the
    rounding of the summed drag, ~6e-16, puts a floor of ~5e-9 under the quotient).  Measured <= 1e-8
    absolute on entries of order 1e-4 to 1e-1; bound 3e-8 absolute + 1e-6 relative."""
    F, gF = case["F"], case["gF"]
    rng = np.random.default_rng(1612)
    nz, ny, nx = F.shape[1:]
    picks = []
    while len(picks) < 16:
        z, y, x = int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))
        if np.any(gF[:, z, y, x] != 0.0):   # fluid in every step (solid nodes have no body force)
            picks.append((z, y, x))
    worst = 0.0
    for (z, y, x) in picks:
        for a in range(3):
            e = np.zeros_like(F)
            e[a, z, y, x] = 1.0

            def cd(h):
                return (case["loss"](Fx=F + h * e) - case["loss"](Fx=F - h * e)) / (2 * h)
            fd = (4 * cd(1e-7) - cd(2e-7)) / 3
            g = gF[a, z, y, x]
            worst = max(worst, abs(g - fd) / (3e-8 + 1e-6 * abs(fd)))
            _say(f"  dL/dF[{a}] at {(x, y, z)}: adjoint {g:.8e} FD {fd:.8e} error {abs(g - fd):.1e}")
    _say(f"dL/dF at 16 nodes x 3: worst error / bound {worst:.2e}")
    assert worst <= 1.0
