"""Differentiable rollouts: a ``torch.autograd.Function`` around ``elbm_step`` (forward) and the
hand-written adjoint ``elbm_adjoint_step`` (reverse), with checkpoints every K steps and
recomputation of the states in between.

The objective is a weighted sum of the momentum-exchange force on body 0 over the rollout,
L = sum_t w_t . F_0(t) (t = 1..T are the time levels produced by the steps); a time-averaged drag
over a window is the case w_t = (1/n, 0, 0) inside the window.  Gradients are returned for the
body-force field F(x) (FP32, [3][nz][ny][nx]) and for body 0's oscillation amplitude.  All compute
runs in the HIP library; this module only orders the calls and keeps the checkpoints.
"""
from __future__ import annotations

import numpy as np
import torch

from . import elbm


class ForceRollout:
    """A T-step rollout on a fresh lattice, re-runnable for different parameters."""

    def __init__(self, shape, nu, body: dict, steps: int, weights, checkpoint: int = 20, channel: bool = False,
                 u_in=(0.0, 0.0, 0.0), storage: str = "f32", rho=None, u=None):
        self.shape = tuple(shape)
        self.nu = nu
        self.body = dict(body)
        self.steps = int(steps)
        self.weights = np.asarray(weights, dtype=np.float64).reshape(self.steps, 3)
        self.K = int(checkpoint)
        self.channel = channel
        self.u_in = u_in
        self.storage = storage
        nx, ny, nz = self.shape
        self.rho = rho
        self.u = np.zeros((3, nz, ny, nx)) if u is None else u
        self.lat = None
        self.ckpt = {}
        self.forces = None

    def _lattice(self):
        flags = elbm.FLAG_BODY_FORCE | elbm.FLAG_ADJOINT
        return elbm.Lattice(self.shape, self.nu, storage=self.storage, channel=self.channel, u_inlet=self.u_in,
                            max_bodies=1, flags=flags, force_ring=max(1, self.steps))

    def forward(self, F: torch.Tensor, amp: float) -> float:
        if self.lat is None:
            self.lat = self._lattice()
        lat = self.lat
        body = dict(self.body)
        body["amp"] = float(amp)
        lat.init_equilibrium(self.rho, self.u)
        lat.set_bodies([body])
        self.F = F.detach().to(torch.float32).contiguous()
        elbm.elbm_set_body_force(lat.ctx, self.F)
        self.ckpt = {0: lat.state_tensor()}
        for t in range(self.steps):
            lat.step(1)
            if (t + 1) % self.K == 0 and t + 1 < self.steps:
                self.ckpt[t + 1] = lat.state_tensor()
        self.forces = lat.force_history(0, 1, self.steps)
        return float(np.sum(self.weights * self.forces[:, :3]))

    def backward(self):
        lat = self.lat
        nx, ny, nz = self.shape
        lam = torch.zeros((27, nz, ny, nx), dtype=torch.float32, device="cuda")
        lam2 = torch.empty_like(lam)
        gF = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device="cuda")
        elbm.elbm_adjoint_param_grad(lat.ctx, 1, reset=True)
        starts = sorted(self.ckpt)
        # the recomputed levels of a segment are stepped straight into these buffers (no copies);
        # they start as copies of a valid state so that nodes a step leaves alone (solid ones) hold
        # finite values
        bufs = [self.ckpt[0].clone() for _ in range(min(self.K, self.steps) - 1)]
        for s0 in reversed(starts):
            s1 = min(s0 + self.K, self.steps)
            lat.load_state(self.ckpt[s0], s0)
            states = [self.ckpt[s0]]
            for t in range(s0, s1 - 1):
                # the forward pass recorded these levels' forces already
                elbm.elbm_step_into(lat.ctx, bufs[t - s0], skip_force=True)
                states.append(bufs[t - s0])
            for t in reversed(range(s0, s1)):
                w = self.weights[t]           # loss weight of time level t+1
                wf = w if np.any(w != 0.0) else None
                elbm.elbm_adjoint_step(lat.ctx, t, states[t - s0], lam, lam2, wf, gF)
                lam, lam2 = lam2, lam
            del states
        gamp = float(elbm.elbm_adjoint_param_grad(lat.ctx, 1, reset=True)[0])
        lat.load_state(self.ckpt[0], 0)
        return gF, gamp


class ForceLoss(torch.autograd.Function):
    """L = sum_t w_t . F_0(t) of a ForceRollout; differentiable in the body-force field and the amplitude."""

    @staticmethod
    def forward(ctx, F, amp, rollout: ForceRollout):
        L = rollout.forward(F, float(amp))
        ctx.rollout = rollout
        return torch.tensor(L, dtype=torch.float64, device=F.device)

    @staticmethod
    def backward(ctx, gL):
        gF, gamp = ctx.rollout.backward()
        g = gL.to(torch.float64)
        return (gF * g.to(gF.dtype)), torch.tensor(gamp, dtype=torch.float64, device=gF.device) * g, None


def window_weights(steps: int, first: int, last: int, component: int = 0):
    """Weights of the mean of force component `component` over time levels first..last (inclusive)."""
    w = np.zeros((steps, 3))
    n = last - first + 1
    for t in range(first, last + 1):
        w[t - 1, component] = 1.0 / n
    return w
