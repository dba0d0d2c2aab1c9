"""Deposit-misfit loss of a Mode-I run as a differentiable torch function.

The back-calculation of basal friction and release volume from a mapped
deposit (the use of many model runs the paper motivates in Sect. 1 and
Sect. 5): ``DepositLoss(prob, target_h, nsteps)`` maps a per-cell friction
field tan(delta_b) and a release-volume scale s to

    L(mu, s) = 1/2 sum_cells (h_n(mu, s) - h_target)^2 dx dy,

where h_n is the bed-normal thickness after ``nsteps`` steps from the release
of ``prob`` scaled by s.  The forward run and the reverse sweep are the
library's (``m2p_adjoint_run``: checkpoints every ``ckpt_every`` steps,
segment recomputation, transposed stage kernels, time steps frozen at the
forward run's values); this module only marshals tensors.  Gradients are
those of the discrete scheme with the forward run's time steps held fixed.
"""
from __future__ import annotations

import numpy as np
import torch

from .sim import Sim


class _DepositLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tan_mu, vol_scale, runner, need):
        mu = tan_mu.detach().to("cpu", torch.float64).numpy()
        s = float(vol_scale.detach().to("cpu", torch.float64))
        loss, gmu, gvol = runner.evaluate(mu, s, need)
        if need:
            ctx.save_for_backward(torch.as_tensor(gmu, dtype=tan_mu.dtype, device=tan_mu.device),
                                  torch.tensor(gvol, dtype=vol_scale.dtype, device=vol_scale.device))
        return torch.tensor(loss, dtype=torch.float64, device=tan_mu.device)

    @staticmethod
    def backward(ctx, grad_out):
        gmu, gvol = ctx.saved_tensors
        g = grad_out.to(gmu.dtype)
        return g * gmu, g.to(gvol.dtype) * gvol, None, None


class DepositLoss:
    """Differentiable deposit misfit of one scenario (Mode-I release).

    ``loss = DepositLoss(prob, target_h, nsteps)(tan_mu, vol_scale)`` with
    ``tan_mu`` a [ny, nx] tensor and ``vol_scale`` a 0-d tensor; ``loss`` is a
    0-d float64 tensor whose ``backward()`` fills ``tan_mu.grad`` and
    ``vol_scale.grad``.  ``precision`` is "f32" (FP32 state) or "f64".
    """

    def __init__(self, prob, target_h, nsteps: int, ckpt_every: int = 100, precision: str = "f32",
                 stream=None):
        self.prob = prob
        self.target = np.ascontiguousarray(target_h, dtype=np.float64)
        if self.target.shape != (prob.ny, prob.nx):
            raise ValueError("target_h must be [ny, nx]")
        if prob.inflows:
            raise ValueError("the adjoint covers Mode-I releases only")
        self.nsteps = int(nsteps)
        self.ckpt_every = int(ckpt_every)
        self.sim = Sim(prob, precision=precision, stream=stream, set_state=False)
        self.evaluations = 0

    def evaluate(self, tan_mu: np.ndarray, vol_scale: float, need_grad: bool):
        """Loss (and, if need_grad, dL/dmu and dL/ds) at (tan_mu, vol_scale)."""
        p = self.prob
        self.sim.set_friction_field(tan_mu)
        self.sim.set_state(p.h_vert * vol_scale, p.phi_s, vertical=True, vel=p.vel)
        self.sim.set_time(0.0)
        self.evaluations += 1
        if need_grad:
            return self.sim.adjoint_run(self.nsteps, self.ckpt_every, self.target, vol_scale)
        self.sim.run(self.nsteps)
        return self.sim.loss(self.target), None, None

    def __call__(self, tan_mu: torch.Tensor, vol_scale: torch.Tensor) -> torch.Tensor:
        if tuple(tan_mu.shape) != (self.prob.ny, self.prob.nx):
            raise ValueError("tan_mu must be [ny, nx]")
        if vol_scale.dim() != 0:
            raise ValueError("vol_scale must be a 0-d tensor")
        need = torch.is_grad_enabled() and (tan_mu.requires_grad or vol_scale.requires_grad)
        return _DepositLossFn.apply(tan_mu, vol_scale, self, need)
