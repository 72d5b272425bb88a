"""Gauge-misfit loss as a differentiable PyTorch function.

The forward and the gradient both run in the HIP library (sgn_gauge_loss_grad):
a rollout that stores sqrt(T) checkpoints, then a reverse sweep of hand-written
vector-Jacobian-product kernels over the RK4 stages.  The autograd node only
hands the precomputed gradients back, scaled by the incoming cotangent.
"""

from __future__ import annotations

import torch


class GaugeMisfitLoss(torch.autograd.Function):
    """L(zeta0, b) = 1/2 sum_n sum_g (zeta_g^n - target_{n,g})^2 over an RK4 rollout."""

    @staticmethod
    def forward(ctx, zeta0, b, solver, nsteps, dt, gauges, target, checkpoint_every):
        solver.set_bathymetry(b.detach().contiguous())
        loss, gz, gb = solver.gauge_loss_grad(zeta0.detach().contiguous(), nsteps, dt, gauges, target,
                                              checkpoint_every)
        ctx.save_for_backward(gz, gb)
        return torch.tensor(loss, dtype=torch.float64, device=zeta0.device)

    @staticmethod
    def backward(ctx, gout):
        gz, gb = ctx.saved_tensors
        g = gout.to(gz.dtype)
        return g * gz, g * gb, None, None, None, None, None, None


def gauge_misfit_loss(zeta0, b, solver, nsteps: int, dt: float, gauges, target, checkpoint_every: int = 0):
    """Differentiable gauge misfit of a rollout from surface zeta0 over bathymetry b."""
    return GaugeMisfitLoss.apply(zeta0, b, solver, nsteps, dt, gauges, target, checkpoint_every)
