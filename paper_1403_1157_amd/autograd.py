"""torch.autograd front end of the CDG2 adjoint.

:class:`CDG2RK` runs ``nsteps`` SSP-RK3 steps of the HIP operator in its forward
pass, keeping a checkpoint of the state every ``ckpt`` steps.  Its backward pass
walks the checkpoints in reverse; for each segment one library call
(``cdg2_rk_adjoint_segment``) recomputes the segment's states and stages with the
forward kernels and applies the discrete adjoint of each step from the last to
the first, accumulating the parameter derivatives on the device.  It returns
gradients with respect to the initial state and to the 21 differentiable
coefficients (diffusion, chemotaxis, reactions).  The arithmetic runs in the
library; this module only orders the calls and holds the checkpoints.
"""
from __future__ import annotations

import torch

from .cdg2 import COEFF_NAMES, Operator

NDIFF = 21


def coeffs_with(base: dict, theta) -> dict:
    """Copy of ``base`` with the 21 differentiable coefficients taken from theta."""
    c = dict(base)
    vals = theta.detach().cpu().double().tolist() if isinstance(theta, torch.Tensor) else list(theta)
    for name, v in zip(COEFF_NAMES[:NDIFF], vals):
        c[name] = float(v)
    return c


def theta_of(coeffs: dict) -> torch.Tensor:
    return torch.tensor([float(coeffs[k]) for k in COEFF_NAMES[:NDIFF]], dtype=torch.float64)


class CDG2RK(torch.autograd.Function):
    """U_T = Phi^nsteps(U0; theta) with checkpointed discrete-adjoint backward."""

    @staticmethod
    def forward(ctx, U0: torch.Tensor, theta: torch.Tensor, op: Operator, base: dict,
                dt: float, nsteps: int, ckpt: int = 20):
        op.set_coeffs(coeffs_with(base, theta))
        U = U0.detach().clone()
        checkpoints = [U.clone()]
        for n in range(nsteps):
            op.rk_step(U, dt, 1)
            if (n + 1) % ckpt == 0 and n + 1 < nsteps:
                checkpoints.append(U.clone())
        op.sync()
        ctx.op, ctx.dt, ctx.nsteps, ctx.ckpt = op, dt, nsteps, ckpt
        ctx.checkpoints = checkpoints
        ctx.base, ctx.theta = base, theta.detach().clone()
        return U

    @staticmethod
    def backward(ctx, gU: torch.Tensor):
        op, dt, nsteps, ckpt = ctx.op, ctx.dt, ctx.nsteps, ctx.ckpt
        op.set_coeffs(coeffs_with(ctx.base, ctx.theta))
        lam = gU.detach().contiguous().clone()
        dth = torch.zeros(NDIFF, dtype=torch.float64, device=lam.device)
        nseg = (nsteps + ckpt - 1) // ckpt
        for seg in reversed(range(nseg)):
            start = seg * ckpt
            end = min(start + ckpt, nsteps)
            # recompute of the segment and its reverse sweep, enqueued by the library
            op.rk_adjoint_segment(ctx.checkpoints[seg], end - start, dt, lam, dth)
        op.sync()
        return lam, dth.cpu(), None, None, None, None, None


def mismatch_loss(U: torch.Tensor, target: torch.Tensor, vol: float, species=(0, 5)) -> torch.Tensor:
    """L = 1/2 sum_{s in species} ||u_s - t_s||^2_{L2} = 1/2 |K| sum (U - T)^2 over the
    selected species (orthonormal modes)."""
    d = U[list(species)] - target[list(species)]
    return 0.5 * vol * (d * d).sum()
