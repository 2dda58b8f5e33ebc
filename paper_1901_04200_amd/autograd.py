"""torch.autograd view of the Monte Carlo prices.

forward(theta) = calibrate_forward_store (the paper's step 1, keeping the path
state every K steps); backward(dL/dEy) = calibrate_vjp_stored (its step 2
summed over paths, eq. 0711A) seeded with the incoming adjoint, from those
checkpoints.  If another checkpoint-writing call ran on the same context in
between, backward re-runs the forward sweep instead (calibrate_vjp).  For
L = G = 1/2 sum (Ey - C)^2 the incoming adjoint is exactly lambda = Ey - C,
so autograd reproduces the paper's two-pass gradient; any other
differentiable function of the prices works the same way.
"""
from __future__ import annotations

import torch

from . import capi
from .mc import MonteCarloCalibration


class MonteCarloPrices(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, mc):
        ctx.mc = mc
        th = theta.detach().to(torch.float64).contiguous()
        ctx.save_for_backward(th)
        Ey = mc.forward_store(th)
        ctx.ckpt_id = mc.ckpt_writes
        return Ey

    @staticmethod
    def backward(ctx, grad_out):
        (th,) = ctx.saved_tensors
        lam = grad_out.detach().to(torch.float64).contiguous()
        if ctx.mc.ckpt_writes == ctx.ckpt_id:
            g = ctx.mc.vjp_stored(th, lam)
        else:
            g = ctx.mc.vjp(th, lam)
        return g, None


def mc_prices(theta, mc: MonteCarloCalibration):
    return MonteCarloPrices.apply(theta, mc)


def checkpoint_bytes(problem, precision: str, ckpt_every: int) -> int:
    nv = 2 if problem.model in (1, 3) else 1   # Heston and SLV checkpoint (x, v)
    real = 8 if precision == "fp64" else 4
    nseg = -(-problem.n_steps // ckpt_every)
    return nseg * nv * problem.n_paths * real


def choose_ckpt_every(problem, precision: str = "fp32", budget_bytes: int | None = None) -> int:
    """The densest checkpoint spacing (least recomputation per segment and
    fewest registers) whose buffer fits the budget; the default budget is
    an eighth of the device memory free now."""
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info()
        budget_bytes = free // 8
    for k in (8, 16, 32):
        if checkpoint_bytes(problem, precision, k) <= budget_bytes:
            return k
    raise MemoryError(f"even 32-step checkpoints need {checkpoint_bytes(problem, precision, 32)} bytes "
                      f"> budget {budget_bytes}")


def make(problem, precision: str = "fp32", budget_bytes: int | None = None) -> MonteCarloCalibration:
    k = choose_ckpt_every(problem, precision, budget_bytes)
    return MonteCarloCalibration(problem, precision=precision, ckpt_every=k, ckpt_mode="store")
