"""torch.autograd access to the governor's margins.

Both functions run entirely in librg: the forward is the rollout kernel
(``rg_margin``), the backward the reverse-mode adjoint kernel (``rg_grad``).
``kappa`` is a 0-d float64 tensor; ``theta_nom`` a float64 tensor of the plant's
nominal uncertain coefficients (FC9: 20 values; pass ``None`` for LQ4).
"""
from __future__ import annotations

import numpy as np
import torch

from .rg import Governor


def _set_theta(gov: Governor, theta_nom) -> None:
    if theta_nom is not None and gov.problem.n_theta > 0:
        gov.set_theta(theta_nom.detach().cpu().numpy().astype(np.float64))


class ScenarioMargins(torch.autograd.Function):
    """m[k] = worst constraint margin of scenario k's rollout under kappa (FP32
    rollouts); backward sums the upstream-weighted per-scenario derivatives."""

    @staticmethod
    def forward(ctx, kappa, theta_nom, gov: Governor, x, r: float, v_prev: float):
        _set_theta(gov, theta_nom)
        t = gov.get_step()
        out = gov.margin(x, r, v_prev, [float(kappa)], per_scenario=True)
        ctx.gov, ctx.x, ctx.r, ctx.v_prev, ctx.t = gov, np.asarray(x), r, v_prev, t
        ctx.kappa = float(kappa)
        ctx.has_theta = theta_nom is not None
        return torch.from_numpy(out["per_scenario"][0].copy())

    @staticmethod
    def backward(ctx, grad_m):
        gov = ctx.gov
        gov.set_step(ctx.t)
        up = grad_m.detach().cpu().numpy().astype(np.float32)
        g = gov.grad(ctx.x, ctx.r, ctx.v_prev, ctx.kappa, upstream=up)
        dk = torch.tensor(g["dkappa"], dtype=torch.float64)
        dth = torch.from_numpy(g["dtheta"].copy()) if ctx.has_theta else None
        return dk, dth, None, None, None, None


class WorstMargin(torch.autograd.Function):
    """M(kappa) = min(min_k m^k, m_ss); backward is the derivative of the active
    term (arg-min scenario adjoint or the steady-state implicit derivative)."""

    @staticmethod
    def forward(ctx, kappa, theta_nom, gov: Governor, x, r: float, v_prev: float):
        _set_theta(gov, theta_nom)
        t = gov.get_step()
        g = gov.grad(x, r, v_prev, float(kappa))
        ctx.save_for_backward(torch.tensor(g["dkappa"], dtype=torch.float64),
                              torch.from_numpy(g["dtheta"].copy()))
        ctx.has_theta = theta_nom is not None
        ctx.t = t
        return torch.tensor(g["M"], dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_M):
        dk, dth = ctx.saved_tensors
        return (grad_M * dk, grad_M * dth if ctx.has_theta else None, None, None, None, None)


def scenario_margins(kappa, theta_nom, gov: Governor, x, r: float, v_prev: float):
    return ScenarioMargins.apply(kappa, theta_nom, gov, x, r, v_prev)


def worst_margin(kappa, theta_nom, gov: Governor, x, r: float, v_prev: float):
    return WorstMargin.apply(kappa, theta_nom, gov, x, r, v_prev)
