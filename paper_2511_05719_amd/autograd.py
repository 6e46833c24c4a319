"""log P(record) as a differentiable torch function.

The probability of a fixed trajectory record (its measurement bits and
Kraus branches; the product of the Born and jump probabilities of Sec. III.C,
Eq. 2-3) depends on every noise location's SRX angle (Eq. 1) and damping
(Eq. 3).  `log_prob` wraps the library's forced pass and its hand-written
adjoint (ttn_log_prob_grad) in a torch.autograd.Function: the forward call
runs the forced pass, and, when an input needs a gradient, the reverse sweep
that yields d log P / d theta_l and d log P / d gamma_l for every row and
location in the same call; backward contracts those Jacobian rows with the
incoming gradient (a vector-Jacobian product, no extra library call).

Parameters may be per row [rows, n_loc], shared by all rows [n_loc], or one
scalar tied over every location; the gradient comes back in the same shape
(summed over rows, and over locations for a scalar).
"""
from __future__ import annotations

import torch

from .engine import OpList, TTNEngine


def _as_param(x, device) -> torch.Tensor:
    return torch.as_tensor(x, dtype=torch.float64, device=device)


def _expand(p: torch.Tensor, rows: int, n_loc: int) -> torch.Tensor:
    if p.dim() == 0:
        return p.reshape(1, 1).expand(rows, n_loc).contiguous()
    if p.dim() == 1:
        return p.reshape(1, -1).expand(rows, n_loc).contiguous()
    if p.shape != (rows, n_loc):
        raise ValueError(f"parameters must be a scalar, [n_loc] or [{rows}, {n_loc}]")
    return p.contiguous()


def _reduce(g: torch.Tensor, like: torch.Tensor) -> torch.Tensor:
    if like.dim() == 0:
        g = g.sum()
    elif like.dim() == 1:
        g = g.sum(dim=0)
    return g.to(device=like.device, dtype=like.dtype)


class LogProb(torch.autograd.Function):
    """log P(records, branches | theta, gamma) per row (float64 [rows])."""

    @staticmethod
    def forward(ctx, theta, gamma, engine: TTNEngine, oplist: OpList, records, branches):
        rows, n_loc = engine.batch, max(oplist.n_loc, 1)
        th = _expand(theta.detach(), rows, n_loc)
        ga = _expand(gamma.detach(), rows, n_loc)
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            lp, dth, dga, st = engine.log_prob_grad(oplist, records, branches, theta=th, gamma=ga)
            ctx.save_for_backward(dth, dga)
        else:
            lp, st = engine.log_prob(oplist, records, branches, theta=th, gamma=ga)
        ctx.like = (theta, gamma)
        ctx.flagged = st.get("flagged_rows", 0)
        return lp.clone()

    @staticmethod
    def backward(ctx, grad_lp):
        dth, dga = ctx.saved_tensors
        g = grad_lp.to(torch.float64).reshape(-1, 1)
        th_like, ga_like = ctx.like
        gt = _reduce(g * dth, th_like) if ctx.needs_input_grad[0] else None
        gg = _reduce(g * dga, ga_like) if ctx.needs_input_grad[1] else None
        return gt, gg, None, None, None, None


def log_prob(engine: TTNEngine, oplist: OpList, records, branches=None, theta=0.0, gamma=0.0) -> torch.Tensor:
    """Differentiable log P of each row's record (see the module docstring).

    records: [rows, n_rec] uint8, branches: [rows, n_ad] int8 (None without
    AD ops); theta, gamma: scalar, [n_loc] or [rows, n_loc] float64 tensors
    (or numbers) on any device; the result lives on the engine's device."""
    th = theta if torch.is_tensor(theta) else _as_param(theta, engine.device)
    ga = gamma if torch.is_tensor(gamma) else _as_param(gamma, engine.device)
    return LogProb.apply(th, ga, engine, oplist, records, branches)
