"""torch.autograd.Function wrappers: forward runs sox_sigma_*, backward runs
sox_sigma_vjp (the hand-written adjoint kernels, which recompute the
forward intermediates per tau slab instead of storing them)."""
from __future__ import annotations

import torch

from . import binding as B


class SoxSigmaStatic(torch.autograd.Function):
    """Sigma = SOX(U1, U2) with static interactions.  U2 None means the bare
    entry (U1 = U2 = V)."""

    @staticmethod
    def forward(ctx, plan, X, U1, U2, G):
        S = torch.empty_like(G)
        if U2 is None:
            B.sox_sigma_bare(plan, X, U1, G, S)
        else:
            B.sox_sigma_static(plan, X, U1, U2, G, S)
        ctx.plan = plan
        ctx.bare = U2 is None
        ctx.save_for_backward(X, U1, U1 if U2 is None else U2, G)
        return S

    @staticmethod
    def backward(ctx, R):
        X, U1, U2, G = ctx.saved_tensors
        R = R.contiguous()
        dG = torch.empty_like(G) if ctx.needs_input_grad[4] else None
        dX = torch.empty_like(X) if ctx.needs_input_grad[1] else None
        dU1 = torch.empty_like(U1) if ctx.needs_input_grad[2] else None
        dU2 = None
        if ctx.bare:
            B.sox_sigma_vjp(ctx.plan, "bare", X, U1, None, G, R, dG, dX, dU1, None)
        else:
            dU2 = torch.empty_like(U2) if ctx.needs_input_grad[3] else None
            B.sox_sigma_vjp(ctx.plan, "static", X, U1, U2, G, R, dG, dX, dU1, dU2)
        return None, dX, dU1, dU2, dG


class SoxSigmaDynamic(torch.autograd.Function):
    """Sigma = SOX(W_d(tau), V) with the plan's transform pair."""

    @staticmethod
    def forward(ctx, plan, X, W_tau, V, G):
        S = torch.empty_like(G)
        B.sox_sigma_dynamic(plan, X, W_tau, V, G, S)
        ctx.plan = plan
        ctx.save_for_backward(X, W_tau, V, G)
        return S

    @staticmethod
    def backward(ctx, R):
        X, W, V, G = ctx.saved_tensors
        R = R.contiguous()
        dG = torch.empty_like(G) if ctx.needs_input_grad[4] else None
        dX = torch.empty_like(X) if ctx.needs_input_grad[1] else None
        dW = torch.empty_like(W) if ctx.needs_input_grad[2] else None
        dV = torch.empty_like(V) if ctx.needs_input_grad[3] else None
        B.sox_sigma_vjp(ctx.plan, "dynamic", X, W, V, G, R, dG, dX, dW, dV)
        return None, dX, dW, dV, dG


def sox_sigma(plan, X, U1, G, U2=None):
    """Differentiable static / bare SOX self-energy."""
    return SoxSigmaStatic.apply(plan, X, U1, U2, G)


def sox_sigma_dynamic(plan, X, W_tau, V, G):
    """Differentiable dynamically screened SOX self-energy."""
    return SoxSigmaDynamic.apply(plan, X, W_tau, V, G)
