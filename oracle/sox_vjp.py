"""Reference vector-Jacobian products of the SOX self-energy (oracle; test
infrastructure only).

L = sum_{tau,t,r} R[tau,t,r] Sigma[tau,t,r] is differentiated with torch CPU
float64 autograd through the paper's step chain (section "THC-SOX and
THC-SOSEX", static list and eq:GG list), written here a second time in torch
so autograd can trace it.  Gradients are with respect to every entry of the
general (not symmetrised) inputs G(tau), X, U1, U2 / W_tau.  The pins
(finite differences of the numpy 4-index brute force) are in
tests/test_oracle_vjp.py.
"""
from __future__ import annotations

import numpy as np
import torch


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def sigma_static_torch(X, U1, U2, G):
    """The static chain (eq:U_contraction, G_Rq, G_wP, A, B, C, D, Sigma) in
    torch; G(beta - tau) is node n_tau-1-k."""
    Gb = torch.flip(G, dims=[0])
    U1t = torch.einsum("PQ,qQ,sQ->Pqs", U1, X, X)
    U2t = torch.einsum("RS,vS,wS->Rvw", U2, X, X)
    GRq = torch.einsum("uR,kuq->kRq", X, G)
    GwP = torch.einsum("kwp,pP->kwP", G, X)
    A = torch.einsum("Pqs,ksv->kPqv", U1t, Gb)
    B = torch.einsum("kPqv,kRq->kPRv", A, GRq)
    C = torch.einsum("Rvw,kwP->kRvP", U2t, GwP)
    D = torch.einsum("kPRv,kRvP->kPR", B, C)
    return -torch.einsum("tR,kPR,rP->ktr", X, D, X)


def sigma_dynamic_torch(X, W_tau, V, G, T_fwd, T_bwd):
    """The dynamic chain (eq:GG, FT, W(Omega) GG(Omega), IFT, B, C, D,
    Sigma) in torch with the supplied transform pair."""
    Gb = torch.flip(G, dims=[0])
    Tf = torch.as_tensor(T_fwd, dtype=torch.complex128)
    Tb = torch.as_tensor(T_bwd, dtype=torch.complex128)
    Wm = torch.einsum("mj,jPQ->mPQ", Tf, W_tau.to(torch.complex128))
    U2t = torch.einsum("RS,vS,wS->Rvw", V, X, X)
    GuQ = torch.einsum("juq,qQ->juQ", G, X)
    GQv = torch.einsum("sQ,jsv->jQv", X, Gb)
    GG = torch.einsum("juQ,jQv->jQuv", GuQ, GQv)
    GGm = torch.einsum("mj,jQuv->mQuv", Tf, GG.to(torch.complex128))
    Am = torch.einsum("mPQ,mQuv->mPuv", Wm, GGm)
    A = torch.einsum("im,mPuv->iPuv", Tb, Am).real
    B = torch.einsum("iPuv,uR->iPRv", A, X)
    C = torch.einsum("Rvw,iwP->iRvP", U2t, GuQ)
    D = torch.einsum("iPRv,iRvP->iPR", B, C)
    return -torch.einsum("tR,iPR,rP->itr", X, D, X)


def vjp_static(X, U1, U2, G, R, bare: bool = False):
    """(dG, dX, dU1, dU2) of L = sum(Sigma * R) for Sigma = SOX(U1, U2).
    With bare=True, U1 = U2 = V is one tensor and dU1 is the total dV."""
    Xt, Gt = _t(X).requires_grad_(), _t(G).requires_grad_()
    if bare:
        Vt = _t(U1).requires_grad_()
        S = sigma_static_torch(Xt, Vt, Vt, Gt)
        L = (S * _t(R)).sum()
        dG, dX, dV = torch.autograd.grad(L, [Gt, Xt, Vt])
        return dG.numpy(), dX.numpy(), dV.numpy(), None
    U1t, U2t = _t(U1).requires_grad_(), _t(U2).requires_grad_()
    S = sigma_static_torch(Xt, U1t, U2t, Gt)
    L = (S * _t(R)).sum()
    dG, dX, d1, d2 = torch.autograd.grad(L, [Gt, Xt, U1t, U2t])
    return dG.numpy(), dX.numpy(), d1.numpy(), d2.numpy()


def vjp_dynamic(X, W_tau, V, G, R, T_fwd, T_bwd):
    """(dG, dX, dW_tau, dV) of L = sum(Sigma * R) for the dynamic entry."""
    Xt, Gt = _t(X).requires_grad_(), _t(G).requires_grad_()
    Wt, Vt = _t(W_tau).requires_grad_(), _t(V).requires_grad_()
    S = sigma_dynamic_torch(Xt, Wt, Vt, Gt, T_fwd, T_bwd)
    L = (S * _t(R)).sum()
    dG, dX, dW, dV = torch.autograd.grad(L, [Gt, Xt, Wt, Vt])
    return dG.numpy(), dX.numpy(), dW.numpy(), dV.numpy()
