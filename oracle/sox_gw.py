"""THC-GW direct term in plain FP64 numpy (oracle; test infrastructure only).

The GW self-energy of fig:diag ("the dynamical part of the GW self-energy",
section "Second-order exchange with and without screened interactions"):
one propagator line and one screened-interaction line between the same two
space-time points,

    Sigma^GW(1, 2) = -G(1, 2) W_d(1, 2),

with W_d the dynamic part of the screened interaction (the bare part makes
the static Hartree-Fock term, which fig:diag draws separately).  The paper
names this term and evaluates it with the same THC factors as the SOX term
but prints no formula for it; the readings used here (also listed in the
design notes):

* Orbital form.  Projecting both points onto orbitals gives
      Sigma_ij(tau) = - sum_kl (i k | l j)_{W_d(tau)} G_kl(tau),
  the interaction in the chemists' notation of the THC section, the first
  pair (i, k) at point 1 and the second pair (l, j) at point 2.
* THC.  With (ik|lj) = sum_PQ X_iP X_kP W_PQ X_lQ X_jQ (section THC-SOX,
  molecular case) the sum factorises through the same projection as the
  SOX chain's half projection G_Rq:
      Gt_PQ(tau) = sum_kl X_kP G_kl(tau) X_lQ,
      Sigma_ij(tau) = - sum_PQ X_iP [Gt_PQ(tau) W_PQ(tau)] X_jQ.
* Solids.  (i k_i, j k_j | s k_s, r k_r) = sum_PQ conj(X^{k_i}_iP)
  X^{k_j}_jP U^q_PQ conj(X^{k_s}_sQ) X^{k_r}_rQ, q = k_i - k_j; one 1/N_k for
  the loop momentum k':
      Sigma^k_ij(tau) = -(1/N_k) sum_k' sum_ls (i k, l k' | s k', j k)_{W(tau)} G^{k'}_ls(tau)
  and in THC form
      Gt^{k'}_PQ = sum_ls X^{k'}_lP G^{k'}_ls conj(X^{k'}_sQ),
      M^k_PQ = (1/N_k) sum_k' W^{k-k'}_PQ(tau) Gt^{k'}_PQ(tau),
      Sigma^k_ij = - sum_PQ conj(X^k_iP) M^k_PQ X^k_jQ.
* W_d(tau) is an input on the tau grid of G (as for the dynamic SOX entry),
  so no transform is involved: the product is local in tau.

Conventions as in sox_mol / sox_solid: molecule X [n, N], W [n_tau, N, N],
G [n_tau, n, n]; solid X [n_k, n, N], W [n_k, n_tau, N, N] (leading index
q), G [n_k, n_tau, n, n].
"""
from __future__ import annotations

import numpy as np

from oracle import sox_mol as om
from oracle import sox_solid as osd


def sigma_gw_eri(X: np.ndarray, W: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Brute force over the 4-index integrals: Sigma_ij = -sum_kl (ik|lj) G_kl."""
    nt, n, _ = G.shape
    out = np.empty((nt, n, n))
    for t in range(nt):
        E = om.eri(X, W[t])                                # (ik|lj) as E[i, k, l, j]
        out[t] = -np.einsum("iklj,kl->ij", E, G[t])
    return out


def sigma_gw_thc(X: np.ndarray, W: np.ndarray, G: np.ndarray) -> np.ndarray:
    """THC chain: Gt = X^T G X, M = Gt * W (elementwise), Sigma = -X M X^T."""
    nt, n, _ = G.shape
    out = np.empty((nt, n, n))
    for t in range(nt):
        Gt = X.T @ G[t] @ X
        out[t] = -X @ (Gt * W[t]) @ X.T
    return out


def sigma_gw_solid_eri(X, W, G, tables) -> np.ndarray:
    """Brute force over the momentum-conserving 4-index integrals."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    out = np.zeros((nk, nt, n, n), dtype=complex)
    for t in range(nt):
        for k in range(nk):
            for kp in range(nk):
                E = osd.eri_k(X, W[:, t], k, kp, kp, k, kdiff)   # (i k, l k' | s k', j k)
                out[k, t] -= np.einsum("ilsj,ls->ij", E, G[kp, t])
    return out / nk


def sigma_gw_solid_thc(X, W, G, tables) -> np.ndarray:
    """THC chain over the mesh: projection per k', momentum convolution of the
    elementwise products, back-projection per k."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    N = X.shape[2]
    out = np.empty((nk, nt, n, n), dtype=complex)
    for t in range(nt):
        Gt = [X[kp].T @ G[kp, t] @ X[kp].conj() for kp in range(nk)]
        for k in range(nk):
            M = np.zeros((N, N), dtype=complex)
            for kp in range(nk):
                M += W[kdiff[k, kp], t] * Gt[kp]
            out[k, t] = -X[k].conj() @ (M / nk) @ X[k].T
    return out
