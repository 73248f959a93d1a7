"""k-point (periodic solid) SOX self-energy in plain numpy complex128 (oracle;
test infrastructure only).

Conventions (one spin channel; mesh of n_k momenta, index tables from
synth.kmesh_index):
  X   [n_k, n, N]        X^k_iP
  U   [n_k, N, N]        U^q_PQ, Hermitian, U^{-q} = conj(U^q)
  G   [n_k, n_tau, n, n] G^k_pq(tau)
  Sigma [n_k, n_tau, n, n]

THC integrals (section THC-SOX and THC-SOSEX):
  (i k_i, j k_j | s k_s, r k_r) = sum_PQ conj(X^{k_i}_iP) X^{k_j}_jP U^q_PQ conj(X^{k_s}_sQ) X^{k_r}_rQ,
  q = k_i - k_j = k_r - k_s.
eq:sox for a solid with the static time relations, the third line read at
beta - tau, and one 1/N_k per loop momentum:
  Sigma^{k_t}_tr = -(1/N_k^2) sum_{k_p,k_q} (p k_p, r k_t | q k_q, s k_s)_1
                   (t k_t, u k_q | v k_s, w k_p)_2 G^{k_p}_wp G^{k_q}_uq G^{k_s}_sv(beta-tau),
  k_s = k_p + k_q - k_t.
"""
from __future__ import annotations

import numpy as np


def g_tau_k(eps: np.ndarray, Q: np.ndarray, mu: float, beta: float, tau: np.ndarray) -> np.ndarray:
    """G^k(tau) = -Q_k diag(n(eps_k, tau)) Q_k^dagger (eq:G_def per momentum)."""
    from oracle.sox_mol import occupation_factor
    out = []
    for k in range(eps.shape[0]):
        occ = occupation_factor(eps[k], mu, beta, tau)
        out.append(-np.einsum("pa,ta,qa->tpq", Q[k], occ, Q[k].conj()))
    return np.stack(out)


def eri_k(X: np.ndarray, U: np.ndarray, ki: int, kj: int, ks: int, kr: int, kdiff) -> np.ndarray:
    """(i k_i, j k_j | s k_s, r k_r) as an [n, n, n, n] array (momentum conserving)."""
    q = kdiff[ki, kj]
    assert q == kdiff[kr, ks]
    L = np.einsum("iP,jP->ijP", X[ki].conj(), X[kj])
    Rr = np.einsum("sQ,rQ->srQ", X[ks].conj(), X[kr])
    return np.einsum("ijP,PQ,srQ->ijsr", L, U[q], Rr, optimize=True)


def sigma_solid_eri(X, U1, U2, G, tables) -> np.ndarray:
    """The 4-index brute force of eq:sox over all (k_p, k_q) for every k_t."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    Gb = G[:, ::-1]
    out = np.zeros((nk, nt, n, n), dtype=complex)
    for kt in range(nk):
        for kp in range(nk):
            for kq in range(nk):
                kss = kdiff[ksum[kp, kq], kt]
                E1 = eri_k(X, U1, kp, kt, kq, kss, kdiff)     # (p kp, r kt | q kq, s ks)
                E2 = eri_k(X, U2, kt, kq, kss, kp, kdiff)     # (t kt, u kq | v ks, w kp)
                for k in range(nt):
                    Y1 = np.einsum("prqs,wp->rqsw", E1, G[kp, k])
                    Y2 = np.einsum("rqsw,uq->rswu", Y1, G[kq, k])
                    Y3 = np.einsum("rswu,sv->rwuv", Y2, Gb[kss, k])
                    out[kt, k] -= np.einsum("tuvw,rwuv->tr", E2, Y3)
    return out / nk ** 2


def sigma_solid_thc(X, U1, U2, G, tables) -> np.ndarray:
    """The paper's k-point step chain.

    U^{q1,k_v}_Pqs = sum_Q U1^{q1}_PQ conj(X^{k_v-q1}_qQ) X^{k_v}_sQ    (eq:U_contraction)
    G^k_Rq = sum_u X^k_uR G^k_uq,  G^k_wP = sum_p G^k_wp conj(X^k_pP)
    A^{q1,k_v}_Pqv = sum_s U^{q1,k_v}_Pqs G^{k_v}_sv(beta - tau)
    B^{q1,k_v}_PRv = sum_q A^{q1,k_v}_Pqv G^{k_v-q1}_Rq
    C^{q2,k_w}_RvP = sum_w U(2)^{q2,k_w}_Rvw G^{k_w}_wP
    D^{k_t}_PR = (1/N_k) sum_{k_w, q2} sum_v C^{q2,k_w}_RvP B^{q1,k_w-q2}_PRv,  q1 = k_w - k_t
    Sigma^{k_t}_RP = -(1/N_k) D^{k_t}_PR;  Sigma^{k_t}_tr = sum_PR conj(X^{k_t}_tR) Sigma_RP X^{k_t}_rP
    """
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    N = X.shape[2]
    Gb = G[:, ::-1]

    def utensor(U, q, kv):
        kq = kdiff[kv, q]
        return np.einsum("PQ,qQ,sQ->Pqs", U[q], X[kq].conj(), X[kv], optimize=True)

    U1t = {(q, kv): utensor(U1, q, kv) for q in range(nk) for kv in range(nk)}
    U2t = {(q, kv): utensor(U2, q, kv) for q in range(nk) for kv in range(nk)}
    out = np.empty((nk, nt, n, n), dtype=complex)
    for k in range(nt):
        GRq = [X[kk].T @ G[kk, k] for kk in range(nk)]             # G^k_Rq
        GwP = [G[kk, k] @ X[kk].conj() for kk in range(nk)]        # G^k_wP
        B = {}
        for q1 in range(nk):
            for kv in range(nk):
                A = np.tensordot(U1t[(q1, kv)], Gb[kv, k], axes=(2, 0))   # A_Pqv
                kq = kdiff[kv, q1]
                B[(q1, kv)] = np.einsum("Pqv,Rq->PRv", A, GRq[kq])
        C = {}
        for q2 in range(nk):
            for kw in range(nk):
                C[(q2, kw)] = np.einsum("Rvw,wP->RvP", U2t[(q2, kw)], GwP[kw])
        for kt in range(nk):
            D = np.zeros((N, N), dtype=complex)
            for kw in range(nk):
                q1 = kdiff[kw, kt]
                for q2 in range(nk):
                    kv = kdiff[kw, q2]
                    D += np.einsum("RvP,PRv->PR", C[(q2, kw)], B[(q1, kv)]) / nk
            SigRP = -D.T / nk
            out[kt, k] = X[kt].conj() @ SigRP @ X[kt].T
    return out


def energy_gm_k(Sigma, G, weights) -> float:
    """E = -1/2 (1/N_k) sum_k sum_tau w_tau Re Tr[Sigma^k(tau) G^k(beta - tau)]."""
    nk = Sigma.shape[0]
    tr = np.einsum("ktab,ktba->t", Sigma, G[:, ::-1])
    return float(-0.5 * np.dot(weights, tr.real) / nk)
