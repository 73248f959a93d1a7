"""Molecular SOX self-energy in plain FP64 numpy (oracle; test infrastructure).

Conventions (one spin channel, real orbitals):
  X [n, N]      THC collocation matrix X_iP
  U [N, N]      symmetric interaction in the auxiliary basis (V, W(0), W_d(tau))
  G [n_tau, n, n]   G[k, p, q] = G_pq(tau_k)
  Gb            G(beta - tau_k), i.e. G[::-1] on a mirror-symmetric grid
  Sigma [n_tau, n, n]   Sigma[k, t, r] = Sigma_tr(tau_k)
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Green's function (eq:G_def for a one-body Hamiltonian F = Q diag(eps) Q^T)
# ---------------------------------------------------------------------------
def occupation_factor(eps: np.ndarray, mu: float, beta: float, tau: np.ndarray) -> np.ndarray:
    """n(e, tau) = e^{-(e-mu) tau} / (1 + e^{-beta (e-mu)}), shape [n_tau, n].

    For a quadratic Hamiltonian the trace in eq:G_def factorises per
    eigenmode: G(tau) = -sum_a |a><a| e^{-(e_a-mu) tau} (1 - f_a) with
    1 - f_a = 1 / (1 + e^{-beta (e_a - mu)}).  For e < mu the same value is
    written as e^{(beta - tau)(e-mu)} / (1 + e^{beta (e-mu)}) so that no
    exponential overflows on [0, beta].
    """
    x = np.asarray(eps, dtype=np.float64)[None, :] - mu
    t = np.asarray(tau, dtype=np.float64)[:, None]
    pos = x >= 0.0
    xp = np.where(pos, x, 0.0)
    xn = np.where(pos, 0.0, x)
    a = np.exp(-xp * t) / (1.0 + np.exp(-beta * xp))
    b = np.exp((beta - t) * xn) / (1.0 + np.exp(beta * xn))
    return np.where(pos, a, b)


def g_tau(eps: np.ndarray, Q: np.ndarray, mu: float, beta: float, tau: np.ndarray) -> np.ndarray:
    """G(tau_k) = -Q diag(n(eps, tau_k)) Q^dagger for every node (eq:G_def)."""
    occ = occupation_factor(eps, mu, beta, tau)             # [n_tau, n]
    G = -np.einsum("pa,ka,qa->kpq", Q, occ, Q.conj())
    return G


def g_mirror(G: np.ndarray) -> np.ndarray:
    """G(beta - tau_k) on a mirror-symmetric grid: node n_tau - 1 - k."""
    return G[::-1].copy()


# ---------------------------------------------------------------------------
# 4-index integrals from the THC factors (section THC-SOX, molecular case)
# ---------------------------------------------------------------------------
def eri(X: np.ndarray, U: np.ndarray) -> np.ndarray:
    """(ij|kl) = sum_PQ X_iP X_jP U_PQ X_kQ X_lQ."""
    XX = np.einsum("iP,jP->ijP", X, X)
    return np.einsum("ijP,PQ,klQ->ijkl", XX, U, XX, optimize=True)


# ---------------------------------------------------------------------------
# brute force over the 4-index integrals (eq:sox, static time relations)
# ---------------------------------------------------------------------------
def sigma_static_eri(E1: np.ndarray, E2: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Sigma_tr(tau) = - sum_{pqsuvw} (pr|qs)_1 (tu|vw)_2 G_wp(tau) G_uq(tau) G_sv(beta-tau).

    eq:sox with both interactions instantaneous: tau_wp = tau_uq = tau and
    the third line runs backwards (read as the stored G(beta - tau)).  The six
    sums are taken one propagator at a time.
    """
    nt, n, _ = G.shape
    out = np.empty((nt, n, n))
    for k in range(nt):
        Y1 = np.einsum("prqs,wp->rqsw", E1, G[k])        # sum over p
        Y2 = np.einsum("rqsw,uq->rswu", Y1, G[k])        # sum over q
        Y3 = np.einsum("rswu,sv->rwuv", Y2, Gb[k])       # sum over s
        out[k] = -np.einsum("tuvw,rwuv->tr", E2, Y3)     # sum over u, v, w
    return out


# ---------------------------------------------------------------------------
# the paper's THC step chain for static interactions (molecule: k = 0)
# ---------------------------------------------------------------------------
def u_tensor(X: np.ndarray, U: np.ndarray) -> np.ndarray:
    """U_Pqs = sum_Q U_PQ X_qQ X_sQ  (eq:U_contraction with k = 0)."""
    return np.einsum("PQ,qQ,sQ->Pqs", U, X, X, optimize=True)


def sigma_static_thc(X: np.ndarray, U1: np.ndarray, U2: np.ndarray, G: np.ndarray,
                     Gb: np.ndarray) -> np.ndarray:
    """Static THC-SOX, step by step as the paper lists it.

    U_Pqs (eq:U_contraction), G_Rq = sum_u X_uR G_uq, G_wP = sum_p G_wp X_pP,
    A_Pqv = sum_s U_Pqs G_sv(beta-tau), B_PRv = sum_q A_Pqv G_Rq,
    C_RvP = sum_w U(2)_Rvw G_wP, D_PR = sum_v C_RvP B_PRv,
    Sigma_RP = -D_PR, Sigma_tr = sum_PR X_tR Sigma_RP X_rP.
    The v sum of D is accumulated one v at a time.
    """
    nt, n, _ = G.shape
    U1t = u_tensor(X, U1)                      # [P, q, s]
    U2t = u_tensor(X, U2)                      # [R, v, w]
    U2v = np.ascontiguousarray(U2t.transpose(1, 0, 2))   # U2t stored per v: [v][R, w]
    out = np.empty((nt, n, n))
    for k in range(nt):
        GRq = X.T @ G[k]                       # [R, q]
        GwP = G[k] @ X                         # [w, P]
        A = np.tensordot(U1t, Gb[k], axes=(2, 0))         # A_Pqv = sum_s U_Pqs G_sv(beta-tau)
        Av = np.ascontiguousarray(A.transpose(2, 0, 1))   # stored per v: [v][P, q]
        D = np.zeros((X.shape[1], X.shape[1]))
        for v in range(n):
            B_v = Av[v] @ GRq.T                # B_PRv  [P, R]
            C_v = U2v[v] @ GwP                 # C_RvP  [R, P]
            D += C_v.T * B_v
        SigRP = -D.T                           # Sigma_RP = -D_PR
        out[k] = X @ SigRP @ X.T               # sum_PR X_tR Sigma_RP X_rP
    return out


def sigma_static_aux(X: np.ndarray, U1: np.ndarray, U2: np.ndarray, G: np.ndarray,
                     Gb: np.ndarray) -> np.ndarray:
    """Everything in the auxiliary space (an N^4 cross-check of the chain).

    With M = X^T G X and Mb = X^T G(beta-tau) X, the orbital sums collapse to
    D_PR = sum_QS U1_PQ U2_RS M_RQ Mb_QS M_SP.
    """
    nt, n, _ = G.shape
    out = np.empty((nt, n, n))
    for k in range(nt):
        M = X.T @ G[k] @ X
        Mb = X.T @ Gb[k] @ X
        Z = np.einsum("QS,RS,SP->QRP", Mb, U2, M)
        D = np.einsum("PQ,RQ,QRP->PR", U1, M, Z)
        out[k] = -(X @ D.T @ X.T)
    return out


# ---------------------------------------------------------------------------
# dynamic interaction in line 1 (the paper's eq:GG scheme)
# ---------------------------------------------------------------------------
def matsubara(T_fwd: np.ndarray, f: np.ndarray) -> np.ndarray:
    """FT along axis 0: f(i Omega_m) = sum_j T_fwd[m, j] f(tau_j)."""
    return np.tensordot(T_fwd, f, axes=(1, 0))


def imag_time(T_bwd: np.ndarray, fw: np.ndarray) -> np.ndarray:
    """IFT along axis 0 for a real function: f(tau_i) = Re sum_m T_bwd[i, m] f_m."""
    return np.ascontiguousarray(np.tensordot(T_bwd, fw, axes=(1, 0)).real)


def sigma_dynamic_eri(X: np.ndarray, W_tau: np.ndarray, V: np.ndarray, G: np.ndarray,
                      Gb: np.ndarray, T_fwd: np.ndarray, T_bwd: np.ndarray) -> np.ndarray:
    """eq:sox with U(1) = W_d(tau) time dependent and U(2) = V instantaneous.

    With the U(2) vertex at the external time tau and the U(1) vertex pair at
    tau_r = 0 and tau', the lines are G_wp(tau), G_uq(tau - tau') and
    G_sv(tau' - tau) (read as G(beta - .)), and the U(1) line carries
    W(tau - (tau - tau')).  Substituting s = tau - tau' gives the periodic
    convolution
      Sigma_tr(tau) = - sum (tu|vw)_V G_wp(tau)
                      int_0^beta (pr|qs)_W(tau - s) G_uq(s) G_sv(beta - s) ds,
    evaluated with the supplied transform pair: the integral is
    Re sum_m T_bwd[i,m] W(i Omega_m) f(i Omega_m).
    """
    nt, n, _ = G.shape
    E2 = eri(X, V)
    E1w = np.stack([eri(X, W_tau[j]) for j in range(nt)])        # [nt, p, r, q, s]
    f = np.einsum("juq,jsv->juqsv", G, Gb)                        # [nt, u, q, s, v]
    E1m = matsubara(T_fwd, E1w)
    fm = matsubara(T_fwd, f)
    Km = np.einsum("mprqs,muqsv->mpruv", E1m, fm)                 # product in frequency
    K = imag_time(T_bwd, Km)                                      # [nt, p, r, u, v]
    out = np.empty((nt, n, n))
    for i in range(nt):
        out[i] = -np.einsum("tuvw,wp,pruv->tr", E2, G[i], K[i], optimize=True)
    return out


def sigma_dynamic_thc(X: np.ndarray, W_tau: np.ndarray, V: np.ndarray, G: np.ndarray,
                      Gb: np.ndarray, T_fwd: np.ndarray, T_bwd: np.ndarray) -> np.ndarray:
    """The paper's dynamic THC-SOSEX chain with the orbital index v outermost.

    GG_Quv(tau) = G_uQ(tau) G_Qv(-tau) (eq:GG; read G_Qv(beta - tau)),
    GG(Omega) = FT(GG), A_Puv(Omega) = sum_Q W_PQ(Omega) GG_Quv(Omega),
    A(tau) = IFT(A(Omega)), B_PRv = sum_u X_uR A_Puv, C_RvP = sum_w V_Rvw G_wP,
    D_PR = sum_v C_RvP B_PRv, Sigma_RP = -D_PR, Sigma_tr = sum X_tR Sigma_RP X_rP.
    """
    nt, n, _ = G.shape
    N = X.shape[1]
    Wm = matsubara(T_fwd, W_tau)                     # [n_omega, P, Q]
    U2t = u_tensor(X, V)                             # [R, v, w]
    U2v = np.ascontiguousarray(U2t.transpose(1, 0, 2))   # stored per v: [v][R, w]
    GuQ = np.einsum("juq,qQ->juQ", G, X)             # G_uQ(tau) = sum_q G_uq X_qQ
    GQv = np.einsum("sQ,jsv->jQv", X, Gb)            # G_Qv(-tau) read as sum_s X_sQ G_sv(beta-tau)
    GwP = GuQ                                        # G_wP(tau) = sum_p G_wp X_pP
    GQu = np.ascontiguousarray(GuQ.transpose(0, 2, 1))
    D = np.zeros((nt, N, N))
    for v in range(n):
        GG = GQu * GQv[:, :, v][:, :, None]                         # GG_Quv(tau) [nt, Q, u]
        GGm = matsubara(T_fwd, GG)                                  # [n_omega, Q, u]
        Am = np.matmul(Wm, GGm)                                     # A_Puv(Omega)
        A = imag_time(T_bwd, Am)                                    # A_Puv(tau) [nt, P, u]
        B_v = np.matmul(A, X)                                       # B_PRv(tau) [nt, P, R]
        C_v = np.matmul(U2v[v], GwP)                                # C_RvP(tau) [nt, R, P]
        D += C_v.transpose(0, 2, 1) * B_v
    out = np.empty((nt, n, n))
    for j in range(nt):
        out[j] = X @ (-D[j].T) @ X.T
    return out


def sigma_dynamic_line2_eri(X: np.ndarray, V: np.ndarray, W_tau: np.ndarray, G: np.ndarray,
                            Gb: np.ndarray, T_fwd: np.ndarray, T_bwd: np.ndarray) -> np.ndarray:
    """eq:sox with U(1) = V instantaneous and U(2) = W_d(tau) time dependent:
    SOX(V, W_d), the other one-dynamic-line term of 2SOSEX (fig:diag).

    With the U(1) vertex pair at tau_r = 0, the U(2) end (t, u) at the
    external time tau and its end (v, w) at tau', the lines are G_uq(tau),
    G_wp(tau') and G_sv(-tau') (read as G(beta - tau'), as for line 1), and
    the U(2) line carries W(tau - tau'):
      Sigma_tr(tau) = - sum (pr|qs)_V G_uq(tau)
                      int_0^beta (tu|vw)_W(tau - s) G_wp(s) G_sv(beta - s) ds,
    the convolution now on the G_wp G_sv pair, evaluated with the same
    transform pair as sigma_dynamic_eri.  Written independently of the
    line-1 form; for a symmetric G it is that form's mirror image
    (tests/test_oracle_vertex.py)."""
    nt, n, _ = G.shape
    E1 = eri(X, V)
    E2w = np.stack([eri(X, W_tau[j]) for j in range(nt)])        # [nt, t, u, v, w]
    f = np.einsum("jwp,jsv->jwpsv", G, Gb)                        # [nt, w, p, s, v]
    E2m = matsubara(T_fwd, E2w)
    fm = matsubara(T_fwd, f)
    Km = np.einsum("mtuvw,mwpsv->mtups", E2m, fm)                 # product in frequency
    K = imag_time(T_bwd, Km)                                      # [nt, t, u, p, s]
    out = np.empty((nt, n, n))
    for i in range(nt):
        out[i] = -np.einsum("prqs,uq,tups->tr", E1, G[i], K[i], optimize=True)
    return out


# ---------------------------------------------------------------------------
# Galitskii-Migdal energy of the SOX self-energy (eq:E2b on the tau grid)
# ---------------------------------------------------------------------------
def energy_gm(Sigma: np.ndarray, Gb: np.ndarray, weights: np.ndarray) -> float:
    """E = -1/2 sum_k w_k sum_tr Sigma_tr(tau_k) G_rt(beta - tau_k).

    (1/beta) sum_n Tr[G(i w_n) Sigma(i w_n)] = -int_0^beta Tr[Sigma(tau) G(beta-tau)] dtau,
    with the Galitskii-Migdal one half for the dynamical part.
    """
    tr = np.einsum("ktr,krt->k", Sigma, Gb)
    return float(-0.5 * np.dot(weights, tr.real))


# ---------------------------------------------------------------------------
# direct second-order term (only used by the Pauli-cancellation pin)
# ---------------------------------------------------------------------------
def sigma_direct2_eri(E: np.ndarray, G: np.ndarray, Gb: np.ndarray) -> np.ndarray:
    """Second-order direct (bubble) self-energy with the same conventions:
    Sigma_tr = + sum (pr|qs)(tu|vw) G_up(tau) G_wq(tau) G_sv(beta - tau)
    (one closed fermion loop: the opposite sign to the exchange term)."""
    nt, n, _ = G.shape
    out = np.empty((nt, n, n))
    for k in range(nt):
        out[k] = np.einsum("prqs,tuvw,up,wq,sv->tr", E, E, G[k], G[k], Gb[k], optimize=True)
    return out
