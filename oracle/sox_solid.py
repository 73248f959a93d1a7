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


def sigma_solid_thc(X, U1, U2, G, tables, v_subset=None) -> np.ndarray:
    """The paper's k-point step chain.

    U^{q1,k_v}_Pqs = sum_Q U1^{q1}_PQ conj(X^{k_v-q1}_qQ) X^{k_v}_sQ    (eq:U_contraction)
    G^k_Rq = sum_u X^k_uR G^k_uq,  G^k_wP = sum_p G^k_wp conj(X^k_pP)
    A^{q1,k_v}_Pqv = sum_s U^{q1,k_v}_Pqs G^{k_v}_sv(beta - tau)
    B^{q1,k_v}_PRv = sum_q A^{q1,k_v}_Pqv G^{k_v-q1}_Rq
    C^{q2,k_w}_RvP = sum_w U(2)^{q2,k_w}_Rvw G^{k_w}_wP
    D^{k_t}_PR = (1/N_k) sum_{k_w, q2} sum_v C^{q2,k_w}_RvP B^{q1,k_w-q2}_PRv,  q1 = k_w - k_t
    Sigma^{k_t}_RP = -(1/N_k) D^{k_t}_PR;  Sigma^{k_t}_tr = sum_PR conj(X^{k_t}_tR) Sigma_RP X^{k_t}_rP

    v_subset (optional): only the orbitals v listed contribute to D (the
    chain's innermost orbital sum); Sigma is linear in the per-v terms, so
    the results of disjoint subsets add up to the full Sigma.
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
    vs = np.arange(n) if v_subset is None else np.asarray(v_subset, dtype=int)
    out = np.empty((nk, nt, n, n), dtype=complex)
    for k in range(nt):
        GRq = [X[kk].T @ G[kk, k] for kk in range(nk)]             # G^k_Rq
        GwP = [G[kk, k] @ X[kk].conj() for kk in range(nk)]        # G^k_wP
        B = {}
        for q1 in range(nk):
            for kv in range(nk):
                A = np.tensordot(U1t[(q1, kv)], Gb[kv, k][:, vs], axes=(2, 0))   # A_Pqv
                kq = kdiff[kv, q1]
                B[(q1, kv)] = np.einsum("Pqv,Rq->PRv", A, GRq[kq])
        C = {}
        for q2 in range(nk):
            for kw in range(nk):
                C[(q2, kw)] = np.einsum("Rvw,wP->RvP", U2t[(q2, kw)][:, vs], GwP[kw])
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


# ---------------------------------------------------------------------------
# dynamic interaction on line 1 (eq:GG scheme for solids)
# ---------------------------------------------------------------------------
# The plan's transform pair acts on functions that are real in imaginary
# time: f(i Omega_m) = sum_j T_fwd[m, j] f(tau_j) for m >= 0 and
# f(tau_i) = Re sum_m T_bwd[i, m] f(i Omega_m).  Momentum-resolved functions
# are complex; their transforms are taken at +Omega_m with T_fwd and at
# -Omega_m with conj(T_fwd), and the inverse transform is
# f(tau_i) = 1/2 sum_m [T_bwd[i, m] f(i Omega_m) + conj(T_bwd[i, m]) f(-i Omega_m)],
# which is the bilinear extension of the real-function pair (it returns
# Re T_bwd T_fwd f for real f), so a periodic convolution becomes a product
# at every signed frequency.

def matsubara_pm(T_fwd: np.ndarray, f: np.ndarray):
    """(f(+i Omega), f(-i Omega)) along axis 0."""
    return np.tensordot(T_fwd, f, axes=(1, 0)), np.tensordot(T_fwd.conj(), f, axes=(1, 0))


def imag_time_pm(T_bwd: np.ndarray, fp: np.ndarray, fm: np.ndarray) -> np.ndarray:
    """f(tau) from its transforms at +Omega and -Omega (axis 0)."""
    return 0.5 * (np.tensordot(T_bwd, fp, axes=(1, 0)) + np.tensordot(T_bwd.conj(), fm, axes=(1, 0)))


def sigma_solid_dynamic_eri(X, W, V, G, T_fwd, T_bwd, tables) -> np.ndarray:
    """4-index brute force of eq:sox with U(1) = W^q(tau) and U(2) = V^q.

    W [n_k, n_tau, N, N] (W^q(tau_j)).  As for molecules, the U(1) line
    couples G_uq(s) G_sv(beta - s) to the external time through the periodic
    convolution K(tau) = int_0^beta (pr|qs)_W(tau - s) G_uq(s) G_sv(beta - s) ds,
    here evaluated with the signed-frequency pair above."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    Gb = G[:, ::-1]
    out = np.zeros((nk, nt, n, n), dtype=complex)
    for kt in range(nk):
        for kp in range(nk):
            for kq in range(nk):
                kss = kdiff[ksum[kp, kq], kt]
                E2 = eri_k(X, V, kt, kq, kss, kp, kdiff)                     # (t kt, u kq | v ks, w kp)
                E1w = np.stack([eri_k(X, W[:, j], kp, kt, kq, kss, kdiff) for j in range(nt)])
                f = np.einsum("juq,jsv->juqsv", G[kq], Gb[kss])
                Ep, Em = matsubara_pm(T_fwd, E1w)
                fp, fm = matsubara_pm(T_fwd, f)
                K = imag_time_pm(T_bwd, np.einsum("mprqs,muqsv->mpruv", Ep, fp),
                                 np.einsum("mprqs,muqsv->mpruv", Em, fm))
                for i in range(nt):
                    out[kt, i] -= np.einsum("tuvw,wp,pruv->tr", E2, G[kp, i], K[i], optimize=True)
    return out / nk ** 2


def sigma_solid_dynamic_line2_eri(X, V, W, G, T_fwd, T_bwd, tables) -> np.ndarray:
    """4-index brute force of eq:sox with U(1) = V^q and U(2) = W^q(tau):
    SOX(V, W_d) on a k-point mesh.  As for molecules (sox_mol's line-2 form)
    the convolution sits on the G_wp G_sv pair and G_uq keeps the external
    time:
      Sigma^{k_t}_tr(tau) = -(1/N_k^2) sum_{k_p,k_q} (p k_p, r k_t | q k_q, s k_s)_V G^{k_q}_uq(tau)
          int (t k_t, u k_q | v k_s, w k_p)_W(tau - s) G^{k_p}_wp(s) G^{k_s}_sv(beta - s) ds,
    with the signed-frequency transforms of complex functions."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    Gb = G[:, ::-1]
    out = np.zeros((nk, nt, n, n), dtype=complex)
    for kt in range(nk):
        for kp in range(nk):
            for kq in range(nk):
                kss = kdiff[ksum[kp, kq], kt]
                E1 = eri_k(X, V, kp, kt, kq, kss, kdiff)                     # (p kp, r kt | q kq, s ks)
                E2w = np.stack([eri_k(X, W[:, j], kt, kq, kss, kp, kdiff) for j in range(nt)])
                f = np.einsum("jwp,jsv->jwpsv", G[kp], Gb[kss])
                Ep, Em = matsubara_pm(T_fwd, E2w)
                fp, fm = matsubara_pm(T_fwd, f)
                K = imag_time_pm(T_bwd, np.einsum("mtuvw,mwpsv->mtups", Ep, fp),
                                 np.einsum("mtuvw,mwpsv->mtups", Em, fm))
                for i in range(nt):
                    out[kt, i] -= np.einsum("prqs,uq,tups->tr", E1, G[kq, i], K[i], optimize=True)
    return out / nk ** 2


def sigma_solid_dynamic_thc(X, W, V, G, T_fwd, T_bwd, tables, v_subset=None) -> np.ndarray:
    """The paper's momentum-resolved eq:GG chain with v outermost.

    v_subset (optional): run the outer orbital loop over the listed v only
    (Sigma is linear in the per-v contributions to D).

    GG^{q1,k_v}_Quv(tau) = G^{k_v-q1}_uQ(tau) G^{k_v}_Qv(-tau) with
    G^k_uQ = sum_q G^k_uq conj(X^k_qQ) and G^k_Qv(-tau) read as
    sum_s X^k_sQ G^k_sv(beta - tau); A = W^{q1} * GG (periodic convolution as
    a product at +-Omega); B^{q1,k_v}_PRv = sum_u X^{k_v-q1}_uR A_Puv;
    C, D and Sigma as for static interactions."""
    ks_list, kdiff, ksum, kneg = tables
    nk, nt, n, _ = G.shape
    N = X.shape[2]
    Gb = G[:, ::-1]
    Wp = [np.tensordot(T_fwd, W[q], axes=(1, 0)) for q in range(nk)]
    Wm = [np.tensordot(T_fwd.conj(), W[q], axes=(1, 0)) for q in range(nk)]
    GwP = [np.einsum("jwp,pP->jwP", G[k], X[k].conj()) for k in range(nk)]        # [nt, w, P]
    GQv = [np.einsum("sQ,jsv->jQv", X[k], Gb[k]) for k in range(nk)]              # [nt, Q, v]

    def utensor(U, q, kv):
        kq = kdiff[kv, q]
        return np.einsum("PQ,qQ,sQ->Pqs", U[q], X[kq].conj(), X[kv], optimize=True)

    U2t = {(q, k): utensor(V, q, k) for q in range(nk) for k in range(nk)}
    D = np.zeros((nk, nt, N, N), dtype=complex)
    for v in (range(n) if v_subset is None else v_subset):
        B = {}
        for q1 in range(nk):
            for kv in range(nk):
                kq = kdiff[kv, q1]
                GG = GwP[kq].transpose(0, 2, 1) * GQv[kv][:, :, v][:, :, None]   # [nt, Q, u]
                GGp, GGm = matsubara_pm(T_fwd, GG)
                A = imag_time_pm(T_bwd, np.matmul(Wp[q1], GGp), np.matmul(Wm[q1], GGm))   # [nt, P, u]
                B[(q1, kv)] = np.matmul(A, X[kq])                                  # [nt, P, R]
        C = {}
        for q2 in range(nk):
            for kw in range(nk):
                C[(q2, kw)] = np.matmul(U2t[(q2, kw)][:, v, :], GwP[kw])          # [nt, R, P]
        for kt in range(nk):
            for kw in range(nk):
                q1 = kdiff[kw, kt]
                for q2 in range(nk):
                    kv = kdiff[kw, q2]
                    D[kt] += C[(q2, kw)].transpose(0, 2, 1) * B[(q1, kv)] / nk
    out = np.empty((nk, nt, n, n), dtype=complex)
    for kt in range(nk):
        for j in range(nt):
            out[kt, j] = X[kt].conj() @ (-D[kt, j].T / nk) @ X[kt].T
    return out
