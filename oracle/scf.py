"""A minimal self-consistent Dyson loop on synthetic inputs (oracle; test
infrastructure only).

Section "Definitions": eq:Dyson and eq:G0 with an orthonormal basis (S = I),
the chemical potential updated every iteration for the target number of
electrons, and the energies eq:E1b and eq:E2b.  One spin channel of a
molecule (the same-spin quantities of the SOX chain); the self-energy is

    Sigma[G] = Sigma^HF[gamma] + Sigma^dyn[G](tau),
    Sigma^HF_ij = sum_kl [(ij|kl) gamma_lk - (ik|lj) gamma_kl]     (bare V)
    Sigma^dyn = sum of the selected terms: "gw" the THC-GW direct term with a
                fixed W_d(tau) (a stand-in for the screened interaction,
                which the loop does not rebuild), "sox" SOX(V, V).

One iteration: gamma_pq = -G_qp(beta^-) (G(0^-) = -G(beta^-) for fermions),
Sigma^HF, Sigma^dyn(tau), Sigma^dyn(i nu_n) = T_fwd Sigma^dyn(tau) on the
fermionic IR samples, then for each trial mu
    G(i nu_n) = [(i nu_n + mu) I - h - Sigma^HF - Sigma^dyn(i nu_n)]^-1,
    G(tau) = Re T_bwd G(i nu), N(mu) = -Tr G(beta^-) = -t_beta . Tr G(tau),
bisection on mu until N(mu) = N_target, and G <- (1 - a) G + a G_new.
Converged when max |G_new - G| <= tol.  Energies (one spin channel):
    E_inf = sum_pq (h_pq + Sigma^HF_pq / 2) gamma_pq                  (eq:E1b)
    E_dyn = -1/2 sum_j w_j Tr[Sigma^dyn(tau_j) G(beta - tau_j)]        (eq:E2b)
(the tau form of eq:E2b with the Galitskii-Migdal one half, as for the SOX
energies).  Readings: the printed gamma = -G(tau = 0^-) is taken as the
boundary value of G on [0, beta], gamma_pq = -G_qp(beta^-).
"""
from __future__ import annotations

import numpy as np

from oracle import sox_gw as ogw
from oracle import sox_mol as om


def hf_thc(X, V, gamma):
    """Sigma^HF = J - K on the THC factors: J_ij = sum_P X_iP X_jP (V rho)_P with
    rho_Q = sum_kl X_kQ gamma_lk X_lQ; K_ij = sum_PQ X_iP V_PQ (X^T gamma X)_PQ X_jQ."""
    rho = np.einsum("kQ,lk,lQ->Q", X, gamma, X)
    J = (X * (V @ rho)[None, :]) @ X.T
    K = X @ (V * (X.T @ gamma @ X)) @ X.T
    return J - K


def hf_eri(X, V, gamma):
    """Sigma^HF from the 4-index integrals (brute force)."""
    E = om.eri(X, V)
    return np.einsum("ijkl,lk->ij", E, gamma) - np.einsum("iklj,kl->ij", E, gamma)


def sigma_dyn(terms, X, V, W_tau, G):
    out = np.zeros_like(G)
    if "gw" in terms:
        out += ogw.sigma_gw_thc(X, W_tau, G)
    if "sox" in terms:
        out += om.sigma_static_thc(X, V, V, G, G[::-1])
    return out


def density(G, t_beta):
    """gamma_pq = -G_qp(beta^-) from the tau samples."""
    return -np.einsum("i,iqp->pq", t_beta, G)


def dyson(h_eff, Sig_nu, mu, nu, T_bwd):
    n = h_eff.shape[0]
    Gnu = np.empty(Sig_nu.shape, dtype=complex)
    for m in range(len(nu)):
        Gnu[m] = np.linalg.inv((1j * nu[m] + mu) * np.eye(n) - h_eff - Sig_nu[m])
    return np.einsum("im,mpq->ipq", T_bwd, Gnu).real


def solve_mu(h_eff, Sig_nu, nu, T_bwd, t_beta, n_elec, lo, hi, iters=100):
    """Bisection on N(mu) = -Tr G(beta^-) (increasing in mu)."""
    for _ in range(iters):
        mu = 0.5 * (lo + hi)
        G = dyson(h_eff, Sig_nu, mu, nu, T_bwd)
        N = -np.einsum("i,ipp->", t_beta, G)
        if N < n_elec:
            lo = mu
        else:
            hi = mu
    mu = 0.5 * (lo + hi)
    return mu, dyson(h_eff, Sig_nu, mu, nu, T_bwd)


def scf(X, V, W_tau, h, n_elec, beta, fgrid, weights, terms=("gw",), mix=0.5, tol=1e-9,
        max_iter=100, h_start=None):
    """Run the loop from G0 (eq:G0 with H0 = h_start, default h, at the mu that
    holds n_elec).  fgrid: oracle.ir_grid.ir_fermion output; weights: tau
    quadrature weights."""
    tau, T_fwd, T_bwd, t_beta = fgrid["tau"], fgrid["T_fwd"], fgrid["T_bwd"], fgrid["t_beta"]
    nu = (2 * fgrid["n"] + 1) * np.pi / beta
    n = h.shape[0]
    eps_h = np.linalg.eigvalsh(h)
    span = np.abs(eps_h).max() + 50.0
    zero = np.zeros((len(nu), n, n), dtype=complex)
    mu, G = solve_mu(h if h_start is None else h_start, zero, nu, T_bwd, t_beta, n_elec,
                     -span, span)
    it = 0
    delta = np.inf
    for it in range(1, max_iter + 1):
        gamma = density(G, t_beta)
        shf = hf_thc(X, V, gamma)
        sd = sigma_dyn(terms, X, V, W_tau, G)
        sd_nu = np.einsum("mj,jpq->mpq", T_fwd, sd)
        mu, Gn = solve_mu(h + shf, sd_nu, nu, T_bwd, t_beta, n_elec, mu - span, mu + span)
        delta = np.abs(Gn - G).max()
        G = (1 - mix) * G + mix * Gn
        if delta <= tol:
            break
    gamma = density(G, t_beta)
    shf = hf_thc(X, V, gamma)
    sd = sigma_dyn(terms, X, V, W_tau, G)
    e_inf = float(np.sum((h + 0.5 * shf) * gamma))
    e_dyn = om.energy_gm(sd, G[::-1], weights) if terms else 0.0
    return dict(G=G, mu=mu, gamma=gamma, sigma_hf=shf, sigma_dyn=sd, e_inf=e_inf,
                e_dyn=float(e_dyn), iterations=it, delta=float(delta))
