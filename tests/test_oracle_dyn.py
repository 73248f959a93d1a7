"""Pins of the dynamic-interaction oracle (PN9) and of the transform pair.

  PN9(i)   the paper's dynamic THC chain (eq:GG, FT, W(Omega) GG(Omega), IFT,
           B, C, D, Sigma) equals the 4-index brute force with the same
           transform pair, to rounding
  PN9(ii)  for G0 and a single bosonic pole W(tau) = a pole_w(tau) S, the
           oracle equals the continuum self-energy, whose frequency integral is
           done in closed form in the MO basis (the transform pair only
           approximates the continuum, so the bound is its accuracy)
  transform pair: the Matsubara transform of the periodic pole matches its
           closed form 2 w / (w^2 + Omega^2); convolution of a pole with an
           exponential matches adaptive quadrature.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import sox_mol as om
from paper_2412_18829_amd import synth


def _pair(tau, beta, omega_max=8.0):
    return synth.bosonic_transform_pair(tau, beta, omega_max=omega_max, tol=1e-10)


def test_transform_of_periodic_pole_closed_form():
    beta = 20.0
    tau, _ = synth.chebyshev_tau_grid(48, beta)
    tp = _pair(tau, beta)
    for w in (0.2, 1.0, 5.0):
        f = synth.periodic_bosonic_pole(tau, beta, w)
        fm = tp["T_fwd"] @ f
        exact = 2.0 * w / (w * w + tp["Omega"] ** 2)
        assert np.abs(fm - exact).max() <= 1e-6 * exact.max()
        # round trip
        back = (tp["T_bwd"] @ fm).real
        assert np.abs(back - f).max() <= 1e-6 * np.abs(f).max()


def _pole_exp_conv(tau, beta, w, d):
    """int_0^beta pole_w(tau - s) e^{-d s} ds for the beta-periodic pole."""
    c = 1.0 / (-np.expm1(-w * beta))
    t = np.asarray(tau)

    def ratio(num, den):
        return num / den

    if abs(w - d) < 1e-12 or abs(w + d) < 1e-12:
        raise ValueError("degenerate exponent")
    a = (np.exp(-d * t) - np.exp(-w * t) + np.exp(-w * t - d * beta) - np.exp(-w * beta - d * t))
    b = (np.exp(-w * (beta - t)) - np.exp(-w * beta - d * t) + np.exp(-d * t)
         - np.exp(-w * (beta - t) - d * beta))
    return c * (ratio(a, w - d) + ratio(b, w + d))


def test_pole_exponential_convolution_closed_form_vs_quadrature():
    beta = 10.0
    tau = np.array([0.05, 1.0, 4.3, 9.9])
    for w, d in [(0.7, 1.3), (2.0, -0.8), (5.0, 0.4)]:
        cf = _pole_exp_conv(tau, beta, w, d)
        for i, t in enumerate(tau):
            f = lambda s: synth.periodic_bosonic_pole(np.array([(t - s) % beta]), beta, w)[0] * np.exp(-d * s)
            q = quad(f, 0, t, epsabs=0, epsrel=1e-13, limit=200)[0] + \
                quad(f, t, beta, epsabs=0, epsrel=1e-13, limit=200)[0]
            assert abs(q - cf[i]) <= 1e-11 * abs(q)


def test_pn9i_dynamic_chain_equals_brute_force():
    wl = synth.small_molecule(5, 12, 24, 20.0, seed=11, dynamic=True)
    tp = _pair(wl["tau"], wl["beta"], omega_max=14.0)
    G, _ = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]), None
    G = G + 0.05 * np.random.default_rng(1).standard_normal(G.shape)
    Gb = G[::-1]
    a = om.sigma_dynamic_eri(wl["X"], wl["W_tau"], wl["V"], G, Gb, tp["T_fwd"], tp["T_bwd"])
    b = om.sigma_dynamic_thc(wl["X"], wl["W_tau"], wl["V"], G, Gb, tp["T_fwd"], tp["T_bwd"])
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


def test_pn9ii_continuum_single_pole_mo_basis():
    n, N, beta, nt = 4, 9, 10.0, 64
    rng = synth.rng_for(91)
    eps = np.array([-0.9, -0.3, 0.4, 1.1])
    Q = synth.haar_orthogonal(rng, n)
    X = rng.standard_normal((n, N)) / np.sqrt(n)
    V = synth.random_spd(rng, N, 1.0 / N)
    S = synth.random_spd(rng, N, 1.0 / N)
    a, w = 0.07, 1.7
    tau, _ = synth.chebyshev_tau_grid(nt, beta)
    W_tau = a * synth.periodic_bosonic_pole(tau, beta, w)[:, None, None] * S[None]
    tp = _pair(tau, beta, omega_max=8.0)
    G = om.g_tau(eps, Q, 0.0, beta, tau)
    got = om.sigma_dynamic_thc(X, W_tau, V, G, om.g_mirror(G), tp["T_fwd"], tp["T_bwd"])

    # continuum, MO basis: G_pq = delta g_p, g = -e^{-e tau} h, gbar = -e^{e tau} f
    f = 1.0 / (1.0 + np.exp(beta * eps))
    h = 1.0 - f
    Xm = Q.T @ X
    EV = om.eri(Xm, V)          # (tq|sp)_V as EV[t,q,s,p]
    ES = om.eri(Xm, S)          # (pr|qs)_S as ES[p,r,q,s]
    conv = np.empty((nt, n, n))  # [tau, q, s]
    for q in range(n):
        for s in range(n):
            conv[:, q, s] = a * h[q] * f[s] * _pole_exp_conv(tau, beta, w, eps[q] - eps[s])
    gp = -np.exp(-np.outer(tau, eps)) * h[None, :]
    ref_mo = -np.einsum("tqsp,kp,prqs,kqs->ktr", EV, gp, ES, conv)
    ref = np.einsum("ta,kab,rb->ktr", Q, ref_mo, Q)
    assert np.abs(got - ref).max() <= 2e-6 * np.abs(ref).max()
