"""Pins of the minimal self-consistent loop (oracle/scf.py) and the fermionic
IR pair it runs on (oracle/ir_grid.ir_fermion).

* Fermionic poles: f(tau) = -e^{-e tau} / (1 + e^{-beta e}) has f(i nu_n) =
  1 / (i nu_n - e) and f(beta^-) = -1 / (1 + e^{beta e}); T_fwd, T_bwd and
  t_beta reproduce them at about 10 eps.
* Sigma^HF on the THC factors equals the 4-index brute force (Hartree minus
  exchange) on a general (non-symmetric) density matrix.
* Non-interacting limit (V = 0, no dynamic term): the loop returns eq:G_def
  for the one-body h at the chemical potential of the Fermi function that
  holds N electrons (found by a scalar root search), and E_inf = sum_a e_a f_a.
* Hartree-Fock fixed point (no dynamic term): the converged G equals eq:G_def
  for F = h + Sigma^HF[gamma] at the converged mu, and Tr gamma = N.
* With the GW term: the converged solution does not depend on the starting
  point (the property of fully self-consistent solutions the paper states),
  and Tr gamma = N.
Convergence floor: with the chemical potential in a gap, N(mu) is flat
(dN/dmu ~ beta e^{-beta gap / 2}), so rounding in N moves mu by up to about
1e-6 without changing G beyond 1e-9; the loops stop at max |dG| <= 1e-8 and
the fixed-point comparisons use 1e-7.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import ir_grid as ir
from oracle import scf as osc
from oracle import sox_mol as om
from paper_2412_18829_amd import synth

BETA, LAM, EPS = 20.0, 300.0, 1e-10


@pytest.fixture(scope="module")
def grids():
    return ir.ir_fermion(BETA, LAM, EPS), ir.ir_grid(BETA, LAM, EPS)


def _system(n, N, seed, dyn=True):
    wl = synth.small_molecule(n, N, 8, BETA, seed=seed)
    h = wl["Q"] @ np.diag(wl["eps"]) @ wl["Q"].T
    return wl, h


def test_fermionic_poles(grids):
    f, _ = grids
    tau, nu = f["tau"], (2 * f["n"] + 1) * np.pi / BETA
    for e in (LAM / BETA) * np.array([-1.0, -0.2, -0.01, 0.03, 0.6, 1.0]):
        if e > 0:
            ft = -np.exp(-e * tau) / (1 + np.exp(-BETA * e))
            fb = -np.exp(-e * BETA) / (1 + np.exp(-BETA * e))
        else:
            ft = -np.exp(-e * (tau - BETA)) / (np.exp(BETA * e) + 1)
            fb = -1.0 / (np.exp(BETA * e) + 1)
        fh = 1.0 / (1j * nu - e)
        assert np.abs(f["T_fwd"] @ ft - fh).max() <= 1e2 * EPS * np.abs(fh).max()
        assert np.abs((f["T_bwd"] @ fh).real - ft).max() <= 1e2 * EPS * np.abs(ft).max()
        assert abs(f["t_beta"] @ ft - fb) <= 1e2 * EPS


def test_hf_thc_equals_bruteforce():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((5, 9))
    V = rng.standard_normal((9, 9))
    V = V + V.T
    gamma = rng.standard_normal((5, 5))
    a = osc.hf_thc(X, V, gamma)
    b = osc.hf_eri(X, V, gamma)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_noninteracting_limit(grids):
    f, b = grids
    wl, h = _system(6, 14, seed=11)
    n_elec = 3.0
    out = osc.scf(wl["X"], 0.0 * wl["V"], None, h, n_elec, BETA, f, b["weights"], terms=())
    e = wl["eps"]
    mu = brentq(lambda m: np.sum(1 / (1 + np.exp(BETA * (e - m)))) - n_elec, -20, 20, xtol=1e-14)
    assert abs(out["mu"] - mu) <= 1e-8
    G = om.g_tau(e, wl["Q"], mu, BETA, f["tau"])
    assert np.abs(out["G"] - G).max() <= 1e-8
    fa = 1 / (1 + np.exp(BETA * (e - mu)))
    assert abs(out["e_inf"] - np.sum(e * fa)) <= 1e-8
    assert abs(np.trace(out["gamma"]) - n_elec) <= 1e-8


def test_hartree_fock_fixed_point(grids):
    f, b = grids
    wl, h = _system(6, 14, seed=12)
    n_elec = 3.0
    out = osc.scf(wl["X"], 3.0 * wl["V"], None, h, n_elec, BETA, f, b["weights"], terms=(),
                  tol=1e-8, max_iter=300)
    assert out["delta"] <= 1e-8
    F = h + osc.hf_thc(wl["X"], 3.0 * wl["V"], out["gamma"])
    ev, Q = np.linalg.eigh(0.5 * (F + F.T))
    G = om.g_tau(ev, Q, out["mu"], BETA, f["tau"])
    assert np.abs(out["G"] - G).max() <= 1e-7
    assert abs(np.trace(out["gamma"]) - n_elec) <= 1e-8


def test_gw_loop_independent_of_start(grids):
    f, b = grids
    wl, h = _system(6, 14, seed=13)
    wl["tau"] = f["tau"]
    synth.add_dynamic_screening(wl)
    n_elec = 3.0
    kw = dict(terms=("gw",), tol=1e-8, max_iter=300)
    a = osc.scf(wl["X"], wl["V"], wl["W_tau"], h, n_elec, BETA, f, b["weights"], **kw)
    rng = np.random.default_rng(5)
    P = rng.standard_normal(h.shape) * 0.3
    c = osc.scf(wl["X"], wl["V"], wl["W_tau"], h, n_elec, BETA, f, b["weights"],
                h_start=h + P + P.T, **kw)
    assert a["delta"] <= 1e-8 and c["delta"] <= 1e-8
    assert np.abs(a["G"] - c["G"]).max() <= 1e-7
    assert abs(a["mu"] - c["mu"]) <= 1e-5
    assert abs(np.trace(a["gamma"]) - n_elec) <= 1e-8
    assert abs(a["e_dyn"] - c["e_dyn"]) <= 1e-6 * abs(a["e_dyn"])
