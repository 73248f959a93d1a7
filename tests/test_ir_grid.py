"""The library's IR grid (sox_ir_grid, host code in libsox.so) against the
closed forms and the oracle (oracle/ir_grid.py), no GPU needed.

* The closed-form pins of the oracle, applied to the library's grid: bosonic
  one-sided and periodic poles through T_fwd and T_bwd, and the quadrature
  weights, at 100 eps (measured about 10 eps, as for the oracle), including
  the paper's Lambda = 1e6 at beta = 1000 (the oracle's dense Matsubara scan
  takes minutes there, so that case is pinned by the closed forms alone).
* Parity with the oracle: the same basis size, the same Matsubara indices
  (exactly), and tau nodes, weights and transform pair within
  1e-14 / eps relative.  The two codings reach the singular functions by
  different routes (LAPACK's divide and conquer, one-sided Jacobi
  rotations), which agree on a function of singular value s_l to about
  eps_mach s_0 / s_l; the sampling points come from the first omitted
  function, s_L < eps s_0 (measured: 1.5e-6 at eps = 1e-10, 6e-9 at 1e-8).
* Argument checks and the capacity protocol.
"""
import numpy as np
import pytest

from oracle import ir_grid as ir


@pytest.fixture(scope="module")
def B():
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


def _pole(w, tau, beta):
    if w > 0:
        return np.exp(-w * tau) / (-np.expm1(-w * beta))
    return -np.exp(-w * (tau - beta)) / (-np.expm1(w * beta))


def _pole_errors(g, beta, lam):
    tau, Om = g["tau"], 2 * np.pi * g["m"] / beta
    wf = wb = wq = 0.0
    for w in (lam / beta) * np.array([-1.0, -0.37, -0.01, 0.003, 0.05, 0.4, 1.0]):
        f = _pole(w, tau, beta)
        fh = -1.0 / (1j * Om - w)
        wf = max(wf, np.abs(g["T_fwd"] @ f - fh).max() / np.abs(fh).max())
        wb = max(wb, np.abs((g["T_bwd"] @ fh).real - f).max() / np.abs(f).max())
        wq = max(wq, abs(np.dot(g["weights"], f) - 1.0 / w) * abs(w))
    for w in (lam / beta) * np.array([0.01, 0.2, 1.0]):
        f = (np.exp(-w * tau) + np.exp(-w * (beta - tau))) / (-np.expm1(-w * beta))
        fh = 2 * w / (w * w + Om * Om)
        wf = max(wf, np.abs(g["T_fwd"] @ f - fh).max() / np.abs(fh).max())
        wb = max(wb, np.abs((g["T_bwd"] @ fh).real - f).max() / np.abs(f).max())
    return wf, wb, wq


@pytest.mark.parametrize("beta,lam,eps", [(1000.0, 1e4, 1e-10), (100.0, 1400.0, 1e-10),
                                          (50.0, 500.0, 1e-8), (1000.0, 1e6, 1e-10),
                                          (1000.0, 1e4, 1e-12)])
def test_library_grid_closed_forms(B, beta, lam, eps):
    g = B.sox_ir_grid(beta, lam, eps)
    tau = g["tau"]
    assert np.all(np.diff(tau) > 0) and tau[0] > 0 and tau[-1] < beta
    assert np.abs(tau + tau[::-1] - beta).max() <= 1e-12 * beta
    wf, wb, wq = _pole_errors(g, beta, lam)
    assert wf <= 1e2 * eps and wb <= 1e2 * eps and wq <= 1e2 * eps, (wf, wb, wq)


@pytest.mark.parametrize("beta,lam,eps", [(1000.0, 1e4, 1e-10), (100.0, 1400.0, 1e-10),
                                          (50.0, 500.0, 1e-8)])
def test_library_grid_matches_oracle(B, beta, lam, eps):
    g = B.sox_ir_grid(beta, lam, eps)
    o = ir.ir_grid(beta, lam, eps)
    assert len(g["tau"]) == o["L"]
    assert np.array_equal(g["m"], o["m"])
    tol = 1e-14 / eps
    assert np.abs(g["tau"] - o["tau"]).max() <= tol * beta
    assert np.abs(g["s"] - o["s"]).max() <= 1e-12
    for key in ("weights", "T_fwd", "T_bwd"):
        err = np.abs(g[key] - o[key]).max() / np.abs(o[key]).max()
        assert err <= tol, (key, err)


def test_argument_checks_and_capacity(B):
    with pytest.raises(B.SoxError) as e:
        B.sox_ir_grid(100.0, 1000.0, 1e-14)
    assert e.value.status == 1
    with pytest.raises(B.SoxError) as e:
        B.sox_ir_grid(-1.0, 1000.0, 1e-8)
    assert e.value.status == 1
    with pytest.raises(B.SoxError) as e:
        B.sox_ir_grid(100.0, 1000.0, 1e-8, capacity=10)
    assert e.value.status == 2
    g = B.sox_ir_grid(100.0, 1000.0, 1e-8, capacity=64)
    assert len(g["tau"]) <= 64 and len(g["m"]) <= 64


@pytest.mark.parametrize("beta,lam,eps", [(20.0, 300.0, 1e-10), (100.0, 1400.0, 1e-10)])
def test_library_fermionic_pair(B, beta, lam, eps):
    """The fermionic pair: closed-form fermionic poles (f(i nu) = 1 / (i nu - e),
    f(beta^-) = -1 / (1 + e^{beta e})) and parity with the oracle's pair."""
    g = B.sox_ir_grid_fermion(beta, lam, eps)
    o = ir.ir_fermion(beta, lam, eps)
    assert np.array_equal(g["n"], o["n"])
    tol = 1e-14 / eps
    assert np.abs(g["tau"] - o["tau"]).max() <= tol * beta
    for key in ("T_fwd", "T_bwd", "t_beta"):
        err = np.abs(g[key] - o[key]).max() / np.abs(o[key]).max()
        assert err <= tol, (key, err)
    tau, nu = g["tau"], (2 * g["n"] + 1) * np.pi / beta
    for e in (lam / beta) * np.array([-1.0, -0.2, 0.01, 0.5, 1.0]):
        if e > 0:
            ft = -np.exp(-e * tau) / (1 + np.exp(-beta * e))
            fb = -np.exp(-e * beta) / (1 + np.exp(-beta * e))
        else:
            ft = -np.exp(-e * (tau - beta)) / (np.exp(beta * e) + 1)
            fb = -1.0 / (np.exp(beta * e) + 1)
        fh = 1.0 / (1j * nu - e)
        assert np.abs(g["T_fwd"] @ ft - fh).max() <= 1e2 * eps * np.abs(fh).max()
        assert np.abs((g["T_bwd"] @ fh).real - ft).max() <= 1e2 * eps * np.abs(ft).max()
        assert abs(g["t_beta"] @ ft - fb) <= 1e2 * eps
