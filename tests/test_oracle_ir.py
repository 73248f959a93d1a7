"""Pins of the in-house IR grid (oracle/ir_grid.py).

* Closed-form Matsubara transforms: a bosonic one-sided pole
  f(tau) = e^{-w tau} / (1 - e^{-w beta}) has f(i Omega_m) = -1 / (i Omega_m - w)
  for any real w; the beta-periodic two-sided pole has 2w / (w^2 + Omega^2).
  T_fwd must reproduce them from the tau samples and T_bwd must return the
  samples from them, for |w| up to omega_max = Lambda / beta, at the level
  of eps times the sampling matrices' conditioning (a wrong frequency sign,
  a lost factor sqrt(2 / beta), a wrong parity or a mis-chosen real part
  each fail it).
* The quadrature weights integrate those poles: int_0^beta f = 1 / w.
* Singular-value-expansion theory: u_l has exactly l roots in (-1, 1), and
  the u_l are orthonormal on [-1, 1] (checked by an independent fine
  composite quadrature of the per-segment Legendre series).
* The per-segment spherical-Bessel Matsubara formula equals a direct fine
  quadrature of e^{i Omega tau} U_l(tau) at small m.
* The sampling times are ascending, mirror symmetric, inside (0, beta); the
  basis grows with Lambda and with smaller eps.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import ir_grid as ir


def _pole(w, tau, beta):
    # e^{-w tau} / (1 - e^{-w beta}), written without overflow for either sign of w
    if w > 0:
        return np.exp(-w * tau) / (-np.expm1(-w * beta))
    return -np.exp(-w * (tau - beta)) / (-np.expm1(w * beta))


GRIDS = [(1000.0, 1e4, 1e-10), (100.0, 1400.0, 1e-10), (50.0, 500.0, 1e-8)]


@pytest.fixture(scope="module", params=GRIDS, ids=lambda g: f"beta{g[0]:g}-L{g[1]:g}-eps{g[2]:g}")
def grid(request):
    beta, lam, eps = request.param
    return beta, lam, eps, ir.ir_grid(beta, lam, eps)


def test_tau_nodes_mirror_symmetric(grid):
    beta, lam, eps, g = grid
    tau = g["tau"]
    assert len(tau) == g["L"]
    assert np.all(np.diff(tau) > 0) and tau[0] > 0 and tau[-1] < beta
    assert np.abs(tau + tau[::-1] - beta).max() <= 1e-10 * beta


def test_pole_transforms(grid):
    beta, lam, eps, g = grid
    tau, Om = g["tau"], 2 * np.pi * g["m"] / beta
    wmax = lam / beta
    worst_f = worst_b = 0.0
    for w in wmax * np.array([-1.0, -0.37, -0.01, 0.003, 0.05, 0.4, 1.0]):
        f = _pole(w, tau, beta)
        fh = -1.0 / (1j * Om - w)
        worst_f = max(worst_f, np.abs(g["T_fwd"] @ f - fh).max() / np.abs(fh).max())
        worst_b = max(worst_b, np.abs((g["T_bwd"] @ fh).real - f).max() / np.abs(f).max())
    for w in wmax * np.array([0.01, 0.2, 1.0]):
        f = (np.exp(-w * tau) + np.exp(-w * (beta - tau))) / (-np.expm1(-w * beta))
        fh = 2 * w / (w * w + Om * Om)
        worst_f = max(worst_f, np.abs(g["T_fwd"] @ f - fh).max() / np.abs(fh).max())
        worst_b = max(worst_b, np.abs((g["T_bwd"] @ fh).real - f).max() / np.abs(f).max())
    tol = 1e2 * eps   # measured about 10 eps (the sampling matrices' conditioning)
    assert worst_f <= tol and worst_b <= tol, (worst_f, worst_b)


def test_weights_integrate_poles(grid):
    beta, lam, eps, g = grid
    for w in (lam / beta) * np.array([-0.5, 0.01, 0.3, 1.0]):
        got = np.dot(g["weights"], _pole(w, g["tau"], beta))
        assert abs(got - 1.0 / w) <= 1e2 * eps * abs(1.0 / w)


def test_singular_functions_roots_and_orthonormality():
    lam = 1000.0
    fs, bx, x, wx = ir.sve(lam)
    t, w = leggauss(48)
    xs = np.concatenate([(a + b) / 2 + (b - a) / 2 * t for a, b in zip(bx[:-1], bx[1:])])
    ws = np.concatenate([(b - a) / 2 * w for a, b in zip(bx[:-1], bx[1:])])
    xs = np.concatenate([-xs[::-1], xs])
    ws = np.concatenate([ws[::-1], ws])
    ls = [0, 1, 2, 5, 10, 17, 30, 41]
    vals = {}
    for l in ls:
        c = ir.legendre_coeffs(fs[l][2])
        assert len(ir.roots(c, fs[l][1], bx)) == l
        vals[l] = ir.evaluate(c, fs[l][1], bx, xs)
    for a in ls:
        for b in ls:
            ip = np.sum(ws * vals[a] * vals[b])
            assert abs(ip - (1.0 if a == b else 0.0)) <= 1e-10


def test_matsubara_formula_vs_quadrature():
    beta, lam = 20.0, 200.0
    fs, bx, x, wx = ir.sve(lam)
    t, w = leggauss(64)
    xs = np.concatenate([(a + b) / 2 + (b - a) / 2 * t for a, b in zip(bx[:-1], bx[1:])])
    ws = np.concatenate([(b - a) / 2 * w for a, b in zip(bx[:-1], bx[1:])])
    xs = np.concatenate([-xs[::-1], xs])
    ws = np.concatenate([ws[::-1], ws])
    ms = np.arange(0, 6)
    for l in (0, 1, 4, 7):
        c = ir.legendre_coeffs(fs[l][2])
        got = ir.matsubara(c, fs[l][1], bx, beta, ms)
        u = ir.evaluate(c, fs[l][1], bx, xs)
        want = np.array([np.sqrt(beta / 2) * np.sum(ws * np.exp(1j * np.pi * m * (xs + 1)) * u)
                         for m in ms])
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_basis_grows_with_lambda_and_precision():
    sizes = {}
    for lam in (100.0, 1000.0, 1e4):
        fs, *_ = ir.sve(lam)
        s = np.array([f[0] for f in fs])
        sizes[lam] = [int(np.sum(s >= e * s[0])) for e in (1e-6, 1e-10)]
    assert sizes[100.0][0] < sizes[1000.0][0] < sizes[1e4][0]
    for lam in sizes:
        assert sizes[lam][0] < sizes[lam][1]
