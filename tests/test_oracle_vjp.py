"""Pins of the reference VJP (PN10): torch autograd through the step chain
against central finite differences of the independent numpy 4-index brute
force, along random directions in every input; plus the Phi-derivability
identity rewritten as a VJP (for U1 = U2 and R = w_k G(beta - tau_k)^T the
G-gradient is 4 w Sigma(beta - tau)^T... checked through F[G])."""
import numpy as np
import pytest

from oracle import sox_mol as om
from oracle import sox_vjp as ov
from paper_2412_18829_amd import synth


def _fd(fun, x, d, h=1e-5):
    return (fun(x + h * d) - fun(x - h * d)) / (2 * h)


@pytest.mark.parametrize("bare", [True, False])
def test_static_vjp_matches_fd_of_bruteforce(bare):
    n, N, nt = 4, 9, 8
    wl = synth.small_molecule(n, N, nt, 6.0, seed=21, static=True)
    rng = np.random.default_rng(3)
    X, V = wl["X"], wl["V"]
    U1 = V if bare else wl["W0"]
    U2 = V
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    R = rng.standard_normal((nt, n, n))

    def L(X_, U1_, U2_, G_):
        S = om.sigma_static_eri(om.eri(X_, U1_), om.eri(X_, U2_), G_, G_[::-1])
        return float(np.sum(S * R))

    dG, dX, d1, d2 = ov.vjp_static(X, U1, U2, G, R, bare=bare)
    for trial in range(2):
        DG = rng.standard_normal(G.shape)
        DX = rng.standard_normal(X.shape)
        D1 = rng.standard_normal(U1.shape)
        fd = _fd(lambda e: L(X, U1, U2, G + e), 0.0, DG)
        assert abs(fd - np.sum(dG * DG)) <= 1e-7 * max(1.0, abs(fd))
        fd = _fd(lambda e: L(X + e, U1, U2, G), 0.0, DX)
        assert abs(fd - np.sum(dX * DX)) <= 1e-7 * max(1.0, abs(fd))
        if bare:
            fd = _fd(lambda e: L(X, V + e, V + e, G), 0.0, D1)
            assert abs(fd - np.sum(d1 * D1)) <= 1e-7 * max(1.0, abs(fd))
        else:
            fd = _fd(lambda e: L(X, U1 + e, U2, G), 0.0, D1)
            assert abs(fd - np.sum(d1 * D1)) <= 1e-7 * max(1.0, abs(fd))
            D2 = rng.standard_normal(U2.shape)
            fd = _fd(lambda e: L(X, U1, U2 + e, G), 0.0, D2)
            assert abs(fd - np.sum(d2 * D2)) <= 1e-7 * max(1.0, abs(fd))


def test_dynamic_vjp_matches_fd_of_bruteforce():
    n, N, nt, beta = 4, 8, 16, 10.0
    wl = synth.small_molecule(n, N, nt, beta, seed=31, dynamic=True)
    tp = synth.bosonic_transform_pair(wl["tau"], beta, omega_max=14.0, tol=1e-10)
    rng = np.random.default_rng(4)
    X, W, V = wl["X"], wl["W_tau"], wl["V"]
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    R = rng.standard_normal((nt, n, n))
    Tf, Tb = tp["T_fwd"], tp["T_bwd"]

    def L(X_, W_, V_, G_):
        S = om.sigma_dynamic_eri(X_, W_, V_, G_, G_[::-1], Tf, Tb)
        return float(np.sum(S * R))

    dG, dX, dW, dV = ov.vjp_dynamic(X, W, V, G, R, Tf, Tb)
    for (grad, shape, f) in [
        (dG, G.shape, lambda e: L(X, W, V, G + e)),
        (dX, X.shape, lambda e: L(X + e, W, V, G)),
        (dW, W.shape, lambda e: L(X, W + e, V, G)),
        (dV, V.shape, lambda e: L(X, W, V + e, G)),
    ]:
        Dd = rng.standard_normal(shape)
        fd = _fd(f, 0.0, Dd)
        assert abs(fd - np.sum(grad * Dd)) <= 1e-6 * max(1.0, abs(fd))


def test_vjp_phi_identity():
    """With R_k = w_k G(beta - tau_k)^T the loss is F[G] of the
    Phi-derivability pin; its full G-derivative is 4 w Sigma(beta-tau)^T
    (U1 = U2), i.e. the VJP through Sigma plus the explicit G(beta-tau) term
    equals 4 times the explicit term."""
    n, N, nt = 4, 10, 10
    wl = synth.small_molecule(n, N, nt, 5.0, seed=8)
    rng = np.random.default_rng(9)
    X, V, w = wl["X"], wl["V"], wl["weights"]
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    R = w[:, None, None] * G[::-1].transpose(0, 2, 1)
    dG, _, _, _ = ov.vjp_static(X, V, V, G, R, bare=True)
    S = om.sigma_static_thc(X, V, V, G, G[::-1])
    explicit = (w[:, None, None] * S.transpose(0, 2, 1))[::-1]      # d/dG of Tr[Sigma G(beta-tau)]
    assert np.allclose(dG + explicit, 4 * explicit, rtol=1e-9, atol=1e-12 * np.abs(explicit).max())
