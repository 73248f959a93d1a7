"""Pins of the THC-GW direct term (oracle/sox_gw.py).

* Identity collocation (X = I, n = N: every THC point is one orbital) makes
  the integrals (ik|lj) = delta_ik delta_lj W_ij, so Sigma = -W * G
  elementwise: the real-space GW product on a grid of points, written out
  with no contraction at all.  A transposed G or W, a wrong sign or a
  dropped factor fails it (G and W are general, non-symmetric matrices).
* Scaled collocation X = diag(c): Sigma_ij = -c_i^2 c_j^2 W_ij G_ij (fixes
  which X factor sits on which side).
* The THC chain equals the 4-index brute force (molecule and mesh), on
  general complex inputs.
* Identity collocation on a mesh: Sigma^k = -sum_R e^{-ikR} g(R) w(R), the
  lattice product of the real-space (inverse DFT) G and W, evaluated with
  numpy's FFT over the mesh axes; this fixes the direction of the momentum
  convolution (W^{k-k'} against W^{k'-k}) and the one 1/N_k.
* Supercell unfolding: a ring of L cells run through the MOLECULAR oracle on
  the supercell, Bloch-transformed, equals the mesh oracle on the
  Bloch-transformed inputs, with scale factor 1.
* Linearity in W, and the mesh oracle on a 1x1x1 mesh with real inputs
  equals the molecular oracle.
"""
import numpy as np
import pytest

from oracle import sox_gw as ogw
from paper_2412_18829_amd import synth


def _tables(mesh):
    return synth.kmesh_index(mesh)


def test_identity_collocation_is_elementwise_product():
    rng = np.random.default_rng(3)
    n, nt = 5, 4
    G = rng.standard_normal((nt, n, n))
    W = rng.standard_normal((nt, n, n))
    X = np.eye(n)
    want = -W * G
    for f in (ogw.sigma_gw_thc, ogw.sigma_gw_eri):
        got = f(X, W, G)
        assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    # a transposed G gives a different answer on these inputs
    assert np.abs(-W * G.transpose(0, 2, 1) - want).max() > 0.1


def test_scaled_collocation():
    rng = np.random.default_rng(4)
    n, nt = 4, 3
    c = rng.uniform(0.5, 2.0, n)
    G = rng.standard_normal((nt, n, n))
    W = rng.standard_normal((nt, n, n))
    got = ogw.sigma_gw_thc(np.diag(c), W, G)
    want = -(c[:, None] ** 2) * (c[None, :] ** 2) * W * G
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.parametrize("n,N", [(3, 5), (4, 2), (2, 6)])
def test_chain_equals_bruteforce_molecule(n, N):
    rng = np.random.default_rng(10 + n + N)
    nt = 3
    X = rng.standard_normal((n, N))
    W = rng.standard_normal((nt, N, N))
    G = rng.standard_normal((nt, n, n))
    a = ogw.sigma_gw_eri(X, W, G)
    b = ogw.sigma_gw_thc(X, W, G)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_linear_in_w():
    rng = np.random.default_rng(5)
    n, N, nt = 3, 4, 2
    X = rng.standard_normal((n, N))
    W1 = rng.standard_normal((nt, N, N))
    W2 = rng.standard_normal((nt, N, N))
    G = rng.standard_normal((nt, n, n))
    s = ogw.sigma_gw_thc(X, 2.0 * W1 - W2, G)
    t = 2.0 * ogw.sigma_gw_thc(X, W1, G) - ogw.sigma_gw_thc(X, W2, G)
    assert np.abs(s - t).max() <= 1e-13 * np.abs(s).max()


def _crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("mesh", [(2, 1, 1), (3, 1, 1), (2, 2, 1)])
def test_chain_equals_bruteforce_mesh(mesh):
    tb = _tables(mesh)
    nk = len(tb[0])
    rng = np.random.default_rng(7 + nk)
    n, N, nt = 3, 4, 2
    X = _crandn(rng, (nk, n, N))
    W = _crandn(rng, (nk, nt, N, N))
    G = _crandn(rng, (nk, nt, n, n))
    a = ogw.sigma_gw_solid_eri(X, W, G, tb)
    b = ogw.sigma_gw_solid_thc(X, W, G, tb)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("mesh", [(3, 1, 1), (2, 3, 1), (2, 2, 2)])
def test_identity_collocation_mesh_is_lattice_product(mesh):
    tb = _tables(mesh)
    nk = len(tb[0])
    rng = np.random.default_rng(20 + nk)
    n, nt = 3, 2
    X = np.broadcast_to(np.eye(n), (nk, n, n)).astype(complex)
    W = _crandn(rng, (nk, nt, n, n))
    G = _crandn(rng, (nk, nt, n, n))
    got = ogw.sigma_gw_solid_thc(X, W, G, tb)
    ax = (0, 1, 2)
    g = np.fft.ifftn(G.reshape(tuple(mesh) + G.shape[1:]), axes=ax)
    w = np.fft.ifftn(W.reshape(tuple(mesh) + W.shape[1:]), axes=ax)
    want = -np.fft.fftn(g * w, axes=ax).reshape(G.shape)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # the reversed convolution (W^{k'-k}: the difference table transposed)
    # differs on these inputs wherever the mesh has a side above 2 (on a
    # side of 2 every momentum is its own negative)
    if max(mesh) > 2:
        tb_rev = (tb[0], tb[1].T.copy(), tb[2], tb[3])
        bad = ogw.sigma_gw_solid_thc(X, W, G, tb_rev)
        assert np.abs(bad - want).max() > 1e-3 * np.abs(want).max()


def _supercell(m, L):
    a, b = m.shape[-2:]
    out = np.zeros(m.shape[:-3] + (L * a, L * b))
    for R1 in range(L):
        for R2 in range(L):
            out[..., R1 * a:(R1 + 1) * a, R2 * b:(R2 + 1) * b] = m[..., (R1 - R2) % L, :, :]
    return out


@pytest.mark.parametrize("L", [2, 3, 4])
def test_supercell_unfolding(L):
    n, N, nt = 2, 3, 3
    rng = np.random.default_rng(40 + L)
    x = rng.standard_normal((L, n, N)) * 0.5
    wt = rng.standard_normal((nt, L, N, N)) * 0.3
    g = rng.standard_normal((nt, L, n, n)) * 0.3
    Ss = ogw.sigma_gw_thc(_supercell(x, L), _supercell(wt, L), _supercell(g, L))
    sig = np.stack([Ss[:, R * n:(R + 1) * n, 0:n] for R in range(L)], axis=1)   # sigma(R)
    tb = synth.kmesh_index((L, 1, 1))
    ph = lambda s: np.exp(s * 2j * np.pi * np.outer(np.arange(L), np.arange(L)) / L)
    Sk = ogw.sigma_gw_solid_thc(np.einsum("kR,Rab->kab", ph(-1), x),
                                np.einsum("kR,tRab->ktab", ph(1), wt),
                                np.einsum("kR,tRab->ktab", ph(1), g), tb)
    pred = np.einsum("kR,tRab->ktab", ph(1), sig)
    assert np.abs(Sk - pred).max() <= 1e-13 * np.abs(pred).max()


def test_gamma_mesh_equals_molecule():
    rng = np.random.default_rng(9)
    n, N, nt = 3, 5, 4
    X = rng.standard_normal((n, N))
    W = rng.standard_normal((nt, N, N))
    G = rng.standard_normal((nt, n, n))
    a = ogw.sigma_gw_thc(X, W, G)
    b = ogw.sigma_gw_solid_thc(X[None].astype(complex), W[None].astype(complex),
                               G[None].astype(complex), _tables((1, 1, 1)))
    assert np.abs(a - b[0]).max() <= 1e-14 * np.abs(a).max()
