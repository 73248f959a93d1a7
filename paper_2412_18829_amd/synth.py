"""Seeded synthetic inputs shaped like the paper's molecules and solids.

This module only draws random numbers and lays out grids.  It contains none
of the self-energy arithmetic: no Green's function, no interaction tensor, no
contraction.  Both the CPU oracle and the GPU library consume what it returns.

What it produces (all float64 / complex128, host numpy arrays):

* an imaginary-time grid on [0, beta]: first-kind Chebyshev nodes with
  Fejer-1 quadrature weights (symmetric about beta/2, so that the node
  n_tau-1-k equals beta - tau_k);
* Fock-operator spectra as (eps, Q): eigenvalues i.i.d. uniform in a stated
  window and a Haar-random orthogonal (or unitary) eigenbasis;
* THC collocation matrices X and SPD interaction matrices V = L L^T (the
  paper's THC factorisation of the two-electron integrals, section
  "THC-SOX and THC-SOSEX", with N/n between 5 and 8);
* the statically screened interaction W(0) = V + V Pi V with a random
  negative-definite Pi, and a dynamically screened W_d(tau) built from
  bosonic poles (periodic on [0, beta]);
* a bosonic imaginary-time <-> Matsubara transform pair (T_fwd, T_bwd) for
  the dynamic path, which the paper takes from its time/frequency grid
  library;
* solid-state inputs on a Monkhorst-Pack mesh with momentum pairing
  U^{-q} = conj(U^q).

Seeds follow numpy.random.Generator(PCG64(20241218 + c)) for workload
c = 1..5, drawing in the order eps, Q, X, L (V), extras, cotangent R.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 20241218


def rng_for(c: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(c)))


# ---------------------------------------------------------------------------
# imaginary-time grid
# ---------------------------------------------------------------------------
def chebyshev_tau_grid(n_tau: int, beta: float):
    """First-kind Chebyshev nodes mapped to [0, beta] and Fejer-1 weights.

    tau_k = beta/2 (1 - cos theta_k), theta_k = (2k+1) pi / (2 n_tau),
    k = 0..n_tau-1 (ascending).  The weights integrate polynomials of degree
    < n_tau exactly.  The node set is symmetric: tau_k + tau_{n-1-k} = beta
    up to one rounding, and we enforce the mirror exactly by construction of
    the upper half from the lower half.
    """
    n = int(n_tau)
    if n < 1:
        raise ValueError("n_tau must be >= 1")
    k = np.arange(n)
    theta = (2 * k + 1) * np.pi / (2 * n)
    half = beta / 2.0
    tau = half * (1.0 - np.cos(theta))
    # exact mirror symmetry: tau[n-1-k] = beta - tau[k]
    for i in range(n // 2):
        tau[n - 1 - i] = beta - tau[i]
    if n % 2 == 1:
        tau[n // 2] = half
    j = np.arange(1, n // 2 + 1)
    s = np.cos(2.0 * np.outer(theta, j)) / (4.0 * j * j - 1.0)
    w = (2.0 / n) * (1.0 - 2.0 * s.sum(axis=1)) * half
    w = 0.5 * (w + w[::-1])
    return tau, w


# ---------------------------------------------------------------------------
# random building blocks
# ---------------------------------------------------------------------------
def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    a = rng.standard_normal((n, n))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    q, r = np.linalg.qr(a)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def random_spd(rng: np.random.Generator, N: int, scale: float) -> np.ndarray:
    """L L^T with L ~ N(0,1) * scale (SPD with probability one)."""
    L = rng.standard_normal((N, N)) * scale
    return L @ L.T


# ---------------------------------------------------------------------------
# molecules
# ---------------------------------------------------------------------------
def molecule(n: int, N: int, n_tau: int, beta: float, *, eps_window=(-2.0, 1.0),
             seed: int | None = None, rng: np.random.Generator | None = None,
             mu: float = 0.0) -> dict:
    """Bare-interaction molecular workload (the paper's molecular THC shapes).

    Draw order: eps, Q, X, L.  X ~ N(0,1)/sqrt(n), V = L L^T with
    L ~ N(0,1)/N.
    """
    if rng is None:
        rng = rng_for(seed if seed is not None else 0)
    eps = rng.uniform(eps_window[0], eps_window[1], size=n)
    Q = haar_orthogonal(rng, n)
    X = rng.standard_normal((n, N)) / np.sqrt(n)
    V = random_spd(rng, N, 1.0 / N)
    tau, w = chebyshev_tau_grid(n_tau, beta)
    return dict(kind="molecule", n=n, N=N, n_tau=n_tau, beta=float(beta), mu=float(mu),
                eps=eps, Q=Q, X=X, V=V, tau=tau, weights=w, rng=rng)


def add_static_screening(wl: dict, pi_scale: float = -0.1) -> dict:
    """W(0) = V + V Pi V with Pi = pi_scale * M M^T / N, M ~ N(0,1)."""
    rng = wl["rng"]
    N = wl["N"]
    M = rng.standard_normal((N, N))
    Pi = pi_scale * (M @ M.T) / N
    V = wl["V"]
    W0 = V + V @ Pi @ V
    W0 = 0.5 * (W0 + W0.T)
    if np.linalg.eigvalsh(W0).min() <= 0.0:
        raise RuntimeError("statically screened interaction is not positive definite")
    wl["W0"] = W0
    return wl


def periodic_bosonic_pole(tau: np.ndarray, beta: float, w: float) -> np.ndarray:
    """[e^{-w tau} + e^{-w (beta - tau)}] / (1 - e^{-w beta}) on [0, beta]."""
    return (np.exp(-w * tau) + np.exp(-w * (beta - tau))) / (-np.expm1(-w * beta))


def add_dynamic_screening(wl: dict, n_poles: int = 8, amp=(0.01, 0.1),
                          log10_w=(-1.0, 1.0)) -> dict:
    """W_d(tau) = sum_k a_k pole_k(tau) S_k, S_k = L_k L_k^T, L_k ~ N(0,1)/N.

    The pole is the beta-periodic bosonic form; its Matsubara transform is
    2 a_k w_k / (w_k^2 + Omega_m^2) per unit S_k.
    """
    rng = wl["rng"]
    N = wl["N"]
    wk = 10.0 ** rng.uniform(log10_w[0], log10_w[1], size=n_poles)
    ak = rng.uniform(amp[0], amp[1], size=n_poles)
    S = np.stack([random_spd(rng, N, 1.0 / N) for _ in range(n_poles)])
    tau, beta = wl["tau"], wl["beta"]
    prof = np.stack([ak[k] * periodic_bosonic_pole(tau, beta, wk[k]) for k in range(n_poles)])
    W = np.einsum("kt,kpq->tpq", prof, S, optimize=True)
    wl.update(W_tau=W, pole_w=wk, pole_a=ak, pole_S=S)
    return wl


def cotangent(wl: dict, shape) -> np.ndarray:
    return wl["rng"].standard_normal(shape)


# ---------------------------------------------------------------------------
# bosonic transform pair for the dynamic path
# ---------------------------------------------------------------------------
def _pivoted_columns(A: np.ndarray, tol: float):
    """Greedy column-pivoted Gram-Schmidt; returns chosen column indices."""
    A = np.array(A, dtype=complex if np.iscomplexobj(A) else float, copy=True)
    norms = np.einsum("ij,ij->j", A.conj(), A).real
    scale = np.sqrt(norms.max())
    chosen = []
    while True:
        j = int(np.argmax(norms))
        if np.sqrt(max(norms[j], 0.0)) <= tol * scale or len(chosen) >= min(A.shape):
            break
        chosen.append(j)
        q = A[:, j] / np.sqrt(norms[j])
        A -= np.outer(q, q.conj() @ A)
        norms = np.einsum("ij,ij->j", A.conj(), A).real
        norms[chosen] = -1.0
    return chosen


def logistic_kernel(tau: np.ndarray, beta: float, omega: np.ndarray) -> np.ndarray:
    """K(tau, w) = e^{-tau w} / (1 + e^{-beta w}), evaluated without overflow."""
    t = np.asarray(tau)[:, None]
    w = np.asarray(omega)[None, :]
    pos = w >= 0
    out = np.empty(np.broadcast(t, w).shape)
    e1 = np.exp(-np.where(pos, t * w, 0.0)) / (1.0 + np.exp(-np.where(pos, beta * w, 0.0)))
    e2 = np.exp(np.where(pos, 0.0, (beta - t) * w)) / (1.0 + np.exp(np.where(pos, 0.0, beta * w)))
    out = np.where(pos, e1, e2)
    return out


def logistic_matsubara(m: np.ndarray, beta: float, omega: np.ndarray) -> np.ndarray:
    """Bosonic transform of K: int_0^beta e^{i Omega_m tau} K(tau,w) dtau.

    Equals tanh(beta w / 2) / (w - i Omega_m) for Omega_m = 2 pi m / beta,
    with the w -> 0, m = 0 limit beta / 2.
    """
    Om = 2.0 * np.pi * np.asarray(m, dtype=float)[:, None] / beta
    w = np.asarray(omega, dtype=float)[None, :]
    th = np.tanh(beta * w / 2.0)
    den = w - 1j * Om
    small = (np.abs(w) < 1e-300) & (Om == 0.0)
    safe = np.where(small, 1.0, den)
    val = th / safe
    return np.where(small, beta / 2.0, val)


def bosonic_transform_pair(tau: np.ndarray, beta: float, omega_max: float,
                           tol: float = 1e-10, n_candidates: int = 4000,
                           m_max: int | None = None) -> dict:
    """Imaginary-time <-> bosonic Matsubara transform pair on a given tau grid.

    A discrete-Lehmann-style construction: real frequencies w_l in
    [-omega_max, omega_max] are picked from a dense candidate set by
    column pivoting of the logistic kernel on the tau nodes; non-negative
    Matsubara indices m are then picked by row pivoting of the transformed
    kernel.  The negative frequencies are implied by conjugation, since
    every function the pair is applied to is real in imaginary time.

    * T_fwd [n_omega, n_tau] complex:  f(i Omega_m) = sum_j T_fwd[m,j] f(tau_j)
    * T_bwd [n_tau, n_omega] complex:  f(tau_i) = Re sum_m T_bwd[i,m] f(i Omega_m)
      (T_bwd carries the factor 2 for m > 0).

    The discrete periodic convolution of two real bosonic functions is then
    Re sum_m T_bwd[i,m] (T_fwd a)_m (T_fwd b)_m.
    """
    tau = np.asarray(tau, dtype=float)
    cand = np.sinh(np.linspace(-np.arcsinh(omega_max * beta), np.arcsinh(omega_max * beta),
                               n_candidates)) / beta
    Kc = logistic_kernel(tau, beta, cand)
    cols = sorted(_pivoted_columns(Kc, tol))
    om = cand[cols]
    if m_max is None:
        m_max = int(np.ceil(8 * omega_max * beta / (2 * np.pi))) + 64
    ms = np.arange(0, m_max + 1)
    F = logistic_matsubara(ms, beta, om)          # [M, r]
    # real stacked rows so that the choice of m is real-arithmetic pivoting
    rows = _pivoted_columns(np.concatenate([F.real, F.imag], axis=1).T, tol * 1e-3)
    rows = sorted(set(rows) | {0})
    msel = ms[rows]
    Fs = F[rows]                                    # [n_omega, r]
    Kt = logistic_kernel(tau, beta, om)            # [n_tau, r]
    # forward: real pole coefficients from tau samples (least squares on the
    # nodes), then their Matsubara values
    T_fwd = Fs @ np.linalg.pinv(Kt, rcond=1e-14)
    # backward: real coefficients from the real and imaginary parts of the
    # Matsubara values, then back to the tau nodes
    P = np.linalg.pinv(np.concatenate([Fs.real, Fs.imag], axis=0), rcond=1e-14)
    nf = Fs.shape[0]
    T_bwd = Kt @ P[:, :nf] - 1j * (Kt @ P[:, nf:])
    return dict(T_fwd=T_fwd, T_bwd=T_bwd, m=msel, omega_l=om,
                Omega=2 * np.pi * msel / beta)


# ---------------------------------------------------------------------------
# solids
# ---------------------------------------------------------------------------
def kmesh_index(mesh):
    """Integer k-vectors of a Gamma-centred Monkhorst-Pack mesh and the tables
    kdiff[a,b] = index of k_a - k_b, kneg[a] = index of -k_a (mod mesh)."""
    m = np.array(mesh, dtype=int)
    ks = np.array([(a, b, c) for a in range(m[0]) for b in range(m[1]) for c in range(m[2])])
    lut = {tuple(k): i for i, k in enumerate(ks)}
    nk = len(ks)
    kdiff = np.empty((nk, nk), dtype=np.int32)
    ksum = np.empty((nk, nk), dtype=np.int32)
    for a in range(nk):
        for b in range(nk):
            kdiff[a, b] = lut[tuple((ks[a] - ks[b]) % m)]
            ksum[a, b] = lut[tuple((ks[a] + ks[b]) % m)]
    kneg = np.array([lut[tuple((-k) % m)] for k in ks], dtype=np.int32)
    return ks, kdiff, ksum, kneg


def solid(mesh, n: int, N: int, n_tau: int, beta: float, *, eps_window=(-1.5, 1.0),
          seed: int | None = None, rng: np.random.Generator | None = None,
          mu: float = 0.0) -> dict:
    """k-point workload with momentum-paired interactions.

    X^k ~ (N(0,1) + i N(0,1)) / sqrt(2 n); U^q = L_q L_q^dagger / N^2-scaled,
    with U^{-q} = conj(U^q) (real at q = -q); eigenbases Haar-unitary per k,
    eigenvalues uniform in eps_window.
    """
    if rng is None:
        rng = rng_for(seed if seed is not None else 0)
    ks, kdiff, ksum, kneg = kmesh_index(mesh)
    nk = len(ks)
    eps = rng.uniform(eps_window[0], eps_window[1], size=(nk, n))
    Q = np.stack([haar_unitary(rng, n) for _ in range(nk)])
    X = (rng.standard_normal((nk, n, N)) + 1j * rng.standard_normal((nk, n, N))) / np.sqrt(2 * n)
    V = paired_hermitian(rng, kneg, N, 1.0 / N)
    tau, w = chebyshev_tau_grid(n_tau, beta)
    return dict(kind="solid", mesh=tuple(mesh), nk=nk, n=n, N=N, n_tau=n_tau, beta=float(beta),
                mu=float(mu), eps=eps, Q=Q, X=X, V=V, tau=tau, weights=w, kvecs=ks,
                kdiff=kdiff, ksum=ksum, kneg=kneg, rng=rng)


def solid_screening_poles(wl: dict, n_poles: int = 8, amp=(0.01, 0.1),
                          log10_w=(-1.0, 1.0)) -> list:
    """The draws of add_dynamic_screening_solid without forming W: a list of
    (a_k, pole_{w_k}(tau) [n_tau], S_k [n_k, N, N]) in drawing order, so that
    W^q(tau_j) = sum_k a_k pole_k[j] S_k[q] can be assembled on a device."""
    rng = wl["rng"]
    N, tau, beta = wl["N"], wl["tau"], wl["beta"]
    out = []
    for _ in range(n_poles):
        w = 10.0 ** rng.uniform(*log10_w)
        a = rng.uniform(*amp)
        S = paired_hermitian(rng, wl["kneg"], N, 1.0 / N)
        out.append((a, periodic_bosonic_pole(tau, beta, w), S))
    return out


def add_dynamic_screening_solid(wl: dict, n_poles: int = 8, amp=(0.01, 0.1),
                                log10_w=(-1.0, 1.0)) -> dict:
    """W^q(tau) = sum_k a_k pole_{w_k}(tau) S_k^q on a k-point workload, with
    each S_k^q momentum-paired Hermitian (S^{-q} = conj(S^q)); the pole
    parameters are drawn as for molecules.  Stored q-major: [n_k, n_tau, N, N]."""
    N, tau = wl["N"], wl["tau"]
    W = np.zeros((wl["nk"], len(tau), N, N), dtype=complex)
    for a, pole, S in solid_screening_poles(wl, n_poles, amp, log10_w):
        W += a * pole[None, :, None, None] * S[:, None]
    wl.update(W_tau=W)
    return wl


def paired_hermitian(rng: np.random.Generator, kneg, N: int, scale: float) -> np.ndarray:
    """Hermitian positive matrices U^q with U^{-q} = conj(U^q)."""
    nk = len(kneg)
    U = np.zeros((nk, N, N), dtype=complex)
    done = np.zeros(nk, dtype=bool)
    for q in range(nk):
        if done[q]:
            continue
        mq = kneg[q]
        if mq == q:
            L = rng.standard_normal((N, N)) * scale
            U[q] = L @ L.T
        else:
            L = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * scale / np.sqrt(2)
            U[q] = L @ L.conj().T
            U[mq] = U[q].conj()
        done[q] = done[mq] = True
    return U


def column_support(N: int, per_band: int, seed: int, band: int = 50) -> np.ndarray:
    """Sorted THC column indices, per_band distinct ones drawn in each band of
    `band` columns: the support of a collocation matrix that is zero
    elsewhere (every 64- or 80-wide column tile holds some)."""
    rng = np.random.default_rng(seed)
    cols = [b0 + rng.choice(min(band, N - b0), size=min(per_band, N - b0), replace=False)
            for b0 in range(0, N, band)]
    return np.sort(np.concatenate(cols))


# ---------------------------------------------------------------------------
# the five workload recipes
# ---------------------------------------------------------------------------
def workload(c: int) -> dict:
    """The five workload recipes, c = 1..5, each seeded by rng_for(c)."""
    rng = rng_for(c)
    if c == 1:
        return molecule(8, 24, 16, 10.0, rng=rng)
    if c == 2:
        return molecule(64, 384, 64, 50.0, rng=rng)
    if c == 3:
        return add_static_screening(molecule(200, 1200, 100, 100.0, rng=rng))
    if c == 4:
        return add_dynamic_screening(molecule(300, 1800, 120, 100.0, rng=rng))
    if c == 5:
        return solid((3, 3, 3), 52, 400, 100, 100.0, rng=rng)
    raise ValueError(f"unknown workload {c}")


def small_molecule(n: int, N: int, n_tau: int, beta: float, seed: int,
                   static: bool = False, dynamic: bool = False) -> dict:
    """Reduced-size molecule built by the same recipe (tests)."""
    wl = molecule(n, N, n_tau, beta, rng=rng_for(seed))
    if static:
        add_static_screening(wl)
    if dynamic:
        add_dynamic_screening(wl)
    return wl
