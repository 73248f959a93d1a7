"""Intermediate-representation (IR) imaginary-time grid, built in-house
(oracle; test infrastructure only).

The paper's computational details run every calculation on sparse IR grids
(beta, Lambda and the number of tau points listed there).  The IR basis is the
singular value expansion of the analytic-continuation kernel; this module
builds it from that definition with numpy's SVD as the one library step:

1. Kernel.  In the dimensionless variables x = 2 tau / beta - 1 and
   y = beta omega / Lambda (both in [-1, 1]) the logistic kernel
       K(x, y) = exp(-Lambda y (x + 1) / 2) / (1 + exp(-Lambda y))
   is centrosymmetric, K(-x, -y) = K(x, y), so its expansion splits into
   even and odd parts on [0, 1] x [0, 1]: K_+- (x, y) = K(x, y) +- K(x, -y).
   The same kernel serves fermionic and bosonic functions (a bosonic
   spectral weight rho(omega) enters as rho(omega) coth(beta omega / 2)).
2. Discretisation.  Composite Gauss-Legendre quadrature (P nodes per
   segment) on segments graded geometrically towards x = 1 and y = 0, where
   the kernel varies on the scale 1 / Lambda, and at most HMAX wide.
3. SVD of sqrt(w_x) K_+- sqrt(w_y); u_l(x) = column / sqrt(w_x) / sqrt(2)
   (normalised on [-1, 1]), sign fixed by u_l(x -> 1) > 0; the two parities
   merged by singular value.  Basis size L = #{s_l >= eps s_0}.
4. u_l between nodes: per-segment Legendre series of degree P - 1 from the
   nodal values (Gauss quadrature projection).
5. Sampling times: the L roots of u_L, the first function left out (u_l has
   exactly l roots), tau_i = beta (x_i + 1) / 2: ascending and mirror
   symmetric.
6. Matsubara transforms U^_l(i Omega_m) = int_0^beta e^{i Omega_m tau} U_l(tau)
   dtau, U_l(tau) = sqrt(2 / beta) u_l(x), Omega_m = 2 pi m / beta, per
   segment from int_{-1}^{1} e^{i a t} P_k(t) dt = 2 i^k j_k(a).
7. Bosonic frequencies: m = 0 and, for the first even and the first odd
   function left out, the integer m just below each sign change of Re U^
   (even) or Im U^ (odd) over m = 0 .. 4 Lambda.
8. Transform pair for functions real in imaginary time: coefficients
   g = U_s^{-1} f(tau) (U_s[i][l] = U_l(tau_i)); T_fwd = U^ U_s^{-1}; T_bwd
   from the least-squares fit of g to [Re f(i Omega_m); Im f(i Omega_m)]
   (f(-i Omega) = conj f(i Omega)): f(tau_i) = Re sum_m T_bwd[i][m] f(i Omega_m).
9. Quadrature weights on the sampling times: w = U_s^{-T} I, I_l =
   int_0^beta U_l(tau) dtau.
10. Fermionic pair (ir_fermion): the same basis and sampling times, odd
   frequencies nu_n = (2n + 1) pi / beta (m = n + 1/2 in step 6), n = 0 and
   the sign changes of Im U^ (first omitted even function: a function even
   about beta / 2 has an imaginary fermionic transform) and of Re U^ (first
   omitted odd function); T_fwd, T_bwd as in step 8, and the row t_beta with
   f(beta^-) = sum_i t_beta[i] f(tau_i) (the basis evaluated at x = 1).

Readings (also in the design notes): the paper gives beta, Lambda and the
number of tau points but not eps, the discretisation or the Matsubara
sampling rule; steps 2, 5 and 7 are this module's choices, eps is a
parameter.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss, legval
from scipy.special import spherical_jn

P = 16        # Gauss-Legendre nodes per segment
HMAX = 0.25   # widest segment (in x or y)


def kernel(x, y, lam):
    """K(x, y) for x, y arrays (outer product), evaluated without overflow."""
    x = np.asarray(x, dtype=float)[:, None]
    y = np.asarray(y, dtype=float)[None, :]
    a = np.abs(y)
    # y >= 0: e^{-L y (x+1)/2} / (1 + e^{-L y});  y < 0: e^{L y (1-x)/2} / (1 + e^{L y})
    return np.where(y >= 0, np.exp(-lam * a * (x + 1) / 2), np.exp(-lam * a * (1 - x) / 2)) \
        / (1 + np.exp(-lam * a))


def _cap(b):
    out = [b[0]]
    for a, c in zip(b[:-1], b[1:]):
        m = int(np.ceil((c - a) / HMAX - 1e-12))
        out += list(a + (c - a) * np.arange(1, m + 1) / m)
    return np.array(out)


def segments(lam, towards_one: bool):
    d = []
    j = 0
    while 2.0 ** j / lam < 1.0:
        d.append(2.0 ** j / lam)
        j += 1
    pts = [1.0 - v for v in d] if towards_one else d
    return _cap(np.array(sorted(set([0.0, 1.0] + pts))))


def _quadrature(br):
    t, w = leggauss(P)
    xs = [(a + b) / 2 + (b - a) / 2 * t for a, b in zip(br[:-1], br[1:])]
    ws = [(b - a) / 2 * w for a, b in zip(br[:-1], br[1:])]
    return np.concatenate(xs), np.concatenate(ws)


def sve(lam):
    """Singular values and left functions of both parities, merged in
    descending order: list of (s, parity, u at the x nodes), plus the x
    segments and quadrature."""
    bx, by = segments(lam, True), segments(lam, False)
    x, wx = _quadrature(bx)
    y, wy = _quadrature(by)
    out = []
    for par in (+1, -1):
        K = kernel(x, y, lam) + par * kernel(x, -y, lam)
        A = np.sqrt(wx)[:, None] * K * np.sqrt(wy)[None, :]
        U, s, _ = np.linalg.svd(A)
        for l in range(len(s)):
            u = U[:, l] / np.sqrt(wx) / np.sqrt(2.0)
            if u[-1] < 0:
                u = -u
            out.append((s[l], par, u))
    out.sort(key=lambda r: -r[0])
    return out, bx, x, wx


def legendre_coeffs(u):
    """Per-segment Legendre coefficients [segment][k] from nodal values."""
    t, w = leggauss(P)
    Pk = np.stack([legval(t, np.eye(P)[k]) for k in range(P)])
    uu = np.asarray(u).reshape(-1, P)
    return ((uu * w[None, :]) @ Pk.T) * ((2 * np.arange(P) + 1) / 2)[None, :]


def evaluate(c, par, bx, xq):
    """u(x) on [-1, 1] from its coefficients on [0, 1] and its parity."""
    xq = np.atleast_1d(np.asarray(xq, dtype=float))
    ax = np.abs(xq)
    j = np.clip(np.searchsorted(bx, ax, side="right") - 1, 0, len(bx) - 2)
    t = (2 * ax - bx[j] - bx[j + 1]) / (bx[j + 1] - bx[j])
    val = np.array([legval(t[i], c[j[i]]) for i in range(len(xq))])
    return np.where(xq < 0, par * val, val)


def roots(c, par, bx):
    """Roots of u on (-1, 1): sign changes on 64 sub-intervals per segment
    of (0, 1], refined by bisection, mirrored by parity (odd u: plus x = 0)."""
    grid = np.unique(np.concatenate([np.linspace(a, b, 65) for a, b in zip(bx[:-1], bx[1:])]))
    if par < 0:
        grid = grid[1:]   # an odd u vanishes at 0: its rounded value there carries no sign
    v = evaluate(c, par, bx, grid)
    rs = []
    for i in range(len(grid) - 1):
        if grid[i] > 0 and v[i] == 0.0:
            rs.append(grid[i])
        elif v[i] * v[i + 1] < 0:
            a, b, fa = grid[i], grid[i + 1], v[i]
            for _ in range(100):
                m = 0.5 * (a + b)
                fm = evaluate(c, par, bx, m)[0]
                if fa * fm <= 0:
                    b = m
                else:
                    a, fa = m, fm
            rs.append(0.5 * (a + b))
    rs = np.array([r for r in rs if r > 0])
    mid = [0.0] if par < 0 else []
    return np.concatenate([-rs[::-1], mid, rs])


def matsubara(c, par, bx, beta, m):
    """U^(i Omega_m) = sqrt(beta / 2) int_{-1}^{1} e^{i pi m (x + 1)} u(x) dx."""
    m = np.asarray(m, dtype=float)
    out = np.zeros(len(m), dtype=complex)
    ks = np.arange(P)
    for j in range(len(bx) - 1):
        a, b = bx[j], bx[j + 1]
        cc, h = (a + b) / 2, (b - a) / 2
        J = np.stack([spherical_jn(k, np.pi * m * h) for k in ks], axis=1)
        plus = (J * (1j ** ks)[None, :]) @ c[j]          # segment [a, b]
        minus = (J * ((-1j) ** ks)[None, :]) @ c[j]      # its mirror [-b, -a]
        out += 2 * h * (np.exp(1j * np.pi * m * (cc + 1)) * plus
                        + par * np.exp(1j * np.pi * m * (1 - cc)) * minus)
    return np.sqrt(beta / 2) * out


def _sign_changes(g):
    return np.where(g[:-1] * g[1:] < 0)[0]


def ir_grid(beta: float, lam: float, eps: float) -> dict:
    """The IR grid: tau nodes, weights, bosonic Matsubara indices m, the
    transform pair (T_fwd [n_omega, n_tau], T_bwd [n_tau, n_omega]) and the
    singular values s_l / s_0 of the basis."""
    fs, bx, x, wx = sve(lam)
    s = np.array([f[0] for f in fs])
    L = int(np.sum(s >= eps * s[0]))
    cs = [legendre_coeffs(f[2]) for f in fs[:L]]
    pars = [f[1] for f in fs[:L]]
    lL = L
    xr = roots(legendre_coeffs(fs[lL][2]), fs[lL][1], bx)
    if len(xr) != L:
        raise RuntimeError(f"u_L has {len(xr)} roots, expected {L}")
    tau = beta * (xr + 1) / 2
    Us = np.stack([evaluate(cs[l], pars[l], bx, xr) for l in range(L)], axis=1) * np.sqrt(2 / beta)
    le = next(l for l in range(L, len(fs)) if fs[l][1] > 0)
    lo = next(l for l in range(L, len(fs)) if fs[l][1] < 0)
    ms = np.arange(0, int(4 * lam) + 1)
    ge = matsubara(legendre_coeffs(fs[le][2]), 1, bx, beta, ms).real
    go = matsubara(legendre_coeffs(fs[lo][2]), -1, bx, beta, ms).imag
    sel = np.unique(np.concatenate([[0], _sign_changes(ge), _sign_changes(go)]))
    Uh = np.stack([matsubara(cs[l], pars[l], bx, beta, sel) for l in range(L)], axis=1)
    T_fwd = Uh @ np.linalg.inv(Us)
    A = Us @ np.linalg.pinv(np.concatenate([Uh.real, Uh.imag], axis=0))
    nm = len(sel)
    T_bwd = A[:, :nm] - 1j * A[:, nm:]
    I = np.array([np.sqrt(beta / 2) * 2 * np.sum(wx * fs[l][2]) if pars[l] > 0 else 0.0
                  for l in range(L)])
    weights = np.linalg.solve(Us.T, I)
    return dict(tau=tau, weights=weights, m=sel, T_fwd=T_fwd, T_bwd=T_bwd,
                s=s[:L] / s[0], L=L, Us=Us, Uhat=Uh)


def ir_fermion(beta: float, lam: float, eps: float) -> dict:
    """Fermionic transform pair on the IR sampling times: n (nu_n = (2n+1)
    pi / beta), T_fwd [n_nu, n_tau], T_bwd [n_tau, n_nu] (f(tau_i) = Re
    sum_n T_bwd[i][n] f(i nu_n) for a function real in imaginary time) and
    t_beta [n_tau] (f(beta^-) = t_beta . f(tau))."""
    fs, bx, x, wx = sve(lam)
    s = np.array([f[0] for f in fs])
    L = int(np.sum(s >= eps * s[0]))
    cs = [legendre_coeffs(f[2]) for f in fs[:L]]
    pars = [f[1] for f in fs[:L]]
    xr = roots(legendre_coeffs(fs[L][2]), fs[L][1], bx)
    if len(xr) != L:
        raise RuntimeError(f"u_L has {len(xr)} roots, expected {L}")
    tau = beta * (xr + 1) / 2
    Us = np.stack([evaluate(cs[l], pars[l], bx, xr) for l in range(L)], axis=1) * np.sqrt(2 / beta)
    le = next(l for l in range(L, len(fs)) if fs[l][1] > 0)
    lo = next(l for l in range(L, len(fs)) if fs[l][1] < 0)
    ns = np.arange(0, int(4 * lam) + 1)
    ge = matsubara(legendre_coeffs(fs[le][2]), 1, bx, beta, ns + 0.5).imag
    go = matsubara(legendre_coeffs(fs[lo][2]), -1, bx, beta, ns + 0.5).real
    sel = np.unique(np.concatenate([[0], _sign_changes(ge), _sign_changes(go)]))
    Uh = np.stack([matsubara(cs[l], pars[l], bx, beta, sel + 0.5) for l in range(L)], axis=1)
    Uinv = np.linalg.inv(Us)
    T_fwd = Uh @ Uinv
    A = Us @ np.linalg.pinv(np.concatenate([Uh.real, Uh.imag], axis=0))
    nm = len(sel)
    T_bwd = A[:, :nm] - 1j * A[:, nm:]
    ub = np.array([evaluate(cs[l], pars[l], bx, 1.0)[0] for l in range(L)]) * np.sqrt(2 / beta)
    return dict(tau=tau, n=sel, T_fwd=T_fwd, T_bwd=T_bwd, t_beta=ub @ Uinv, L=L)
