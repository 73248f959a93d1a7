"""GPU adjoint (sox_sigma_vjp, via torch.autograd) against the FP64 reference
VJP (torch CPU autograd of the step chain, pinned by finite differences of
the 4-index brute force in test_oracle_vjp.py).

Tolerance per gradient (max |diff| / max |ref|): FP64 1e-10, FP32 1e-5.
"""
import numpy as np
import pytest

from oracle import sox_mol as om
from oracle import sox_vjp as ov
from paper_2412_18829_amd import synth
from tests.gpu_util import dev, have_gpu, host, log, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def B():
    if not have_gpu():
        pytest.skip("no GPU")
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


def _inputs(n, N, nt, beta, seed):
    wl = synth.small_molecule(n, N, nt, beta, seed=seed, static=True)
    rng = np.random.default_rng(seed)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    R = rng.standard_normal((nt, n, n))
    return wl, G, R


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("entry", ["bare", "static"])
@pytest.mark.parametrize("shape", [(6, 20, 8), (13, 70, 5), (24, 130, 6)])
def test_static_vjp_vs_reference(B, precision, entry, shape):
    import torch
    from paper_2412_18829_amd import autograd as AG
    n, N, nt = shape
    log(f"vjp {entry} {shape} {precision}")
    wl, G, R = _inputs(n, N, nt, 7.0, 500 + n)
    X, V = wl["X"], wl["V"]
    U1 = V if entry == "bare" else wl["W0"]
    plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision)
    Xd, U1d, Gd = dev(X).requires_grad_(), dev(U1).requires_grad_(), dev(G).requires_grad_()
    U2d = None if entry == "bare" else dev(V).requires_grad_()
    S = AG.sox_sigma(plan, Xd, U1d, Gd, U2d)
    S.backward(dev(R))
    torch.cuda.synchronize()
    dG, dX, d1, d2 = ov.vjp_static(X, U1, V, G, R, bare=(entry == "bare"))
    errs = {"dG": rel_err(host(Gd.grad), dG), "dX": rel_err(host(Xd.grad), dX),
            "dU1": rel_err(host(U1d.grad), d1)}
    if entry == "static":
        errs["dU2"] = rel_err(host(U2d.grad), d2)
    log("  " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[precision], k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_vjp_past_320_orbitals(B, precision):
    """n = 336 > 320: the adjoint's Hadamard-contract kernel runs its output
    columns in two chunks (each recomputing its weighted tile); against the
    reference VJP."""
    import torch
    from paper_2412_18829_amd import autograd as AG
    n, N, nt = 336, 48, 4
    log(f"vjp static n={n} {precision}")
    wl, G, R = _inputs(n, N, nt, 6.0, 336)
    plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision)
    Xd, U1d, U2d, Gd = (dev(a).requires_grad_() for a in (wl["X"], wl["W0"], wl["V"], G))
    S = AG.sox_sigma(plan, Xd, U1d, Gd, U2d)
    S.backward(dev(R))
    torch.cuda.synchronize()
    dG, dX, d1, d2 = ov.vjp_static(wl["X"], wl["W0"], wl["V"], G, R)
    errs = {"dG": rel_err(host(Gd.grad), dG), "dX": rel_err(host(Xd.grad), dX),
            "dU1": rel_err(host(U1d.grad), d1), "dU2": rel_err(host(U2d.grad), d2)}
    log("  " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[precision], k


def test_vjp_slabs_match_single_slab(B, monkeypatch):
    import torch
    n, N, nt = 10, 64, 7
    wl, G, R = _inputs(n, N, nt, 5.0, 9)
    outs = []
    for budget in (None, "2"):
        if budget:
            monkeypatch.setenv("SOX_WS_BUDGET_MB", budget)
        plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp64")
        dG = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
        dX = torch.empty((n, N), dtype=torch.float64, device="cuda")
        dV = torch.empty((N, N), dtype=torch.float64, device="cuda")
        B.sox_sigma_vjp(plan, "bare", dev(wl["X"]), dev(wl["V"]), None, dev(G), dev(R), dG, dX, dV, None)
        torch.cuda.synchronize()
        outs.append((host(dG), host(dX), host(dV)))
    for a, b in zip(outs[0], outs[1]):
        assert rel_err(b, a) <= 1e-13


def test_vjp_bare_rejects_dU2(B):
    import torch
    n, N, nt = 4, 16, 4
    wl, G, R = _inputs(n, N, nt, 5.0, 3)
    plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp32")
    dV = torch.empty((N, N), dtype=torch.float64, device="cuda")
    with pytest.raises(B.SoxError):
        B.sox_sigma_vjp(plan, "bare", dev(wl["X"]), dev(wl["V"]), None, dev(G), dev(R), None, None, dV, dV)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(5, 12, 24, 20.0), (12, 64, 32, 40.0), (20, 140, 40, 100.0)])
def test_dynamic_vjp_vs_reference(B, precision, shape):
    import torch
    from paper_2412_18829_amd import autograd as AG
    n, N, nt, beta = shape
    log(f"dynamic vjp {shape} {precision}")
    wl = synth.small_molecule(n, N, nt, beta, seed=700 + n, dynamic=True)
    tp = synth.bosonic_transform_pair(wl["tau"], beta, omega_max=14.0, tol=1e-10)
    rng = np.random.default_rng(n)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    R = rng.standard_normal((nt, n, n))
    plan = B.Plan(n, N, wl["tau"], wl["weights"], beta, precision=precision,
                  t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
    Xd, Wd, Vd, Gd = (dev(a).requires_grad_() for a in (wl["X"], wl["W_tau"], wl["V"], G))
    S = AG.sox_sigma_dynamic(plan, Xd, Wd, Vd, Gd)
    S.backward(dev(R))
    torch.cuda.synchronize()
    dG, dX, dW, dV = ov.vjp_dynamic(wl["X"], wl["W_tau"], wl["V"], G, R, tp["T_fwd"], tp["T_bwd"])
    errs = {"dG": rel_err(host(Gd.grad), dG), "dX": rel_err(host(Xd.grad), dX),
            "dW": rel_err(host(Wd.grad), dW), "dV": rel_err(host(Vd.grad), dV)}
    log("  " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()) + f"  n_omega={len(tp['m'])}")
    tol = {"fp64": 1e-9, "fp32": 1e-5}[precision]
    for k, v in errs.items():
        assert v <= tol, k


def test_dynamic_vjp_v_slabs_match(B, monkeypatch):
    import torch
    n, N, nt, beta = 21, 90, 20, 40.0
    wl = synth.small_molecule(n, N, nt, beta, seed=78, dynamic=True)
    tp = synth.bosonic_transform_pair(wl["tau"], beta, omega_max=14.0, tol=1e-10)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"])
    R = np.random.default_rng(2).standard_normal((nt, n, n))
    outs = []
    for budget in (None, "20"):
        if budget:
            monkeypatch.setenv("SOX_WS_BUDGET_MB", budget)
        plan = B.Plan(n, N, wl["tau"], wl["weights"], beta, precision="fp64",
                      t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
        dG = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
        dX = torch.empty((n, N), dtype=torch.float64, device="cuda")
        dW = torch.empty((nt, N, N), dtype=torch.float64, device="cuda")
        dV = torch.empty((N, N), dtype=torch.float64, device="cuda")
        B.sox_sigma_vjp(plan, "dynamic", dev(wl["X"]), dev(wl["W_tau"]), dev(wl["V"]), dev(G), dev(R),
                        dG, dX, dW, dV)
        torch.cuda.synchronize()
        outs.append((host(dG), host(dX), host(dW), host(dV)))
    for a, b in zip(outs[0], outs[1]):
        assert rel_err(b, a) <= 1e-12


def test_dynamic_vjp_full_size_directional_fd(B):
    """n=300, N=1800, 120 tau nodes, 8-pole W(tau): the float32 adjoint of
    L = sum(Sigma * R) along one random direction in (G, X, W, V) against a
    central finite difference of the float64 forward path at the same size
    (L is a polynomial of degree 4 in the inputs, so the step 1e-4 leaves a
    truncation error near 1e-8).  The bound 5e-5 is the float32 one (1e-5)
    widened for a derivative summed over 4e8 gradient entries (measured
    7.5e-6)."""
    import time
    import torch
    wl = synth.workload(4)
    n, N, nt = wl["n"], wl["N"], wl["n_tau"]
    tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=14.0, tol=1e-10)
    rng = np.random.default_rng(44)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    R = rng.standard_normal((nt, n, n))
    kw = dict(t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
    p32 = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp32", **kw)
    X, W, V, Gd, Rd = dev(wl["X"]), dev(wl["W_tau"]), dev(wl["V"]), dev(G), dev(R)
    dG, dX, dW, dV = (torch.zeros_like(a) for a in (Gd, X, W, V))
    log(f"dynamic vjp full size n={n} N={N} n_tau={nt} n_omega={len(tp['m'])}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.sox_sigma_vjp(p32, "dynamic", X, W, V, Gd, Rd, dG, dX, dW, dV)
    torch.cuda.synchronize()
    log(f"  fp32 vjp {time.perf_counter() - t0:.2f} s")
    del p32
    # one random direction, scaled to each input's size
    dirs = []
    for a in (Gd, X, W, V):
        d = torch.empty_like(a).normal_(generator=torch.Generator(device="cuda").manual_seed(7))
        dirs.append(d * (a.abs().max() / d.abs().max()))
    ana = sum(float((g * d).sum()) for g, d in zip((dG, dX, dW, dV), dirs))
    del dG, dX, dW, dV
    p64 = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp64", **kw)
    S = torch.empty_like(Gd)
    eps = 1e-4

    def loss(sign):
        a = [x + sign * eps * d for x, d in zip((Gd, X, W, V), dirs)]
        B.sox_sigma_dynamic(p64, a[1], a[2], a[3], a[0], S)
        torch.cuda.synchronize()
        return float((S * Rd).sum())

    fd = (loss(1.0) - loss(-1.0)) / (2 * eps)
    err = abs(ana - fd) / abs(fd)
    log(f"  directional derivative: vjp {ana:.10e} fd {fd:.10e} rel diff {err:.2e}")
    assert err <= 5e-5
