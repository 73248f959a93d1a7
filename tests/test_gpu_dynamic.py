"""GPU parity of the dynamically screened SOX path (U1 = W_d(tau), U2 = V)
against the FP64 oracle's eq:GG chain, through the C ABI.

The oracle's chain is pinned to the 4-index brute force and to the
continuum single-pole result in test_oracle_dyn.py.  Both sides use the same
transform pair (an input).  Tolerances (max |diff| / max |oracle|): FP32
1e-6; BF16x3 (the fused contraction in split precision) 1e-4; FP64 1e-11, raised to 10x the input's own rounding floor (the
disagreement of two exact float64 codings of the oracle) when a coarse grid
makes the transform pair ill-conditioned.

The full-size case (n=300, N=1800, 120 tau nodes) runs the GPU in its
production launch configuration on a collocation matrix that is zero
outside 64 scattered THC columns: the exact result then equals the reduced
problem on those columns, which the oracle evaluates quickly.
"""
import numpy as np
import pytest

from oracle import sox_mol as om
from paper_2412_18829_amd import synth
from tests.gpu_util import dev, have_gpu, host, log, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-6, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def B():
    if not have_gpu():
        pytest.skip("no GPU")
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


def _pair(wl, omega_max=14.0):
    return synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=omega_max, tol=1e-10)


def _run(B, wl, tp, precision, X, W, V, G):
    import torch
    n, N, nt = X.shape[0], X.shape[1], G.shape[0]
    plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision,
                  t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_dynamic(plan, dev(X), dev(W), dev(V), dev(G), S)
    torch.cuda.synchronize()
    return host(S), plan


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("shape", [(5, 12, 24, 20.0), (13, 70, 30, 30.0), (24, 150, 40, 100.0)])
def test_dynamic_small_general_G(B, precision, shape):
    n, N, nt, beta = shape
    log(f"dynamic {shape} {precision}")
    wl = synth.small_molecule(n, N, nt, beta, seed=300 + n, dynamic=True)
    tp = _pair(wl)
    rng = np.random.default_rng(n)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    got, _ = _run(B, wl, tp, precision, wl["X"], wl["W_tau"], wl["V"], G)
    ref = om.sigma_dynamic_thc(wl["X"], wl["W_tau"], wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
    tol = TOL[precision]
    if precision == "fp64" and n <= 13:
        # rounding floor of this input: two exact float64 codings of the same
        # quantity (4-index brute force and the step chain) differ by this
        # much when the transform pair is ill-conditioned
        bf = om.sigma_dynamic_eri(wl["X"], wl["W_tau"], wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
        tol = max(tol, 10.0 * rel_err(bf, ref))
    err = rel_err(got, ref)
    log(f"  rel err {err:.3e} (tol {tol:.1e})  n_omega={len(tp['m'])}")
    assert err <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_dynamic_many_tau_nodes_generic_transforms(B, precision):
    """140 tau nodes: past the 128 rows the transform kernels hold in LDS, so
    both transforms run on the generic float64 product; parity as above."""
    n, N, nt, beta = 7, 30, 140, 30.0
    log(f"dynamic {n} {N} {nt} {precision} (generic transforms)")
    wl = synth.small_molecule(n, N, nt, beta, seed=901, dynamic=True)
    tp = _pair(wl)
    rng = np.random.default_rng(901)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    got, _ = _run(B, wl, tp, precision, wl["X"], wl["W_tau"], wl["V"], G)
    ref = om.sigma_dynamic_thc(wl["X"], wl["W_tau"], wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
    err = rel_err(got, ref)
    tol = TOL[precision]
    if precision == "fp64":
        bf = om.sigma_dynamic_eri(wl["X"], wl["W_tau"], wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
        tol = max(tol, 10.0 * rel_err(bf, ref))
    log(f"  rel err {err:.3e} (tol {tol:.1e})  n_omega={len(tp['m'])}")
    assert err <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_dynamic_v_slabs_match(B, precision, monkeypatch):
    """A small workspace budget forces several v slabs (D accumulated across
    slabs); the result must match the single-slab run and the oracle."""
    n, N, nt, beta = 21, 90, 20, 40.0
    wl = synth.small_molecule(n, N, nt, beta, seed=77, dynamic=True)
    tp = _pair(wl)
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"])
    one, p1 = _run(B, wl, tp, precision, wl["X"], wl["W_tau"], wl["V"], G)
    monkeypatch.setenv("SOX_WS_BUDGET_MB", "12")
    many, p2 = _run(B, wl, tp, precision, wl["X"], wl["W_tau"], wl["V"], G)
    assert p2.workspace_size("dynamic") < p1.workspace_size("dynamic")
    ref = om.sigma_dynamic_thc(wl["X"], wl["W_tau"], wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
    assert rel_err(one, ref) <= TOL[precision]
    assert rel_err(many, ref) <= TOL[precision]
    assert rel_err(many, one) <= {"fp64": 1e-14, "fp32": 1e-6, "bf16x3": 1e-5}[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_dynamic_full_size_on_column_subset(B, precision):
    """n=300, N=1800, 120 tau nodes, beta=100, 8 poles: the full launch
    configuration (in bf16x3 the split W(Omega) GG(Omega) product and the
    split fused contraction), checked on a collocation matrix supported on 64
    columns."""
    import torch
    wl = synth.workload(4)
    n, N, nt = wl["n"], wl["N"], wl["n_tau"]
    tp = _pair(wl)
    rng = np.random.default_rng(4)
    cols = np.sort(rng.choice(N, size=64, replace=False))
    X = np.zeros_like(wl["X"])
    X[:, cols] = wl["X"][:, cols]
    log(f"dynamic full size {precision}, support {len(cols)} columns, n_omega={len(tp['m'])}")
    G = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    got, plan = _run(B, wl, tp, precision, X, wl["W_tau"], wl["V"], G)
    Xs = wl["X"][:, cols]
    Ws = np.ascontiguousarray(wl["W_tau"][:, cols][:, :, cols])
    Vs = wl["V"][np.ix_(cols, cols)]
    ref = om.sigma_dynamic_thc(Xs, Ws, Vs, G, G[::-1], tp["T_fwd"], tp["T_bwd"])
    err = rel_err(got, ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_real_w_product_and_asymmetric_w(B, precision):
    """The float32 and bf16x3 plans run the real W(Omega) product when the
    plan's transform of W_d(tau) has an imaginary part below float32
    resolution of its real part: a W(tau) mirror symmetric in tau on the
    120-node, beta = 100 grid (dynamic_real_w = 1).  On a coarse 20-node grid
    the same kind of W keeps an imaginary part, and a W with an added part odd
    about beta/2 always does: those keep the complex block product, as do
    float64 plans.  Every case against the oracle, which transforms W(tau) as
    it is."""
    cases = []
    for nt, beta in ((120, 100.0), (20, 40.0)):
        wl = synth.small_molecule(21, 90, nt, beta, seed=79, dynamic=True)
        odd = (wl["tau"] - beta / 2) / beta
        W_asym = wl["W_tau"] + 0.5 * odd[:, None, None] * wl["W_tau"][nt // 2][None]
        fine = nt == 120
        cases += [(wl, wl["W_tau"], fine and precision != "fp64"), (wl, W_asym, False)]
    for wl, W, want in cases:
        n, nt, beta = wl["n"], wl["n_tau"], wl["beta"]
        tp = _pair(wl)
        rng = np.random.default_rng(5)
        G = om.g_tau(wl["eps"], wl["Q"], 0.0, beta, wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
        log(f"dynamic real-W check {precision}, n_tau={nt}, mirror symmetric: {W is wl['W_tau']}")
        got, plan = _run(B, wl, tp, precision, wl["X"], W, wl["V"], G)
        assert B.sox_plan_describe(plan)["dynamic_real_w"] == (1 if want else 0)
        ref = om.sigma_dynamic_thc(wl["X"], W, wl["V"], G, G[::-1], tp["T_fwd"], tp["T_bwd"])
        err = rel_err(got, ref)
        log(f"  rel err {err:.3e}")
        assert err <= TOL[precision]


def test_dynamic_requires_transform_pair(B):
    import torch
    wl = synth.small_molecule(4, 8, 6, 5.0, seed=1, dynamic=True)
    plan = B.Plan(4, 8, wl["tau"], wl["weights"], wl["beta"], precision="fp32")
    S = torch.empty((6, 4, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SoxError) as ei:
        B.sox_sigma_dynamic(plan, dev(wl["X"]), dev(wl["W_tau"]), dev(wl["V"]),
                            dev(np.zeros((6, 4, 4))), S, ws=ws)
    assert ei.value.status == 1
