"""GPU parity of the static SOX path (bare and statically screened) against
the FP64 oracle, through the C ABI.

Tolerances (max |diff| / max |oracle|): FP64 path 1e-12, FP32 path 1e-6
(the stated FP32 target).  Sizes span several fused tiles and ragged tails
(n not a multiple of 16, N not a multiple of 64).
"""
import numpy as np
import pytest

from oracle import sox_mol as om
from paper_2412_18829_amd import synth
from tests.gpu_util import dev, have_gpu, host, log, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def B():
    if not have_gpu():
        pytest.skip("no GPU")
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


def _plan(B, wl, precision):
    return B.Plan(wl["n"], wl["N"], wl["tau"], wl["weights"], wl["beta"], precision=precision)


def _gpu_g(B, plan, wl):
    import torch
    G = torch.empty((wl["n_tau"], wl["n"], wl["n"]), dtype=torch.float64, device="cuda")
    B.sox_build_g_tau(plan, dev(wl["Q"]), dev(wl["eps"]), wl["mu"], G)
    return G


def test_g_tau_build_matches_oracle(B):
    for c in (1, 2):
        wl = synth.workload(c)
        log(f"g_tau workload {c}")
        plan = _plan(B, wl, "fp64")
        G = host(_gpu_g(B, plan, wl))
        ref = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
        assert np.abs(G - ref).max() <= 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bare_workload1_vs_bruteforce(B, precision):
    import torch
    wl = synth.workload(1)
    log(f"bare workload1 {precision}")
    plan = _plan(B, wl, precision)
    G = _gpu_g(B, plan, wl)
    S = torch.empty_like(G)
    B.sox_sigma_bare(plan, dev(wl["X"]), dev(wl["V"]), G, S)
    torch.cuda.synchronize()
    Gr = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
    E = om.eri(wl["X"], wl["V"])
    ref = om.sigma_static_eri(E, E, Gr, om.g_mirror(Gr))
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(13, 50, 6), (17, 130, 5), (40, 200, 4), (3, 7, 1), (5, 70, 2)])
def test_static_ragged_general_G(B, precision, shape):
    """U1 != U2, a general (non-symmetric) G, ragged n and N, several tiles."""
    import torch
    n, N, nt = shape
    log(f"static ragged {shape} {precision}")
    wl = synth.small_molecule(n, N, nt, 7.0, seed=100 + n, static=True)
    rng = np.random.default_rng(n)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    plan = _plan(B, wl, precision)
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_static(plan, dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr), S)
    torch.cuda.synchronize()
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bare_workload2_full_size(B, precision):
    """n=64, N=384, 64 tau nodes: the benchmarked configuration."""
    import torch
    wl = synth.workload(2)
    log(f"bare workload2 {precision}")
    plan = _plan(B, wl, precision)
    G = _gpu_g(B, plan, wl)
    S = torch.empty_like(G)
    B.sox_sigma_bare(plan, dev(wl["X"]), dev(wl["V"]), G, S)
    torch.cuda.synchronize()
    Gr = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
    ref = om.sigma_static_thc(wl["X"], wl["V"], wl["V"], Gr, om.g_mirror(Gr))
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL[precision]
    # energy through the ABI against the oracle's
    e = B.sox_energy_gm(plan, S, G)
    e_ref = om.energy_gm(ref, om.g_mirror(Gr), wl["weights"])
    assert abs(e - e_ref) <= 10 * TOL[precision] * abs(e_ref)
    # the device-output form: the same value, queued twice without a sync
    E = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    B.sox_energy_gm_device(plan, S, G, E[0])
    B.sox_energy_gm_device(plan, S, G, E[1])
    torch.cuda.synchronize()
    assert host(E).tolist() == [e, e]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_static_workload3_full_size_sampled_tau(B, precision):
    """n=200, N=1200, 100 tau nodes, beta=100, W(0) = V + V Pi V: the full
    launch configuration (all tau nodes in one slab; in the split path the
    A operand holds more than 2^32 elements, so its flat launches stride).
    The static Sigma(tau) depends only on G(tau) and G(beta - tau), so the
    oracle evaluates two sampled nodes on their own."""
    import torch
    wl = synth.workload(3)
    log(f"static workload3 {precision}")
    plan = _plan(B, wl, precision)
    G = _gpu_g(B, plan, wl)
    S = torch.empty_like(G)
    B.sox_sigma_static(plan, dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), G, S)
    torch.cuda.synchronize()
    got = host(S)
    assert np.isfinite(got).all()
    Gr = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
    Gb = om.g_mirror(Gr)
    ts = [0, wl["n_tau"] // 2 + 1]
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr[ts], Gb[ts])
    err = rel_err(got[ts], ref)
    log(f"  rel err {err:.3e} at tau nodes {ts}")
    assert err <= {"fp32": 1e-6, "bf16x3": 1e-4}[precision]


def test_bare_equals_static_with_same_interaction(B):
    import torch
    wl = synth.small_molecule(20, 96, 6, 9.0, seed=5)
    plan = _plan(B, wl, "fp64")
    G = _gpu_g(B, plan, wl)
    X, V = dev(wl["X"]), dev(wl["V"])
    S1 = torch.empty_like(G)
    S2 = torch.empty_like(G)
    B.sox_sigma_bare(plan, X, V, G, S1)
    B.sox_sigma_static(plan, X, V, V, G, S2)
    torch.cuda.synchronize()
    assert rel_err(host(S1), host(S2)) <= 1e-14


def test_tau_slabs_match_single_slab(B, monkeypatch):
    """A workspace budget that forces several tau slabs gives the same Sigma
    (to the float32 bound: the split of the v sum over workgroups follows the
    slab's tile count, so the summation order may differ)."""
    import torch
    wl = synth.small_molecule(24, 120, 9, 9.0, seed=6)
    plan1 = _plan(B, wl, "fp32")
    monkeypatch.setenv("SOX_WS_BUDGET_MB", "1")
    plan2 = _plan(B, wl, "fp32")
    G = _gpu_g(B, plan1, wl)
    X, V = dev(wl["X"]), dev(wl["V"])
    S1 = torch.empty_like(G)
    S2 = torch.empty_like(G)
    B.sox_sigma_bare(plan1, X, V, G, S1)
    B.sox_sigma_bare(plan2, X, V, G, S2)
    torch.cuda.synchronize()
    assert plan2.workspace_size("bare") < plan1.workspace_size("bare")
    assert rel_err(host(S2), host(S1)) <= 1e-6


def test_workspace_too_small_is_an_error(B):
    import torch
    wl = synth.small_molecule(8, 32, 4, 5.0, seed=2)
    plan = _plan(B, wl, "fp32")
    G = _gpu_g(B, plan, wl)
    S = torch.empty_like(G)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SoxError) as ei:
        B.sox_sigma_bare(plan, dev(wl["X"]), dev(wl["V"]), G, S, ws=small)
    assert ei.value.status == 4


@pytest.mark.parametrize("shape", [(13, 50, 6), (40, 200, 4), (64, 384, 8)])
def test_bf16x3_static_vs_oracle(B, shape):
    """Split precision (x = hi + lo in bf16, three bf16 MFMA products per
    product, float32 accumulation): max relative error <= 1e-4 before any
    refinement."""
    import torch
    n, N, nt = shape
    log(f"bf16x3 static {shape}")
    wl = synth.small_molecule(n, N, nt, 7.0, seed=200 + n, static=True)
    rng = np.random.default_rng(n)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    plan = _plan(B, wl, "bf16x3")
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_static(plan, dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr), S)
    torch.cuda.synchronize()
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("shape,cfg", [((13, 50, 6), 8), ((40, 200, 4), 8), ((70, 300, 5), 8),
                                       ((64, 384, 3), 8), ((40, 200, 4), 6), ((70, 300, 5), 7)])
def test_bf16x3_kernels_vs_oracle(B, shape, cfg, monkeypatch):
    """The LDS-staged split-precision kernel (128 x 128 workgroup tile,
    32-deep k stages; config 8, the default) on one, two and three k stages
    per v, padded P/R tiles and the v-split its occupancy selects; and the
    direct-load kernels (configs 6 and 7)."""
    import torch
    monkeypatch.setenv("SOX_FUSED_CFG", str(cfg))
    n, N, nt = shape
    log(f"bf16x3 static {shape} config {cfg}")
    wl = synth.small_molecule(n, N, nt, 7.0, seed=300 + n, static=True)
    rng = np.random.default_rng(n + 1)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    plan = _plan(B, wl, "bf16x3")
    info = B.sox_plan_describe(plan)
    assert info["fused_cfg"] == cfg
    log(f"  v split {info['fused_vsplit']}")
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_static(plan, dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr), S)
    torch.cuda.synchronize()
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("shape", [(13, 50, 6), (40, 200, 4), (70, 300, 5), (64, 384, 3)])
def test_fp32_lds_kernel_vs_oracle(B, shape, monkeypatch):
    """The LDS-staged float32 fused kernel (config 9, 128 x 128 workgroup
    tile, 16-deep k stages) against the oracle at the float32 tolerance."""
    import torch
    monkeypatch.setenv("SOX_FUSED_CFG", "9")
    n, N, nt = shape
    log(f"fp32 lds static {shape}")
    wl = synth.small_molecule(n, N, nt, 7.0, seed=400 + n, static=True)
    rng = np.random.default_rng(n + 2)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    plan = _plan(B, wl, "fp32")
    info = B.sox_plan_describe(plan)
    assert info["fused_cfg"] == 9
    log(f"  v split {info['fused_vsplit']}")
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_static(plan, dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr), S)
    torch.cuda.synchronize()
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("precision,wg", [("fp32", 1), ("fp32", 3), ("bf16x3", 3), ("fp32", 7)])
@pytest.mark.parametrize("shape", [(13, 50, 6), (40, 200, 4)])
def test_dense_multi_tile_workgroups_vs_oracle(B, shape, precision, wg, monkeypatch):
    """The A step and U-contraction GEMM with several output tiles per
    workgroup (at most `wg` workgroups: every tile in one, or several with a
    short last one) against the oracle; the result matches the default
    launch to rounding."""
    import torch
    n, N, nt = shape
    log(f"dense multi-tile {shape} {precision} wg={wg}")
    wl = synth.small_molecule(n, N, nt, 7.0, seed=500 + n, static=True)
    rng = np.random.default_rng(n + 3)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]) + 0.05 * rng.standard_normal((nt, n, n))
    args = (dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr))
    S0 = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    B.sox_sigma_static(_plan(B, wl, precision), *args, S0)
    monkeypatch.setenv("SOX_DENSE_WG", str(wg))
    S = torch.empty_like(S0)
    B.sox_sigma_static(_plan(B, wl, precision), *args, S)
    torch.cuda.synchronize()
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}, vs default launch {rel_err(host(S), host(S0)):.3e}")
    assert err <= {"fp32": TOL["fp32"], "bf16x3": 1e-4}[precision]
    assert rel_err(host(S), host(S0)) <= 1e-12


@pytest.mark.parametrize("precision,n,expect", [("fp32", 512, 3), ("bf16x3", 736, 7)])
def test_lds_kernel_offset_limit_falls_back(B, precision, n, expect):
    """Past the LDS-staged kernel's 32-bit panel offsets (NP nP^2 element
    bytes >= 2^32) the plan picks the direct-load kernel of the same
    precision."""
    tau, w = synth.chebyshev_tau_grid(4, 10.0)
    plan = B.Plan(n, 4100, tau, w, 10.0, precision=precision)
    info = B.sox_plan_describe(plan)
    log(f"n={n} N=4100 {precision}: fused config {info['fused_cfg']} (nP {info['nP']}, NP {info['NP']})")
    assert info["fused_cfg"] == expect
    small = B.Plan(64, 384, tau, w, 10.0, precision=precision)
    assert B.sox_plan_describe(small)["fused_cfg"] in (8, 9)
