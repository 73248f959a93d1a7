"""Whole-sweep HIP graph replay and the fused-tile autotuner.

Graph replays are checked one by one against an eager plan of the same
configuration (bitwise: same kernels, same launch shapes), with eager torch
work, synchronisations and new input values between the replays.
"""
import os

import numpy as np
import pytest

from oracle import sox_mol as om
from paper_2412_18829_amd import synth
from tests.gpu_util import dev, have_gpu, host, log, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not have_gpu():
        pytest.skip("no GPU")
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("precision", ["fp32", "fp64", "bf16x3"])
def test_static_graph_replays_match_eager(B, precision):
    import torch
    wl = synth.small_molecule(24, 200, 10, 8.0, seed=41, static=True)
    n, N, nt = wl["n"], wl["N"], wl["n_tau"]
    pg = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision)
    pe = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision)
    B.sox_plan_set_graph(pg, True)
    X, W0, V = dev(wl["X"]), dev(wl["W0"]), dev(wl["V"])
    G = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    Sg = torch.empty_like(G)
    Se = torch.empty_like(G)
    wsg = pg.workspace("static")
    wse = pe.workspace("static")
    rng = np.random.default_rng(0)
    G0 = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    for rep in range(4):
        G.copy_(dev(G0 + 0.01 * rep * rng.standard_normal(G0.shape)))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # unrelated eager work between replays
        B.sox_sigma_static(pg, X, W0, V, G, Sg, ws=wsg)
        B.sox_sigma_static(pe, X, W0, V, G, Se, ws=wse)
        torch.cuda.synchronize()
        assert torch.equal(Sg, Se), f"replay {rep}"
        del junk
    assert B.sox_plan_describe(pg)["graph"] == 1


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_solid_vertex_graph_replays_match_eager(B, precision):
    """The benchmarked solid step (SOSEX_dyn in one pass, even n: the block
    form of W(Omega) GG(Omega) and the register-GG forward transform) as
    graph replays, one by one against eager runs, with new G values and
    unrelated eager work between the replays."""
    import torch
    from oracle import sox_solid as osd
    wl = synth.add_dynamic_screening_solid(synth.solid((3, 1, 1), 6, 40, 12, 10.0, seed=43),
                                           n_poles=2)
    tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=10.0, tol=1e-10)
    mk = lambda: B.Plan(wl["n"], wl["N"], wl["tau"], wl["weights"], wl["beta"],
                        precision=precision, kmesh=wl["mesh"], t_fwd=tp["T_fwd"],
                        t_bwd=tp["T_bwd"])
    pg, pe = mk(), mk()
    B.sox_plan_set_graph(pg, True)
    c = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")
    X, W, V = c(wl["X"]), c(wl["W_tau"]), c(wl["V"])
    G0 = osd.g_tau_k(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    G = c(G0)
    Sg, Se = torch.empty_like(G), torch.empty_like(G)
    wsg, wse = pg.workspace("vertex"), pe.workspace("vertex")
    for rep in range(3):
        G.copy_(c(G0 * (1.0 + 0.02 * rep)))
        junk = torch.randn(1 << 20, device="cuda") * 2.0
        B.sox_sigma_vertex(pg, "sosex_dyn", X, V, W, G, Sg, ws=wsg)
        B.sox_sigma_vertex(pe, "sosex_dyn", X, V, W, G, Se, ws=wse)
        torch.cuda.synchronize()
        assert torch.equal(Sg, Se), f"replay {rep}"
        del junk
    assert B.sox_plan_describe(pg)["graph"] == 1


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_dynamic_graph_replays_match_eager(B, precision):
    import torch
    wl = synth.small_molecule(13, 70, 24, 30.0, seed=42, dynamic=True)
    tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=14.0, tol=1e-10)
    n, N, nt = wl["n"], wl["N"], wl["n_tau"]
    mk = lambda: B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision,
                        t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
    pg, pe = mk(), mk()
    B.sox_plan_set_graph(pg, True)
    X, W, V = dev(wl["X"]), dev(wl["W_tau"]), dev(wl["V"])
    G = dev(om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]))
    Sg, Se = torch.empty_like(G), torch.empty_like(G)
    wsg, wse = pg.workspace("dynamic"), pe.workspace("dynamic")
    for rep in range(3):
        G.mul_(1.0 + 0.01 * rep)
        B.sox_sigma_dynamic(pg, X, W, V, G, Sg, ws=wsg)
        B.sox_sigma_dynamic(pe, X, W, V, G, Se, ws=wse)
        torch.cuda.synchronize()
        assert torch.equal(Sg, Se), f"replay {rep}"


def test_autotuner_and_cache(B, tmp_path, monkeypatch):
    import torch
    wl = synth.small_molecule(32, 260, 6, 8.0, seed=43)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SOX_AUTOTUNE", "1")
    monkeypatch.setenv("SOX_TUNE_CACHE", str(cache))
    p1 = B.Plan(wl["n"], wl["N"], wl["tau"], wl["weights"], wl["beta"], precision="fp32")
    d1 = B.sox_plan_describe(p1)
    log(f"autotune {d1}")
    assert len(d1["tune_ms_per_tau"]) >= 2 and d1["tune_from_cache"] == 0
    best = min(d1["tune_ms_per_tau"], key=lambda t: t[1])[0]
    assert d1["fused_cfg"] == best
    p2 = B.Plan(wl["n"], wl["N"], wl["tau"], wl["weights"], wl["beta"], precision="fp32")
    d2 = B.sox_plan_describe(p2)
    assert d2["tune_from_cache"] == 1 and d2["fused_cfg"] == best
    G = dev(om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"]))
    S = torch.empty_like(G)
    B.sox_sigma_bare(p2, dev(wl["X"]), dev(wl["V"]), G, S)
    torch.cuda.synchronize()
    Gr = host(G)
    ref = om.sigma_static_thc(wl["X"], wl["V"], wl["V"], Gr, Gr[::-1])
    assert rel_err(host(S), ref) <= 1e-6


@pytest.mark.parametrize("entry", ["bare", "dynamic"])
def test_solid_graph_replays_match_eager(B, entry):
    """k-point plans (3x1x1 mesh): every launch of a sweep (all tau nodes,
    all momentum pairs) replayed as one graph equals the eager sweep."""
    import torch
    wl = synth.solid((3, 1, 1), 9, 40, 10, 10.0, seed=43)
    tp = None
    if entry == "dynamic":
        synth.add_dynamic_screening_solid(wl, n_poles=2)
        tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=10.0, tol=1e-10)
    n, N, nt, nk = wl["n"], wl["N"], wl["n_tau"], wl["nk"]
    extra = dict(t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"]) if tp is not None else {}
    mk = lambda: B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp32",
                        kmesh=wl["mesh"], **extra)
    pg, pe = mk(), mk()
    B.sox_plan_set_graph(pg, True)
    c = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")
    X, V = c(wl["X"]), c(wl["V"])
    W = c(wl["W_tau"]) if tp is not None else None
    G = torch.empty((nk, nt, n, n), dtype=torch.complex128, device="cuda")
    Sg = torch.empty_like(G)
    Se = torch.empty_like(G)
    wsg, wse = pg.workspace(entry), pe.workspace(entry)
    rng = np.random.default_rng(1)
    from oracle import sox_solid as osd
    G0 = osd.g_tau_k(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    log(f"solid graph {entry}")
    for rep in range(3):
        G.copy_(c(G0 + 0.01 * rep * (rng.standard_normal(G0.shape) + 0j)))
        junk = torch.randn(1 << 20, device="cuda") * 2.0
        if entry == "bare":
            B.sox_sigma_bare(pg, X, V, G, Sg, ws=wsg)
            B.sox_sigma_bare(pe, X, V, G, Se, ws=wse)
        else:
            B.sox_sigma_dynamic(pg, X, W, V, G, Sg, ws=wsg)
            B.sox_sigma_dynamic(pe, X, W, V, G, Se, ws=wse)
        torch.cuda.synchronize()
        assert torch.equal(Sg, Se), f"replay {rep}"
        del junk


def _check_autotune(desc):
    """Every candidate timed, the plan left on the fastest one."""
    at = desc["autotune"]
    assert len(at) >= 2 and desc["autotune_cached"] == 0, desc
    assert all(r["ms"] > 0 for r in at)
    best = min(at, key=lambda r: r["ms"])
    return best


def test_autotuned_bf16x3_molecule_vs_oracle(B, tmp_path, monkeypatch):
    """sox_autotune on the caller's operands (split precision: the LDS-staged
    and direct-load fused configurations, v splits), then the tuned plan
    against the oracle at the split-precision bound; a second plan of the
    same shape takes the cached choice without timing."""
    import torch
    cache = tmp_path / "auto.txt"
    monkeypatch.setenv("SOX_TUNE_CACHE", str(cache))
    n, N, nt = 40, 200, 4
    wl = synth.small_molecule(n, N, nt, 7.0, seed=240, static=True)
    Gr = om.g_tau(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    mk = lambda: B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="bf16x3")
    X, W0, V, G = dev(wl["X"]), dev(wl["W0"]), dev(wl["V"]), dev(Gr)
    S = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    p1 = mk()
    B.sox_autotune(p1, "static", X, W0, V, G, S)
    d1 = B.sox_plan_describe(p1)
    log(f"autotuned bf16x3 molecule: {d1['autotune']}")
    best = _check_autotune(d1)
    assert (d1["fused_cfg"], d1["fused_vsplit"]) == (best["fused_cfg"], best["fused_vsplit"])
    assert {r["fused_cfg"] for r in d1["autotune"]} >= {8}
    ref = om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr, Gr[::-1])
    err_tune = rel_err(host(S), ref)      # the last candidate's Sigma
    B.sox_sigma_static(p1, X, W0, V, G, S)
    torch.cuda.synchronize()
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e} (last candidate {err_tune:.3e})")
    assert err <= 1e-4 and err_tune <= 1e-4
    p2 = mk()
    B.sox_autotune(p2, "static", X, W0, V, G, S)
    d2 = B.sox_plan_describe(p2)
    assert d2["autotune_cached"] == 1 and d2["autotune"] == []
    assert (d2["fused_cfg"], d2["fused_vsplit"]) == (d1["fused_cfg"], d1["fused_vsplit"])


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_autotuned_solid_dynamic_vs_oracle(B, precision, tmp_path, monkeypatch):
    """k-point plan (3x1x1 mesh, even n: the register-GG transforms and the
    block-form W(Omega) GG(Omega)): sox_autotune over the tau slab of the
    B, C, D steps and the pair slab of the transforms, then the tuned plan
    against the oracle's eq:GG chain."""
    import torch
    from oracle import sox_solid as osd
    monkeypatch.setenv("SOX_TUNE_CACHE", str(tmp_path / "auto.txt"))
    wl = synth.add_dynamic_screening_solid(synth.solid((3, 1, 1), 6, 40, 12, 10.0, seed=47),
                                           n_poles=2)
    tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=10.0, tol=1e-10)
    plan = B.Plan(wl["n"], wl["N"], wl["tau"], wl["weights"], wl["beta"], precision=precision,
                  kmesh=wl["mesh"], t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
    c = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")
    G0 = osd.g_tau_k(wl["eps"], wl["Q"], 0.0, wl["beta"], wl["tau"])
    X, W, V, G = c(wl["X"]), c(wl["W_tau"]), c(wl["V"]), c(G0)
    S = torch.empty_like(G)
    B.sox_autotune(plan, "dynamic", X, W, V, G, S)
    d = B.sox_plan_describe(plan)
    log(f"autotuned solid dynamic {precision}: {d['autotune']}")
    best = _check_autotune(d)
    assert (d["solid_dyn_tau_slab"], d["solid_dyn_pair_slab"]) == (best["tau_slab"], best["pair_slab"])
    assert len({(r["tau_slab"], r["pair_slab"]) for r in d["autotune"]}) >= 2
    B.sox_sigma_dynamic(plan, X, W, V, G, S)
    torch.cuda.synchronize()
    tables = (wl["kvecs"], wl["kdiff"], wl["ksum"], wl["kneg"])
    ref = osd.sigma_solid_dynamic_thc(wl["X"], wl["W_tau"], wl["V"], G0, tp["T_fwd"], tp["T_bwd"],
                                      tables)
    err = rel_err(host(S), ref)
    log(f"  rel err {err:.3e}")
    assert err <= (1e-6 if precision == "fp32" else 1e-4)
