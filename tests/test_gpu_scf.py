"""The library's self-consistent loop (sox_scf) against the oracle's
(oracle/scf.py), each on its own IR grid (library: sox_ir_grid_fermion and
sox_ir_grid; oracle: oracle/ir_grid.py), for one spin channel of a small
molecule (n = 6, N = 14, beta = 20, Lambda = 300, eps = 1e-10: 40 tau nodes,
30 fermionic samples), three electrons.

* Hartree-Fock only, GW with a fixed eight-pole W_d (bit 0), and GW plus the
  bare SOX term (bits 0 and 1, FP64 plan).
* Compared: the converged G(tau) (1e-7: the loops stop at max |dG| <= 1e-8,
  and the two grids differ by about 1e-6 of T_fwd), E_inf and E_dyn (1e-7
  relative), the chemical potential (1e-5: in a gap N(mu) is flat, so mu is
  determined only to about that), Tr gamma = N through the library's G.
* The Dyson inversions past the LDS size (n = 100, held in device memory):
  three iterations of the GW loop against the oracle's three (G 1e-7).
* The LDS and device-memory forms of the Dyson inversion on the same
  n = 64 loop (SOX_SCF_DYSON_IN_MEMORY=1 forces the latter): the same
  iteration count, G and mu to 1e-10 (pivots and rounding order agree; the
  bracketing search may land on a different mu in its last step).
"""
import numpy as np
import pytest

from oracle import ir_grid as ir
from oracle import scf as osc
from paper_2412_18829_amd import synth
from tests.gpu_util import dev, have_gpu, host, log

pytestmark = pytest.mark.gpu

BETA, LAM, EPS = 20.0, 300.0, 1e-10
N_ELEC = 3.0


@pytest.fixture(scope="module")
def B():
    if not have_gpu():
        pytest.skip("no GPU")
    from paper_2412_18829_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def system():
    of, ob = ir.ir_fermion(BETA, LAM, EPS), ir.ir_grid(BETA, LAM, EPS)
    wl = synth.small_molecule(6, 14, len(of["tau"]), BETA, seed=13)
    wl["tau"] = of["tau"]
    synth.add_dynamic_screening(wl)
    h = wl["Q"] @ np.diag(wl["eps"]) @ wl["Q"].T
    return wl, h, of, ob


def _w_on(wl, tau):
    return sum(a * synth.periodic_bosonic_pole(tau, BETA, w)[:, None, None] * S[None]
               for w, a, S in zip(wl["pole_w"], wl["pole_a"], wl["pole_S"]))


@pytest.mark.parametrize("terms", [(), ("gw",), ("gw", "sox")], ids=["hf", "gw", "gw+sox"])
def test_scf_vs_oracle(B, system, terms):
    import torch
    wl, h, of, ob = system
    ref = osc.scf(wl["X"], wl["V"], wl["W_tau"], h, N_ELEC, BETA, of, ob["weights"],
                  terms=terms, tol=1e-8, max_iter=300)
    lf = B.sox_ir_grid_fermion(BETA, LAM, EPS)
    lb = B.sox_ir_grid(BETA, LAM, EPS)
    n, N, nt = wl["n"], wl["N"], len(lf["tau"])
    log(f"scf {terms or 'hf'}: n={n} N={N} nt={nt} n_nu={len(lf['n'])}; oracle "
        f"{ref['iterations']} iterations, mu {ref['mu']:.10f}")
    plan = B.Plan(n, N, lf["tau"], lb["weights"], BETA, "fp64")
    G = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    out = B.sox_scf(plan, lf, dev(wl["X"]), dev(wl["V"]), dev(_w_on(wl, lf["tau"])), dev(h),
                    N_ELEC, G, terms=terms, tol=1e-8, max_iter=300)
    torch.cuda.synchronize()
    Gh = host(G)
    log(f"  library {out['iterations']} iterations, mu {out['mu']:.10f}, delta {out['delta']:.1e}, "
        f"E_inf {out['e_inf']:.12f} ({ref['e_inf']:.12f}), E_dyn {out['e_dyn']:.12e} "
        f"({ref['e_dyn']:.12e}), max |dG| {np.abs(Gh - ref['G']).max():.1e}")
    assert out["delta"] <= 1e-8
    assert np.abs(Gh - ref["G"]).max() <= 1e-7
    assert abs(out["mu"] - ref["mu"]) <= 1e-5
    assert abs(out["e_inf"] - ref["e_inf"]) <= 1e-7 * abs(ref["e_inf"])
    if terms:
        assert abs(out["e_dyn"] - ref["e_dyn"]) <= 1e-7 * abs(ref["e_dyn"])
    gam = -np.einsum("i,iqp->pq", lf["t_beta"], Gh)
    assert abs(np.trace(gam) - N_ELEC) <= 1e-8


def _loop(B, wl, h, n_elec, terms, tol, max_iter):
    import torch
    lf = B.sox_ir_grid_fermion(BETA, LAM, EPS)
    lb = B.sox_ir_grid(BETA, LAM, EPS)
    n, N, nt = wl["n"], wl["N"], len(lf["tau"])
    plan = B.Plan(n, N, lf["tau"], lb["weights"], BETA, "fp64")
    G = torch.empty((nt, n, n), dtype=torch.float64, device="cuda")
    out = B.sox_scf(plan, lf, dev(wl["X"]), dev(wl["V"]), dev(_w_on(wl, lf["tau"])), dev(h),
                    n_elec, G, terms=terms, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    return out, host(G)


def _molecule(n, N, seed):
    of = ir.ir_fermion(BETA, LAM, EPS)
    wl = synth.small_molecule(n, N, len(of["tau"]), BETA, seed=seed)
    wl["tau"] = of["tau"]
    synth.add_dynamic_screening(wl)
    h = wl["Q"] @ np.diag(wl["eps"]) @ wl["Q"].T
    return wl, h, of


def test_scf_dyson_in_device_memory_vs_oracle(B):
    wl, h, of = _molecule(100, 120, 17)
    ob = ir.ir_grid(BETA, LAM, EPS)
    ref = osc.scf(wl["X"], wl["V"], wl["W_tau"], h, 50.0, BETA, of, ob["weights"], terms=("gw",),
                  tol=1e-300, max_iter=3)
    log(f"scf gw n=100 N=120: three iterations; oracle mu {ref['mu']:.10f}")
    out, Gh = _loop(B, wl, h, 50.0, ("gw",), 1e-300, 3)
    err = np.abs(Gh - ref["G"]).max()
    log(f"  library {out['iterations']} iterations, mu {out['mu']:.10f}, max |dG| {err:.1e}")
    assert out["iterations"] == 3
    assert err <= 1e-7
    assert abs(out["mu"] - ref["mu"]) <= 1e-5


def test_scf_dyson_lds_and_device_memory_agree(B, monkeypatch):
    wl, h, _ = _molecule(64, 96, 19)
    a, Ga = _loop(B, wl, h, 32.0, ("gw",), 1e-8, 100)
    monkeypatch.setenv("SOX_SCF_DYSON_IN_MEMORY", "1")
    b, Gb = _loop(B, wl, h, 32.0, ("gw",), 1e-8, 100)
    log(f"scf gw n=64: LDS {a['iterations']} iterations mu {a['mu']:.12f}; device memory "
        f"{b['iterations']} iterations mu {b['mu']:.12f}; max |dG| {np.abs(Ga - Gb).max():.1e}")
    assert a["iterations"] == b["iterations"]
    assert np.abs(Ga - Gb).max() <= 1e-10
    assert abs(a["mu"] - b["mu"]) <= 1e-10
