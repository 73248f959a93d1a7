#!/usr/bin/env python3
"""Benchmark of the SOX self-energy hot path on one MI355X.

One step = one pass of the whole path over the workload: G(tau) synthesis
from the Fock eigenbasis, the U-contraction, the half projections, the A
step (or, for the dynamic interaction, GG -> FT -> W(Omega) GG(Omega) -> IFT),
the B, C -> D contraction, the back-transform to orbitals (all tau nodes and
momenta: one "sweep") and the Galitskii-Migdal energy (queued into device
memory each step, read after the timed region).  Inputs are seeded and
synthetic and resident in HBM before the timed region.

The default workload (5) is the largest: the 3x3x3 k-point solid, n=52 and
N=400 per k, 100 tau nodes, beta=100, with an 8-pole W^q(tau); its step is
the bare plus dynamically screened SOX self-energy SOX(V,V) + SOX(W_d(tau),V)
in one pass (sox_sigma_vertex, SOSEX_dyn), in bf16x3 by default.
--workload selects the molecules (1, 2: bare n=8 / n=64; 3: static
screening n=200 N=1200; 4: dynamic screening n=300 N=1800).

Prints ONE JSON line.  `value` is sweeps/s of the chosen precision path; the
float64 path is timed on the same inputs for the mixed-vs-FP64 comparison,
max_rel_err is taken against the FP64 oracle (for the solid: a sweep of the
same launch configuration on a column-supported collocation matrix, against
the oracle values stored by tests/golden/make_c5_reference.py), the oracle
is timed on the host as a baseline on a bounded sample, and the dominant
kernel's roofline fraction is measured with HIP events on the stream it runs
on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2516.6}
HBM_PEAK_GBS = 8000.0
DTYPE_NAME = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}
METRIC = "SOX Sigma(all tau) sweeps/sec + TFLOP/s vs MFMA peak; mixed vs FP64 path at stated err"
WORKLOADS = {
    1: ("molecule bare SOX n=8 N=24 n_tau=16 beta=10", "bare"),
    2: ("molecule bare SOX n=64 N=384 n_tau=64 beta=50", "bare"),
    3: ("molecule static SOX n=200 N=1200 n_tau=100 beta=100, W0 = V + V Pi V", "static"),
    4: ("molecule dynamic SOX n=300 N=1800 n_tau=120 beta=100, 8-pole W(tau)", "dynamic"),
    5: ("solid SOX(V,V) + SOX(W_d(tau),V) 3x3x3 k-mesh n=52 N=400 n_tau=100 beta=100, "
        "8-pole W^q(tau)", "solid"),
}
ENTRY = {"bare": "sox_sigma_bare", "static": "sox_sigma_static", "dynamic": "sox_sigma_dynamic",
         "solid": "sox_sigma_vertex (SOSEX_dyn, bare and dynamic terms in one pass)"}
GOLDEN_C5 = os.path.join(ROOT, "tests", "golden", "c5_sosex_dyn_support8.npz")
# dominant kernel per kind: (profiling stage, kernel name)
# the fused kernel each molecular configuration launches (rocprofv3 names)
FUSED_KERNEL = {0: "fused_bcd_kernel<float|double, 32, 32>", 3: "fused_bcd_kernel<float, 64, 64>",
                6: "fused_bcd_bf16x3_kernel<32, 32>", 7: "fused_bcd_bf16x3_kernel<64, 32>",
                8: "fused_bcd_lds_kernel<0, 2> (bf16 x 3)", 9: "fused_bcd_lds_kernel<1, 2> (float32)"}
DOMINANT = {"bare": ("fused", "fused_bcd_kernel"), "static": ("fused", "fused_bcd_kernel"),
            "dynamic": ("fused", "fused_bcd_kernel"), "solid": ("kbc", "cgemm_panel_kernel")}


_T_START = time.perf_counter()
_last_note = [0.0]


def note(msg: str, every: float = 0.0) -> None:
    """Progress line on stderr (stdout carries only the JSON line); with
    `every`, at most one such line per that many seconds."""
    now = time.perf_counter()
    if every and now - _last_note[0] < every:
        return
    _last_note[0] = now
    print(f"[bench {now - _T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def flops_per_sweep(n: int, N: int, nt: int, kind: str = "bare", n_omega: int = 0,
                    nk: int = 1) -> dict:
    """Algorithmic FLOPs of one sweep, by stage (the paper's step costs).

    Complex products count 8 real FLOPs per multiply-add.  The U-contraction
    is reported but excluded from the sweep total by the caller (it is set up
    once per X and U)."""
    if kind == "solid":
        # SOX(V,V) + SOX(W_d,V) in one pass: the bare A step and its product
        # with G(tau) join the dynamic chain's A(tau); B, C, D and the
        # back-transform run once (complex multiply-adds: 8 real FLOPs)
        np2 = nk * nk
        nw = n_omega
        return {
            "gbuild": nk * nt * 8.0 * n ** 3,
            "utensor": np2 * 8.0 * N * N * n * n,
            "project": nt * nk * 3 * 8.0 * N * n * n,
            "astep": nt * np2 * 2 * 8.0 * N * n ** 3,
            "gg_ft": 2 * 8.0 * nw * nt * nk * N * N + nt * np2 * N * n * n * 6.0
                     + 2 * 8.0 * nw * nt * np2 * N * n * n,
            "wgemm": 2 * nw * np2 * 8.0 * N * N * n * n,
            "ift": 8.0 * nt * 2 * nw * np2 * N * n * n,
            "kbc": nt * np2 * 2 * 8.0 * N * N * n * n,
            "kd": nt * nk ** 3 * 8.0 * N * N * n,
            "back": nt * nk * 8.0 * (N * N * n + N * n * n),
            "energy": nk * nt * 8.0 * n * n,
        }
    f = {
        "gbuild": nt * 2.0 * n ** 3,
        "utensor": (2 if kind == "static" else 1) * 2.0 * N * N * n * n,
        "project": nt * 4.0 * N * n * n,
        "fused": nt * (4.0 * N * N * n * n + 2.0 * N * N * n),
        "back": nt * (2.0 * N * N * n + 2.0 * N * n * n),
        "energy": nt * 2.0 * n * n,
    }
    if kind == "dynamic":
        f["utensor"] = 2.0 * N * N * n * n
        f["gg_ft"] = nt * N * n * n + 4.0 * n_omega * nt * N * n * n
        # a real W(Omega) times a complex GG(Omega): 4 N^2 n^2 per frequency
        f["wgemm"] = n_omega * 4.0 * N * N * n * n
        f["ift"] = 4.0 * n_omega * nt * N * n * n
    else:
        f["astep"] = nt * 2.0 * N * n ** 3
    return f


def kernel_source_hash(kind: str = "bare") -> str:
    """Hash of the dominant kernel's source: the fused kernels' files for
    molecules; for solids the split panel kernel and its launcher (the text
    between their markers in sox_complex.hpp) and the shared helpers."""
    csrc = os.path.join(ROOT, "paper_2412_18829_amd", "csrc")
    h = hashlib.sha256()
    if kind == "solid":
        src = open(os.path.join(csrc, "sox_complex.hpp")).read()
        a = src.index("template <bool FIXA, int NW, bool DMA>")
        b = src.index("#undef SOX_PANEL3", a)
        h.update(src[a:b].encode())
        with open(os.path.join(csrc, "sox_common.hpp"), "rb") as fh:
            h.update(fh.read())
        return h.hexdigest()[:16]
    for f in ("sox_fused.hpp", "sox_fused_lds.hpp", "sox_common.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def solid_bc_bytes(n: int, N: int, nt: int, nk: int, ts: int) -> float:
    """Algorithmic HBM bytes of one sweep's B and C products (complex64, the
    dynamic chain's tau slabs of ts nodes per orbital v): every output
    written once, every distinct operand read once per launch.
      B[l][pair] = A(tau_l)[pair] X^{k_v - q1}^T: A read once, the n_k X panels
      C[l][pair] = GwPt^{k_w}(tau_l) Ut2[pair][v]^T: the n_k GwPt panels of each
      node, the Ut2 rows of v"""
    np2, e = nk * nk, 8.0
    slabs = (nt + ts - 1) // ts
    writes = 2 * nt * np2 * N * N * e
    reads_b = nt * np2 * N * n * e + slabs * nk * N * n * e
    reads_c = nt * nk * N * n * e + slabs * np2 * N * n * e
    return n * (writes + reads_b + reads_c)


def read_traffic(workload: int, precision: str, kind: str = "bare"):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when absent or taken on a different
    kernel source."""
    stem = "cgemm_panel_bf16x3" if kind == "solid" else "fused_bcd"
    path = os.path.join(ROOT, "profiles", f"{stem}_w{workload}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash(kind):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_oracle_baseline(wl: dict, kind: str, budget_s: float):
    """Time the FP64 oracle on the host.  Bare molecules: whole sweeps (G(tau)
    synthesis + THC chain) until the budget is spent.  Static molecules:
    single tau nodes (Sigma(tau_j) needs only G(tau_j) and G(beta - tau_j);
    every call redoes the U-contraction), scaled to sweeps/s.  Dynamic
    molecules and solids: not run (one oracle sweep needs the whole GG(tau)
    array on the host, or minutes per tau node).  Returns (record, Sigma of
    the last timed sweep or None); that Sigma is the error reference of the
    bare workloads."""
    from oracle import sox_mol as om
    nt = wl["n_tau"]
    if kind == "bare":
        sweeps = 0
        c0 = time.perf_counter()
        while True:
            Gr = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
            sig = om.sigma_static_thc(wl["X"], wl["V"], wl["V"], Gr, om.g_mirror(Gr))
            sweeps += 1
            if time.perf_counter() - c0 >= budget_s:
                break
        sec = time.perf_counter() - c0
        return ({"value": sweeps / sec, "unit": "sweeps/s", "cores": blas_threads(), "kind": "oracle",
                 "sample": f"{sweeps} full sweep(s) ({nt} tau nodes) of the FP64 numpy THC route "
                           "(G(tau) synthesis + static SOX chain), same workload and seed"}, sig)
    if kind == "static":
        Gr = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
        nodes = 0
        c0 = time.perf_counter()
        while nodes < nt:
            j = nodes
            om.sigma_static_thc(wl["X"], wl["W0"], wl["V"], Gr[[j]], Gr[[nt - 1 - j]])
            nodes += 1
            if time.perf_counter() - c0 >= budget_s:
                break
        sec = time.perf_counter() - c0
        return ({"value": nodes / nt / sec, "unit": "sweeps/s", "cores": blas_threads(),
                 "kind": "oracle",
                 "sample": f"{nodes} of {nt} tau nodes of the FP64 numpy THC route (U-contraction "
                           "redone per node), scaled to whole sweeps; same workload and seed"}, None)
    return None, None


GW_CALLS = 5
# the IR grid leg: Lambda = beta * omega_max of the workloads' transform pair
IR_OMEGA_MAX = 14.0
IR_EPS = 1e-10
# the self-consistent loop leg: one spin channel of a synthetic molecule
SCF_N, SCF_NTHC, SCF_BETA, SCF_LAMBDA, SCF_SEED, SCF_TOL = 64, 384, 50.0, 500.0, 7, 1e-8

# workspace budget of the timed k-mesh plans (the main run and the IR-grid
# leg): 192 GiB of the GPU's 288 GB, against the library's default cap of
# 64 GiB, so that the tuner can take 16-node tau slabs; a budget set by the
# caller (SOX_WS_BUDGET_MB) is kept.  The float64 comparison sweep keeps the
# library default.
SOLID_WS_BUDGET_MB = 196608


class ws_budget:
    def __init__(self, active: bool):
        self.active = active and "SOX_WS_BUDGET_MB" not in os.environ

    def __enter__(self):
        if self.active:
            os.environ["SOX_WS_BUDGET_MB"] = str(SOLID_WS_BUDGET_MB)
        return self

    def __exit__(self, *exc):
        if self.active:
            del os.environ["SOX_WS_BUDGET_MB"]
        return False


def gw_flops(n: int, N: int, nt: int, nk: int = 1) -> float:
    """Flops of one sox_sigma_gw call: per node and momentum the projections
    X^T G (n^2 N), (X^T G) X (N^2 n), X M (n N^2) and (X M) X^T (n^2 N)
    multiply-adds, 2 flops each (8 for complex); the mesh's momentum
    convolution as its direct n_k^2 N^2 complex multiply-adds per node."""
    macs = 2.0 * n * n * N + 2.0 * N * N * n
    if nk == 1:
        return 2.0 * nt * macs
    return 8.0 * nk * nt * macs + 8.0 * nk * nk * nt * N * N


def cpu_oracle_gw(wl: dict, poles):
    """Oracle sample of the THC-GW direct term: G(tau) synthesis and the
    THC chain for two tau nodes at full rank (the term is local in tau),
    timed and scaled to one call over every node; also the error reference
    of the GPU call at those nodes."""
    from oracle import sox_gw as ogw
    from oracle import sox_mol as om
    from oracle import sox_solid as osd
    nt = wl["n_tau"]
    nodes = [0, nt // 2]
    tn = wl["tau"][nodes]
    c0 = time.perf_counter()
    if poles is not None:
        G = osd.g_tau_k(wl["eps"], wl["Q"], wl["mu"], wl["beta"], tn)
        Wn = sum(a * pole[None, nodes, None, None] * S[:, None] for a, pole, S in poles)
        tb = (wl["kvecs"], wl["kdiff"], wl["ksum"], wl["kneg"])
        ref = ogw.sigma_gw_solid_thc(wl["X"], Wn, G, tb)
    else:
        G = om.g_tau(wl["eps"], wl["Q"], wl["mu"], wl["beta"], tn)
        ref = ogw.sigma_gw_thc(wl["X"], wl["W_tau"][nodes], G)
    sec = time.perf_counter() - c0
    rec = {"value": len(nodes) / nt / sec, "unit": "calls/s", "cores": blas_threads(),
           "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
           "kind": "oracle", "extrapolated": True,
           "sample": (f"numpy float64 oracle (THC chain, full rank) for {len(nodes)} of {nt} "
                      f"tau nodes ({sec:.2f} s, G(tau) and W_d(tau) at those nodes formed inside), "
                      "scaled to one call over every node")}
    return rec, ref, nodes


def cpu_oracle_solid(wl: dict, poles: list, tp: dict, cols) -> dict:
    """Oracle sample of the solid step SOX(V,V) + SOX(W_d,V).  At the full
    THC rank one oracle node and orbital v already take minutes on the host,
    so the sample is the same workload (mesh, n, tau grid, inputs) with the
    collocation matrix restricted to the `cols` support: the eq:GG chain for
    one orbital v (all nodes and momenta; the chain is a sum over v) and the
    static chain for one mirror pair of nodes (independent per node),
    scaled to one sweep of that reduced-rank problem."""
    from oracle import sox_solid as osd
    nt, n = wl["n_tau"], wl["n"]
    tb = (wl["kvecs"], wl["kdiff"], wl["ksum"], wl["kneg"])
    Xs = wl["X"][:, :, cols]
    Vs = wl["V"][:, cols][:, :, cols]
    Ws = sum(a * pole[None, :, None, None] * S[:, None][:, :, cols][:, :, :, cols]
             for a, pole, S in poles)
    c0 = time.perf_counter()
    G = osd.g_tau_k(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
    osd.sigma_solid_dynamic_thc(Xs, Ws, Vs, G, tp["T_fwd"], tp["T_bwd"], tb, v_subset=[0])
    t_dyn = time.perf_counter() - c0
    c1 = time.perf_counter()
    osd.sigma_solid_thc(Xs, Vs, Vs, G[:, [0, nt - 1]], tb)
    t_bare = time.perf_counter() - c1
    sweep = n * t_dyn + (nt / 2) * t_bare
    return {"value": 1.0 / sweep, "unit": "sweeps/s", "cores": blas_threads(),
            "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "kind": "oracle", "extrapolated": True,
            "sample": (f"numpy complex128 oracle on the same workload reduced to a "
                       f"{len(cols)}-of-{wl['N']}-column THC support (reduced rank: the full-rank "
                       f"oracle takes minutes per node and orbital): the eq:GG chain for 1 of {n} "
                       f"orbitals v ({t_dyn:.1f} s, all {nt} nodes and {wl['nk']} momenta, "
                       f"linear in v) and the static chain for 1 mirror pair of nodes "
                       f"({t_bare:.1f} s, linear in the nodes), scaled to one sweep of that "
                       f"reduced-rank problem")}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default by workload: 100, 100, 5, 3, 5)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default by workload: 10, 10, 1, 1, 1)")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16x3"],
                    help="default: bf16x3 for the solid, fp32 for the molecules")
    ap.add_argument("--workload", type=int, default=5, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-bf16x3-compare", action="store_true",
                    help="skip the split-precision run reported beside a float32 run")
    ap.add_argument("--no-vjp", action="store_true",
                    help="skip the adjoint (vector-Jacobian product) call timed after a "
                         "dynamic molecular run")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time of the oracle sample")
    ap.add_argument("--no-gw", action="store_true",
                    help="skip the THC-GW direct term (sox_sigma_gw) timed after a dynamic run")
    ap.add_argument("--no-ir", action="store_true",
                    help="skip the sweep on the library's IR grid after a dynamic run")
    ap.add_argument("--no-scf", action="store_true",
                    help="skip the self-consistent loop (sox_scf) on its own molecular system")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's own launch choices (no sox_autotune before the warmup)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of HIP graph replays")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in the design notes, not built)",
              file=sys.stderr)
        return 2
    desc, kind = WORKLOADS[args.workload]
    # defaults keep each timed region under a minute; the small workloads run
    # long enough for the clocks to settle and the launch ramp to amortise
    if args.steps is None:
        args.steps = {1: 100, 2: 100, 3: 5, 4: 3, 5: 5}[args.workload]
    if args.warmup is None:
        args.warmup = {1: 10, 2: 10}.get(args.workload, 1)
    if args.precision is None:
        args.precision = "bf16x3" if kind == "solid" else "fp32"
    import numpy as np
    import torch

    from paper_2412_18829_amd import binding as B
    from paper_2412_18829_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.workload(args.workload)
    n, N, nt = wl["n"], wl["N"], wl["n_tau"]
    solid = kind == "solid"
    nk = wl.get("nk", 1)
    cdt = torch.complex128 if solid else torch.float64
    t = lambda a, dt=cdt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    X, V, Q = t(wl["X"]), t(wl["V"]), t(wl["Q"])
    eps = t(wl["eps"], torch.float64)
    poles = None
    if solid:
        # W^q(tau_j) = sum_k a_k pole_k(tau_j) S_k^q, assembled on the device
        poles = synth.solid_screening_poles(wl)
        U1 = torch.zeros((nk, nt, N, N), dtype=cdt, device=dev)
        for a, pole, S_k in poles:
            U1 += t(a * pole)[None, :, None, None] * t(S_k)[:, None]
    else:
        U1 = t(wl["W0"]) if kind == "static" else (t(wl["W_tau"]) if kind == "dynamic" else V)
    tp = None
    if kind in ("dynamic", "solid"):
        tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=14.0, tol=1e-10)
    n_omega = len(tp["m"]) if tp is not None else 0
    gshape = (nk, nt, n, n) if solid else (nt, n, n)

    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib * 1048576
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def run(precision: str, steps: int, warmup: int, profile: bool, Xwarm=None,
            graph: bool = False, tune: bool = False):
        """warmup untimed steps, then `steps` timed ones.  Xwarm: the first
        warmup step runs on this collocation matrix instead (its Sigma is
        returned as Sigma_warm).  With profile, a later warmup step records
        every stage (the per-stage breakdown and the dominant kernel's launch
        times); with graphs, the last warmup step captures the sweep as a HIP
        graph and the timed steps replay it.  With tune, the plan's launch
        choices are first autotuned on the workload's own operands
        (sox_autotune, one call per candidate, before the warmup steps).
        None of this adds steps."""
        Xr = X
        use_graph = graph and warmup >= (3 if profile else 2)
        prof_step = warmup - 2 if use_graph else warmup - 1
        extra = {}
        if tp is not None:
            extra = dict(t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
        plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=precision,
                      kmesh=wl.get("mesh", (1, 1, 1)), **extra)
        G = torch.empty(gshape, dtype=cdt, device=dev)
        S = torch.empty_like(G)
        entry = "static" if kind == "static" else ("dynamic" if kind == "dynamic" else "bare")
        went = "vertex" if solid else entry
        vkind = "sosex_dyn" if solid else 0
        ws = plan.workspace(went, plan.autotune_workspace_size(went, vkind) if tune else None)
        if tune:
            B.sox_build_g_tau(plan, Q, eps, wl["mu"], G)
            u1, u2 = ((V, U1) if solid else (U1, V) if kind in ("static", "dynamic")
                      else (V, None))
            note(f"{precision}: autotuning the plan's launch choices")
            if use_graph:
                # candidates timed as graph replays, the mode the timed steps use
                B.sox_plan_set_graph(plan, True)
            B.sox_autotune(plan, went, X, u1, u2, G, S, kind=vkind, ws=ws)
            B.sox_plan_set_graph(plan, False)
            torch.cuda.synchronize()
            note(f"{precision}: autotuned {len(B.sox_plan_describe(plan)['autotune'])} candidates")
        # the energy of every step is queued into device memory (no host
        # synchronisation per step) and read after the timed region
        E = torch.zeros((warmup + steps + 3, 2), dtype=torch.float64, device=dev)
        cur = [0]

        def step():
            B.sox_build_g_tau(plan, Q, eps, wl["mu"], G)
            e = E[cur[0]]
            if kind == "static":
                B.sox_sigma_static(plan, Xr, U1, V, G, S, ws=ws)
            elif kind == "dynamic":
                B.sox_sigma_dynamic(plan, Xr, U1, V, G, S, ws=ws)
            elif solid:
                B.sox_sigma_vertex(plan, "sosex_dyn", Xr, V, U1, G, S, ws=ws)
            else:
                B.sox_sigma_bare(plan, Xr, V, G, S, ws=ws)
            B.sox_energy_gm_device(plan, S, G, e[0])
            cur[0] += 1

        sig_warm = None
        for w in range(warmup):
            note(f"{precision}: warmup step {w + 1} of {warmup}", every=20.0)
            if solid:
                torch.cuda.synchronize()
            if w == 0 and Xwarm is not None:
                Xr = Xwarm
                step()
                torch.cuda.synchronize()
                sig_warm = S.cpu().numpy()
                Xr = X
                continue
            if use_graph and w == warmup - 1:
                B.sox_plan_set_graph(plan, True)   # this step captures, later ones replay
            if profile and w == prof_step and warmup >= 2:
                B.sox_profile_select(plan, None)
                B.sox_profile_enable(plan, True)
                B.sox_profile_read(plan, reset=True)
                step()
                torch.cuda.synchronize()
                prof_warm = B.sox_profile_read(plan, reset=True)
                stages_warm = {k: round(v[0], 4) for k, v in prof_warm.items()
                               if k != "dropped" and v[1] > 0}
                B.sox_profile_enable(plan, False)
                continue
            step()
        torch.cuda.synchronize()
        if profile and not use_graph:
            # inside the timed region only the dominant stage is bracketed
            # with events (on the stream its kernels run on); graph replays
            # record none, so with graphs the profiled warmup step times it
            B.sox_profile_select(plan, [DOMINANT[kind][0]])
            B.sox_profile_enable(plan, True)
            B.sox_profile_read(plan, reset=True)
        # per-step device times from events on the stream the steps run on
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        note(f"{precision}: {steps} timed steps")
        for i in range(steps):
            evs[i][0].record()
            step()
            evs[i][1].record()
            if solid:
                # seconds per step: wait for each step (a few microseconds of
                # launch gap against seconds of work) to print progress now and then
                evs[i][1].synchronize()
                note(f"{precision}: timed step {i + 1} of {steps} done", every=30.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        note(f"{precision}: timed steps done")
        step_ms = sorted(a.elapsed_time(b) for a, b in evs)
        prof = stages = None
        prof_steps = steps
        if profile and use_graph:
            prof, prof_steps = prof_warm, 1
            stages = stages_warm
        elif profile:
            prof = B.sox_profile_read(plan, reset=True)
            if warmup >= 2:
                stages = stages_warm
            else:
                # the per-stage breakdown from a short untimed pass with every
                # stage recorded
                B.sox_profile_select(plan, None)
                kb = min(steps, 1 if solid else 3)
                for _ in range(kb):
                    step()
                torch.cuda.synchronize()
                stages = {k: round(v[0] / kb, 4) for k, v in
                          B.sox_profile_read(plan, reset=True).items()
                          if k != "dropped" and v[1] > 0}
            B.sox_profile_enable(plan, False)
        energies = E.cpu().numpy()[:cur[0]]
        res = dict(seconds=t1 - t0, Sigma=S.cpu().numpy(), prof=prof, stages=stages,
                   Sigma_warm=sig_warm, prof_steps=prof_steps, graph=use_graph,
                   median_step_ms=step_ms[len(step_ms) // 2] if len(step_ms) % 2
                   else 0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2]),
                   energy=float(energies[warmup + steps - 1, 0]),
                   # over the steps on the workload's own inputs (the first
                   # warmup step of the solid runs on the error input)
                   energy_spread=float(np.ptp(energies[1 if Xwarm is not None else 0:, 0])),
                   plan=B.sox_plan_describe(plan))
        # release this plan's workspace before the next leg builds its own
        del plan, ws, G, S, E
        torch.cuda.empty_cache()
        return res

    gold = Xc = None
    if solid and os.path.exists(GOLDEN_C5):
        # the error run: the first warmup step on a collocation matrix supported
        # on the stored oracle reference's columns (same launch configuration)
        gold = np.load(GOLDEN_C5)
        Xc = torch.zeros_like(X)
        Xc[:, :, gold["cols"]] = X[:, :, gold["cols"]]
        args.warmup = max(args.warmup, 1)
    with ws_budget(solid):
        main_run = run(args.precision, args.steps, args.warmup, profile=True, Xwarm=Xc,
                       graph=not args.no_graph, tune=not args.no_autotune)
    sec = main_run["seconds"]
    ms_per_step = 1e3 * sec / args.steps
    value = args.steps / sec

    fl = flops_per_sweep(n, N, nt, kind, n_omega, nk)
    sweep_flops = sum(v for k, v in fl.items() if k != "utensor")
    prof = main_run["prof"]
    stage, kname = DOMINANT[kind]
    if not solid:
        kname = FUSED_KERNEL.get(main_run["plan"]["fused_cfg"], kname)
    elif args.precision == "bf16x3":
        kname = "cgemm_panel_bf16x3_kernel"
    dom_ms, dom_launches = prof[stage]
    dom_avg_ms = dom_ms / max(dom_launches, 1)
    dom_flops_per_launch = fl[stage] * main_run["prof_steps"] / max(dom_launches, 1)
    mfma_tflops = dom_flops_per_launch / (dom_avg_ms * 1e-3) / 1e12
    peak_tflops = PEAK_TFLOPS[args.precision]
    if solid:
        # the B and C products write N x N outputs per K = n inputs: HBM-bound
        dom_bytes_per_launch = (solid_bc_bytes(n, N, nt, nk, main_run["plan"]["solid_dyn_tau_slab"])
                                * main_run["prof_steps"] / max(dom_launches, 1))
        roofline = {"kernel": kname, "bound": "hbm",
                    "achieved": dom_bytes_per_launch / (dom_avg_ms * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        roofline["frac"] = roofline["achieved"] / HBM_PEAK_GBS
        roofline["traffic"] = read_traffic(args.workload, args.precision, kind)
        roofline.update({"avg_launch_ms": dom_avg_ms, "bytes_per_launch": dom_bytes_per_launch,
                         "flops_per_launch": dom_flops_per_launch,
                         "mfma_tflops_fp32_equivalent": mfma_tflops,
                         "mfma_peak_tflops": peak_tflops})
    else:
        roofline = {"kernel": kname, "bound": "mfma", "achieved": mfma_tflops,
                    "peak": peak_tflops, "unit": "TFLOP/s", "frac": mfma_tflops / peak_tflops,
                    "traffic": read_traffic(args.workload, args.precision, kind),
                    "avg_launch_ms": dom_avg_ms, "flops_per_launch": dom_flops_per_launch}
    stage_ms = main_run["stages"]

    # every GPU run first (host-side numpy work between them would perturb
    # the launch timing), then the FP64 oracle on the host: the error
    # reference (bare molecules) and the CPU baseline
    out = {}
    r64 = rb = None
    if not args.no_fp64_compare and args.precision != "fp64":
        # the solid's float64 sweep takes tens of seconds: one sweep, no warmup
        k64 = 1 if solid else max(1, args.steps // 2)
        r64 = run("fp64", k64, 0 if solid else 1, profile=False)
    solid_err = None
    if gold is not None:
        got = main_run["Sigma_warm"][gold["k"]][:, gold["nodes"]]
        ref = gold["sigma"]
        solid_err = {"max_rel_err": float(np.abs(got - ref).max() / np.abs(ref).max()),
                     "against": ("FP64 oracle (tests/golden/c5_sosex_dyn_support8.npz) on the "
                                 f"workload with X restricted to {len(gold['cols'])} of {N} THC "
                                 f"columns, first warmup step; momenta "
                                 f"{[int(k) for k in gold['k']]}, nodes "
                                 f"{[int(j) for j in gold['nodes']]}")}
    if (args.precision == "fp32" and kind in ("bare", "static", "dynamic") and not solid
            and not args.no_bf16x3_compare):
        # the split-precision path on the same workload, same step
        rb = run("bf16x3", args.steps, args.warmup, profile=True, graph=not args.no_graph)

    vjp = None
    if kind == "dynamic" and not args.no_vjp and args.precision != "bf16x3":
        # one adjoint call of L = sum(Sigma * R) for a seeded R, on the same
        # inputs: dG, dX, dW(tau), dV (the forward chain is recomputed inside)
        plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision=args.precision,
                      t_fwd=tp["T_fwd"], t_bwd=tp["T_bwd"])
        G = torch.empty(gshape, dtype=cdt, device=dev)
        B.sox_build_g_tau(plan, Q, eps, wl["mu"], G)
        Rr = torch.as_tensor(np.random.default_rng(2024).standard_normal(gshape), device=dev)
        grads = [torch.zeros_like(a) for a in (G, X, U1, V)]
        torch.cuda.synchronize()
        B.sox_profile_enable(plan, True)
        B.sox_profile_read(plan, reset=True)
        t0 = time.perf_counter()
        B.sox_sigma_vjp(plan, "dynamic", X, U1, V, G, Rr, *grads)
        torch.cuda.synchronize()
        tv = time.perf_counter() - t0
        pv = B.sox_profile_read(plan, reset=True)
        vjp = {"entry": "sox_sigma_vjp (dynamic)", "seconds_per_call": tv,
               "forward_steps_equivalent": tv / (ms_per_step * 1e-3),
               "stage_ms": {k: round(v[0], 2) for k, v in pv.items()
                            if k != "dropped" and v[1] > 0},
               "note": "one call after the timed forward steps, no warmup"}
        del plan, G, Rr, grads

    gw = None
    if kind in ("dynamic", "solid") and not args.no_gw:
        # the THC-GW direct term on the same W_d(tau), G(tau) and X: one warm
        # call, then GW_CALLS timed calls (float64 whatever the precision)
        note("gw: THC-GW direct term")
        plan = B.Plan(n, N, wl["tau"], wl["weights"], wl["beta"], precision="fp64",
                      kmesh=wl.get("mesh", (1, 1, 1)))
        G = torch.empty(gshape, dtype=cdt, device=dev)
        Sg = torch.empty_like(G)
        B.sox_build_g_tau(plan, Q, eps, wl["mu"], G)
        wsg = plan.workspace("gw")
        B.sox_sigma_gw(plan, X, U1, G, Sg, ws=wsg)
        torch.cuda.synchronize()
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record()
        for _ in range(GW_CALLS):
            B.sox_sigma_gw(plan, X, U1, G, Sg, ws=wsg)
        ev[1].record()
        torch.cuda.synchronize()
        gms = ev[0].elapsed_time(ev[1]) / GW_CALLS
        gfl = gw_flops(n, N, nt, nk)
        gw = {"entry": "sox_sigma_gw", "ms_per_call": gms, "calls_timed": GW_CALLS,
              "dtype": "c128" if solid else "f64", "flops_per_call": gfl,
              "roofline": {"scope": "whole call (float64 MFMA products and, for the mesh, the "
                                    "momentum convolution)",
                           "bound": "mfma", "achieved": gfl / (gms * 1e-3) / 1e12,
                           "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                           "frac": gfl / (gms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"]},
              "workspace_bytes": plan.workspace_size("gw")}
        gw_sigma = Sg.cpu().numpy()
        del plan, G, Sg, wsg
        torch.cuda.empty_cache()

    irr = None
    if kind in ("dynamic", "solid") and not args.no_ir:
        # the same step on the library's IR grid (sox_ir_grid) for the
        # workload's beta and omega_max: one warmup and one timed sweep
        lam = wl["beta"] * IR_OMEGA_MAX
        note(f"ir: IR grid beta={wl['beta']:g} Lambda={lam:g} eps={IR_EPS:g}")
        ir_budget = ws_budget(solid).__enter__()
        c0 = time.perf_counter()
        g = B.sox_ir_grid(wl["beta"], lam, IR_EPS)
        build_s = time.perf_counter() - c0
        nti = len(g["tau"])
        wir = synth.workload(args.workload)      # same draws, sampled on the IR nodes
        wir["tau"] = g["tau"]
        if solid:
            Wir = torch.zeros((nk, nti, N, N), dtype=cdt, device=dev)
            for a, pole, S_k in synth.solid_screening_poles(wir):
                Wir += t(a * pole)[None, :, None, None] * t(S_k)[:, None]
        else:
            Wir = t(sum(a * synth.periodic_bosonic_pole(g["tau"], wl["beta"], w)[:, None, None] * S
                        for w, a, S in zip(wl["pole_w"], wl["pole_a"], wl["pole_S"])))
        plan = B.Plan(n, N, g["tau"], g["weights"], wl["beta"], precision=args.precision,
                      kmesh=wl.get("mesh", (1, 1, 1)), t_fwd=g["T_fwd"], t_bwd=g["T_bwd"])
        Gi = torch.empty((nk, nti, n, n) if solid else (nti, n, n), dtype=cdt, device=dev)
        Si = torch.empty_like(Gi)
        went = "vertex" if solid else "dynamic"
        wsi = plan.workspace(went)
        Ei = torch.zeros(2, dtype=torch.float64, device=dev)

        if not args.no_autotune:
            # the same launch-choice tuning as the main run, on this grid's operands
            B.sox_build_g_tau(plan, Q, eps, wl["mu"], Gi)
            wsi = plan.workspace(went, plan.autotune_workspace_size(went, "sosex_dyn" if solid
                                                                    else 0))
            u1, u2 = (V, Wir) if solid else (Wir, V)
            note("ir: autotuning the plan's launch choices")
            B.sox_autotune(plan, went, X, u1, u2, Gi, Si, kind="sosex_dyn" if solid else 0,
                           ws=wsi)
            torch.cuda.synchronize()

        def ir_step():
            B.sox_build_g_tau(plan, Q, eps, wl["mu"], Gi)
            if solid:
                B.sox_sigma_vertex(plan, "sosex_dyn", X, V, Wir, Gi, Si, ws=wsi)
            else:
                B.sox_sigma_dynamic(plan, X, Wir, V, Gi, Si, ws=wsi)
            B.sox_energy_gm_device(plan, Si, Gi, Ei[0])

        ir_step()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        ir_step()
        torch.cuda.synchronize()
        sweep_s = time.perf_counter() - c0
        # the per-stage breakdown from one more sweep with every stage recorded
        B.sox_profile_select(plan, None)
        B.sox_profile_enable(plan, True)
        B.sox_profile_read(plan, reset=True)
        ir_step()
        torch.cuda.synchronize()
        ir_stages = {k: round(v[0], 2) for k, v in B.sox_profile_read(plan, reset=True).items()
                     if k != "dropped" and v[1] > 0}
        B.sox_profile_enable(plan, False)
        irr = {"beta": wl["beta"], "lambda": lam, "eps": IR_EPS, "n_tau": nti,
               "n_omega": int(len(g["m"])), "build_s": build_s,
               "sweep_s": sweep_s, "sweeps_per_s": 1.0 / sweep_s,
               "vs_main_grid": {"n_tau": nt, "n_omega": n_omega, "sweep_s": sec / args.steps},
               "energy_gm": float(Ei[0].item()), "stage_ms": ir_stages,
               "note": ("the timed step of this workload (same inputs, precision and entry) on "
                        "the IR grid sox_ir_grid builds in host code for the workload's beta "
                        "and the transform pair's omega_max; plan tuned as the main run's, one "
                        "timed sweep")}
        del plan, Gi, Si, wsi, Wir
        torch.cuda.empty_cache()
        ir_budget.__exit__()

    scf = None
    if not args.no_scf:
        # the minimal self-consistent loop on its own system (every workload):
        # one spin channel, n = 64, N = 384, GW with a fixed 8-pole W_d, IR grid
        note("scf: self-consistent loop")
        fg = B.sox_ir_grid_fermion(SCF_BETA, SCF_LAMBDA, IR_EPS)
        bg = B.sox_ir_grid(SCF_BETA, SCF_LAMBDA, IR_EPS)
        swl = synth.small_molecule(SCF_N, SCF_NTHC, len(fg["tau"]), SCF_BETA, seed=SCF_SEED)
        swl["tau"] = fg["tau"]
        synth.add_dynamic_screening(swl)
        hs = swl["Q"] @ np.diag(swl["eps"]) @ swl["Q"].T
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        plan = B.Plan(SCF_N, SCF_NTHC, fg["tau"], bg["weights"], SCF_BETA, precision="fp64")
        Gs = torch.empty((len(fg["tau"]), SCF_N, SCF_N), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        so = B.sox_scf(plan, fg, f64(swl["X"]), f64(swl["V"]), f64(swl["W_tau"]), f64(hs),
                       SCF_N / 2, Gs, terms=("gw",), tol=SCF_TOL, max_iter=100)
        torch.cuda.synchronize()
        scf_s = time.perf_counter() - c0
        scf = {"entry": "sox_scf (terms: GW with a fixed W_d)", "n_orb": SCF_N, "n_thc": SCF_NTHC,
               "beta": SCF_BETA, "lambda": SCF_LAMBDA, "eps": IR_EPS, "n_tau": len(fg["tau"]),
               "n_nu": int(len(fg["n"])), "n_elec": SCF_N / 2, "tol": SCF_TOL,
               "seconds": scf_s, "iterations": so["iterations"],
               "ms_per_iteration": 1e3 * scf_s / max(so["iterations"], 1), "mu": so["mu"],
               "e_inf": so["e_inf"], "e_dyn": so["e_dyn"], "delta": so["delta"],
               "data": "synthetic one-spin-channel molecule, seed %d" % SCF_SEED}
        scf_G = Gs.cpu().numpy()
        del plan, Gs
        torch.cuda.empty_cache()

    # the oracle runs only in the CPU baseline leg; the last sweep it timed
    # (bare molecules) is also the FP64 reference of max_rel_err
    cpu = ref = None
    if not args.no_cpu_baseline:
        if solid:
            cpu = cpu_oracle_solid(wl, poles, tp, synth.column_support(N, 1, 502))
        else:
            cpu, ref = cpu_oracle_baseline(wl, kind, args.cpu_seconds)
    out["cpu_baseline"] = cpu
    if gw is not None and not args.no_cpu_baseline:
        gcpu, gref, gnodes = cpu_oracle_gw(wl, poles)
        gw["cpu_baseline"] = gcpu
        gw["max_rel_err"] = float(np.abs(gw_sigma[..., gnodes, :, :] - gref).max()
                                  / np.abs(gref).max())
        gw["max_rel_err_reference"] = (f"FP64 oracle (full rank, its own G(tau)) at tau "
                                       f"nodes {gnodes}")
    if gw is not None:
        out["gw"] = gw
    if scf is not None:
        if not args.no_cpu_baseline:
            from oracle import ir_grid as oir
            from oracle import scf as oscf
            c0 = time.perf_counter()
            ofg, obg = oir.ir_fermion(SCF_BETA, SCF_LAMBDA, IR_EPS), oir.ir_grid(SCF_BETA, SCF_LAMBDA, IR_EPS)
            sref = oscf.scf(swl["X"], swl["V"], swl["W_tau"], hs, SCF_N / 2, SCF_BETA, ofg,
                           obg["weights"], terms=("gw",), tol=SCF_TOL, max_iter=100)
            osec = time.perf_counter() - c0
            scf["cpu_baseline"] = {"value": 1.0 / osec, "unit": "loops/s", "cores": blas_threads(),
                                   "kind": "oracle",
                                   "sample": (f"the whole loop by the numpy oracle on its own IR "
                                              f"grid ({sref['iterations']} iterations, {osec:.1f} s)")}
            scf["max_abs_dG_vs_oracle"] = float(np.abs(scf_G - sref["G"]).max())
            scf["e_inf_rel_err"] = abs(scf["e_inf"] - sref["e_inf"]) / abs(sref["e_inf"])
            scf["e_dyn_rel_err"] = abs(scf["e_dyn"] - sref["e_dyn"]) / abs(sref["e_dyn"])
            scf["mu_abs_err"] = abs(scf["mu"] - sref["mu"])
        out["scf"] = scf
    if irr is not None:
        if not args.no_cpu_baseline:
            from oracle import ir_grid as oir
            c0 = time.perf_counter()
            og = oir.ir_grid(irr["beta"], irr["lambda"], irr["eps"])
            osec = time.perf_counter() - c0
            irr["cpu_baseline"] = {"value": 1.0 / osec, "unit": "grids/s", "cores": blas_threads(),
                                   "kind": "oracle",
                                   "sample": "one full IR grid construction by the numpy oracle "
                                             "(same beta, Lambda, eps)"}
            irr["grid_matches_oracle"] = bool(len(og["tau"]) == irr["n_tau"]
                                              and len(og["m"]) == irr["n_omega"])
        out["ir_grid"] = irr
    if cpu is None:
        out["cpu_baseline_note"] = ("not run: " + ("disabled by flag" if args.no_cpu_baseline else
                                    "no bounded oracle sample fits this workload on the host"))

    def err_of(S):
        if ref is None:
            return None
        return float(np.abs(S - ref).max() / np.abs(ref).max())

    main_err = err_of(main_run["Sigma"])
    if solid_err is not None:
        main_err = solid_err["max_rel_err"]
        out["max_rel_err_reference"] = solid_err["against"]
    if r64 is not None:
        s64 = r64["seconds"] / k64
        d = np.abs(main_run["Sigma"] - r64["Sigma"]).max() / np.abs(r64["Sigma"]).max()
        out["fp64_path"] = {"sweeps_per_s": 1.0 / s64, "ms_per_step": 1e3 * s64,
                            "max_rel_err": err_of(r64["Sigma"]),
                            "max_rel_diff_to_main": float(d)}
        tol = 1e-6 if args.precision == "fp32" else 1e-4
        acc = main_err if main_err is not None else float(d)
        out["mixed_beats_fp64"] = bool(value > 1.0 / s64 and acc <= tol)
    if rb is not None:
        sb = rb["seconds"] / args.steps
        fb_ms, fb_n = rb["prof"]["fused"]
        fb_ach = fl["fused"] * rb["prof_steps"] / max(fb_n, 1) / (fb_ms / max(fb_n, 1) * 1e-3) / 1e12
        d = np.abs(rb["Sigma"] - main_run["Sigma"]).max() / np.abs(main_run["Sigma"]).max()
        out["bf16x3_path"] = {
            "sweeps_per_s": 1.0 / sb, "ms_per_step": 1e3 * sb,
            "max_rel_err": err_of(rb["Sigma"]), "max_rel_diff_to_fp32": float(d),
            "fused_kernel": FUSED_KERNEL.get(rb["plan"]["fused_cfg"], "?"),
            "fused_avg_launch_ms": fb_ms / max(fb_n, 1),
            "fused_achieved_tflops_alg": fb_ach,
            "fused_frac_of_bf16_peak": fb_ach / PEAK_TFLOPS["bf16x3"],
            "fused_frac_of_bf16_peak_mfma_work": 3.0 * fb_ach / PEAK_TFLOPS["bf16x3"],
            "stage_ms_per_step": rb["stages"],
        }

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (DTYPE_NAME[args.precision] if not solid
                  else "c" + DTYPE_NAME[args.precision] if args.precision != "bf16x3"
                  else "c64-bf16x3"),
        "data": "synthetic",
        "config": {"workload": desc, "entry": ENTRY[kind], "n_orb": n, "n_thc": N, "n_tau": nt,
                   "beta": wl["beta"], "kmesh": list(wl.get("mesh", (1, 1, 1))),
                   "n_omega": n_omega, "precision": args.precision,
                   "step": ("G(tau) + Sigma(all tau" + (", all k; SOX(V,V) + SOX(W_d,V)" if solid
                                                          else "") + ") + E_GM")},
        "tflops_alg": sweep_flops / (ms_per_step * 1e-3) / 1e12,
        "median_step_ms": main_run["median_step_ms"],
        "timed_as": ("HIP graph replays of the whole sweep (captured in the last warmup step)"
                     if main_run["graph"] else "eager launches"),
        "energy_gm": main_run["energy"],
        "energy_gm_spread_over_steps": main_run["energy_spread"],
        "max_rel_err": main_err,
        "roofline": roofline,
        "stage_ms_per_step": stage_ms,
        "plan": main_run["plan"],
        "workspace_budget_mb": int(os.environ.get("SOX_WS_BUDGET_MB", 0)) or
                               (SOLID_WS_BUDGET_MB if solid else 65536),
        "peak_device_memory_gib": round(torch.cuda.max_memory_allocated() / 2 ** 30, 2),
    }
    if vjp is not None:
        out["vjp"] = vjp
    rec.update(out)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
