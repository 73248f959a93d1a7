"""Host bounds check of the GPU library (no GPU needed).

The library's own sources are compiled for the CPU under AddressSanitizer
with a small HIP shim (tests/cpu_emu): every kernel launch runs all blocks
and threads sequentially, caller buffers have their exact sizes and every
buffer carved from the workspace is followed by a poisoned guard gap.  Any
out-of-bounds read or write of any kernel aborts the case.  The shapes cover
ragged n and N, one tau node, multiple tau / v slabs and both fused tiles.

The cases run as concurrent processes (up to eight at once, one fixture per
module that starts every selected case), each test then checks its own
case's output: the cases are independent processes, and the suite's wall
time is that of the longest few instead of their sum.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "cpu_emu")
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ not available")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("emu") / "emu")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I", EMU, "-x", "c++", os.path.join(EMU, "driver.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _env(**extra):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    env.update({k: v for k, v in extra.items() if v is not None})
    return env


def _mol(c, env_extra=None):  # (n, N, nt, prec, entry, vjp, budget)
    n, N, nt, prec, entry, vjp, budget = c[:7]
    return ([str(n), str(N), str(nt), str(prec), str(entry), str(vjp)],
            _env(SOX_WS_BUDGET_MB=budget, **(env_extra or {})))


def _solid(c, env_extra=None):  # (n, N, nt, prec, entry, mesh[, budget])
    n, N, nt, prec, entry, mesh = c[:6]
    budget = c[6] if len(c) > 6 else None
    return ([str(n), str(N), str(nt), str(prec), str(entry), "0", *[str(m) for m in mesh]],
            _env(SOX_WS_BUDGET_MB=budget, **(env_extra or {})))


def _tune(c):
    kind, case = c
    if kind == "mol":
        args, env = _mol(case[:6] + (None,), {"EMU_AUTOTUNE": "1"})
        args[-1] = "0"
        return args, env
    return _solid(case[:6] + (None,), {"EMU_AUTOTUNE": "1"})


# test name -> (case -> (arguments, environment), time limit in seconds)
JOBS = {
    "test_entry_point_in_bounds": (lambda c: _mol(c), 600),
    "test_solid_entry_in_bounds": (lambda c: _solid(c), 600),
    "test_solid_wide_frequency_in_bounds": (lambda c: _solid(c, {"EMU_NW": "48"}), 900),
    "test_lds_fused_kernel_in_bounds": (lambda c: _mol(c, {"SOX_FUSED_CFG": str(c[7])}), 900),
    "test_dense_multi_tile_in_bounds": (lambda c: _mol(c, {"SOX_DENSE_WG": str(c[7])}), 900),
    "test_noalloc_entry_in_bounds": (lambda c: (["noalloc", str(c)], _env()), 600),
    "test_autotune_in_bounds": (_tune, 900),
    "test_scf_in_bounds": (lambda c: (["scf", *[str(x) for x in c]], _env()), 900),
}
WORKERS = max(1, min(8, os.cpu_count() or 1))


def _run(emu, args, env, limit):
    try:
        r = subprocess.run([emu, *args], capture_output=True, text=True, env=env, timeout=limit)
        return r.returncode, r.stdout + r.stderr
    except subprocess.TimeoutExpired as e:
        return -1, f"time limit of {limit} s: {e}"


class _Runs:
    """(return code, output) per test id: every selected case run up front in
    a pool of processes, or (under pytest-xdist, whose workers each collect
    every test but run only their share) each case when its test asks."""

    def __init__(self, emu, jobs, eager):
        self.emu, self.jobs, self.done = emu, jobs, {}
        if eager:
            with ThreadPoolExecutor(max_workers=WORKERS) as pool:
                fut = {k: pool.submit(_run, emu, *v) for k, v in jobs.items()}
                self.done = {k: f.result() for k, f in fut.items()}

    def __getitem__(self, key):
        if key not in self.done:
            self.done[key] = _run(self.emu, *self.jobs[key])
        return self.done[key]


@pytest.fixture(scope="module")
def runs(emu, request):
    jobs = {}
    for item in request.session.items:
        if item.module.__name__ != __name__ or item.originalname not in JOBS:
            continue
        params = item.callspec.params
        case = params["case"] if "case" in params else params["prec"]
        build, limit = JOBS[item.originalname]
        args, env = build(case)
        jobs[item.nodeid] = (args, env, limit)
    return _Runs(emu, jobs, eager="PYTEST_XDIST_WORKER" not in os.environ)


def _ok(runs, request, marker="status 0"):
    rc, out = runs[request.node.nodeid]
    assert rc == 0 and marker in out and "AddressSanitizer" not in out, out[-4000:]
    return out


CASES = [
    # n, N, n_tau, precision(0 fp64 / 1 fp32 / 2 bf16x3), entry(0 bare, 1 static, 2 dynamic,
    # 4 GW), vjp, env budget
    (6, 20, 8, 0, 0, 0, None),
    (13, 70, 5, 1, 1, 0, None),
    (3, 7, 1, 1, 1, 0, None),
    (16, 256, 2, 1, 0, 0, None),
    (10, 40, 6, 1, 0, 0, "1"),
    (5, 12, 6, 1, 2, 0, None),
    (13, 70, 5, 0, 2, 0, None),
    (21, 90, 6, 1, 2, 0, "3"),
    (6, 20, 8, 0, 0, 1, None),
    (6, 20, 8, 1, 1, 1, None),
    (13, 70, 5, 1, 1, 1, None),
    (3, 7, 1, 1, 1, 1, None),
    (16, 256, 2, 1, 1, 1, None),
    (10, 64, 7, 0, 0, 1, "2"),
    (5, 12, 6, 1, 2, 1, None),
    (5, 12, 6, 0, 2, 1, None),
    (13, 70, 5, 1, 2, 1, None),
    (16, 256, 3, 1, 2, 1, None),
    (21, 90, 6, 1, 2, 1, "4"),
    (330, 20, 2, 1, 1, 1, None),   # adjoint past 320 orbitals: two y chunks of the hc kernel
    (13, 70, 5, 2, 1, 0, None),
    (6, 20, 8, 2, 0, 0, None),
    (16, 256, 3, 2, 0, 0, None),
    (10, 40, 6, 2, 0, 0, "1"),
    # GW entry (4): one slab, and two tau slabs under a 1 MB budget
    (7, 23, 5, 1, 4, 0, None),
    (20, 150, 8, 2, 4, 0, "1"),
]


# k-point meshes: n, N, n_tau, precision, entry, mesh, env budget (the
# templated D step for 2x1x1, 1x3x1 (canonicalised), 2x2x2, 3x3x3; the any-mesh
# D step for 4x1x1; several v slabs under a small budget)
SOLID_CASES = [
    (5, 20, 3, 0, 0, (2, 1, 1), None),
    (7, 33, 2, 1, 1, (1, 3, 1), None),
    (6, 18, 2, 1, 0, (2, 2, 2), None),
    (3, 10, 2, 1, 0, (3, 3, 3), None),
    (5, 17, 2, 0, 1, (4, 1, 1), None),
    (9, 40, 2, 1, 1, (3, 1, 1), "1"),
    (5, 160, 1, 1, 0, (3, 1, 1), None),   # 80 x 80 B / C tiles (float32)
    (4, 80, 1, 0, 1, (2, 1, 1), None),    # 80 x 16 B / C tiles (float64)
    (3, 10, 4, 1, 2, (3, 1, 1), None),    # dynamic entry, templated D step
    (4, 17, 3, 0, 2, (4, 1, 1), None),    # dynamic entry, any-mesh D step
    (5, 80, 3, 1, 2, (2, 2, 1), "1"),     # dynamic entry, pair and tau slabs
    (5, 160, 1, 2, 0, (3, 1, 1), None),   # bf16 x 3 split B / C products
    (3, 10, 4, 2, 2, (3, 1, 1), None),    # bf16 x 3, dynamic entry
    (4, 20, 4, 1, 2, (3, 1, 1), None),    # dynamic, even n: W(Omega) GG(Omega) in real block form
    (6, 33, 3, 2, 2, (2, 2, 1), "1"),     # the same in bf16 x 3, pair and tau slabs
    (4, 17, 3, 1, 2, (1, 3, 1), "1"),     # ragged N, several slabs
    # vertex entry, kind = entry - 3: SOSEX_dyn (bare and dynamic terms in one
    # pass) with the real-form transforms, 2SOSEX_dyn, G3W2_stat
    (4, 20, 4, 1, 6, (3, 1, 1), None),
    (6, 33, 3, 2, 6, (2, 2, 1), "1"),
    (5, 17, 3, 1, 7, (1, 3, 1), None),
    (4, 20, 2, 2, 5, (2, 1, 1), None),
    # SOSEX_dyn with n = 20 and n = 54: the bare-term merge kernel's 8- and
    # 16-step K loops
    (20, 44, 2, 1, 6, (2, 1, 1), None),
    (54, 56, 2, 2, 6, (2, 1, 1), None),
    # GW entry (8): LDS element blocks of 64 (3 momenta), 32 (64 momenta) and
    # 16 (75 momenta), and tau slabs under a 1 MB budget
    (5, 20, 3, 1, 8, (3, 1, 1), None),
    (3, 9, 2, 0, 8, (4, 4, 4), None),
    (2, 5, 1, 1, 8, (5, 5, 3), None),
    (8, 60, 4, 1, 8, (3, 1, 1), "1"),
]


@pytest.mark.parametrize("case", SOLID_CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_solid_entry_in_bounds(runs, request, case):
    _ok(runs, request)


# more than 40 bosonic samples (IR grids): the inverse transform's 64-wide
# instantiation, in float32 and bf16 x 3, plain dynamic and SOSEX_dyn
WIDE_CASES = [(4, 20, 6, 1, 2, (2, 1, 1)), (4, 20, 5, 2, 6, (3, 1, 1))]


@pytest.mark.parametrize("case", WIDE_CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_solid_wide_frequency_in_bounds(runs, request, case):
    _ok(runs, request)


# the LDS-staged fused kernel, split precision (config 8) and float32
# (config 9): one, two and three k stages per v, padded tiles, several tau
# slabs, the dynamic entry's v slabs
LDS_CASES = [
    (13, 70, 5, 2, 1, 0, None, 8),
    (40, 130, 3, 2, 0, 0, None, 8),
    (70, 300, 2, 2, 1, 0, None, 8),
    (10, 40, 6, 2, 0, 0, "1", 8),
    (13, 70, 5, 1, 1, 0, None, 9),
    (40, 130, 3, 1, 0, 0, None, 9),
    (10, 40, 6, 1, 0, 0, "1", 9),
    (21, 90, 6, 1, 2, 0, "3", 9),
    (5, 12, 6, 2, 2, 0, None, 8),
    (21, 90, 6, 2, 2, 0, "3", 8),
]


@pytest.mark.parametrize("case", LDS_CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_lds_fused_kernel_in_bounds(runs, request, case):
    out = _ok(runs, request)
    assert f'"fused_cfg":{case[7]}' in out, out[-2000:]


# the LDS-staged GEMM with several output tiles per workgroup (A step and
# U-contraction): every tile in one workgroup, and three workgroups with a
# short last one
DENSE_WG_CASES = [
    (13, 70, 5, 1, 1, 0, None, 1),
    (13, 70, 5, 1, 1, 0, None, 3),
    (13, 70, 5, 2, 1, 0, None, 3),
    (16, 256, 3, 1, 0, 0, None, 5),
    (10, 40, 6, 1, 0, 0, "1", 2),
]


@pytest.mark.parametrize("case", DENSE_WG_CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_dense_multi_tile_in_bounds(runs, request, case):
    _ok(runs, request)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_entry_point_in_bounds(runs, request, case):
    _ok(runs, request)


def test_launchers_refuse_grids_past_32bit_work_items(emu):
    """A dispatch packet holds each grid extent in work-items as 32 bits: every
    tiled launcher must refuse an x extent of 2^32 work-items or more with
    hipErrorInvalidValue instead of launching (the shim aborts on any such
    launch, here and in every case above)."""
    r = subprocess.run([emu, "guards"], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "guards: 0 launched" in out, out[-4000:]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_entry_in_bounds(runs, request, prec):
    """sox_sigma_bare_noalloc on its static scratch array: an oversize plan is
    refused with SOX_ERR_WORKSPACE, two later calls (the second smaller)
    stay inside the array (AddressSanitizer guards the global)."""
    _ok(runs, request, "noalloc ok")


# the operand-based autotuner: every candidate's launch sequence on the
# caller's buffers, then the entry with the chosen settings (molecules:
# fused configs and v splits, float32 and bf16 x 3; k-point: tau and pair
# slabs of the dynamic chain, v slabs of the static one)
TUNE_CASES = [
    ("mol", (13, 70, 5, 2, 1, 0, None)),
    ("mol", (16, 256, 2, 1, 0, 0, None)),
    ("solid", (4, 20, 4, 1, 6, (3, 1, 1), None)),
    ("solid", (5, 17, 2, 0, 1, (4, 1, 1), None)),
]


@pytest.mark.parametrize("case", TUNE_CASES, ids=lambda c: c[0] + "-" + "-".join(str(x) for x in c[1]))
def test_autotune_in_bounds(runs, request, case):
    out = _ok(runs, request)
    assert '"autotune":[{' in out, out[-4000:]


# the self-consistent loop: HF only, GW (bit 0), GW + bare SOX (bits 0, 1),
# a ragged N over several tiles, 300 frequencies (one Dyson workgroup each)
# and n = 100 (the Dyson matrix past the LDS size, inverted in device memory)
SCF_CASES = [(5, 9, 4, 3, 0, 0), (6, 70, 6, 5, 1, 0), (7, 20, 4, 3, 3, 1), (4, 11, 2, 300, 1, 0),
             (100, 110, 2, 2, 1, 0)]


@pytest.mark.parametrize("case", SCF_CASES, ids=lambda c: "-".join(str(x) for x in c))
def test_scf_in_bounds(runs, request, case):
    _ok(runs, request)
