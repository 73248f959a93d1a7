"""The C ABI library loads and exports every symbol include/sox.h declares;
argument checks that return before any device work is queued (no GPU needed).
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2412_18829_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sox.h")

pytestmark = pytest.mark.skipif(not os.path.exists(binding.LIB_PATH),
                                reason="libsox.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sox_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for required in ("sox_sigma_bare", "sox_sigma_static", "sox_sigma_dynamic", "sox_sigma_vjp",
                     "sox_plan_create", "sox_workspace_size", "sox_build_g_tau", "sox_energy_gm"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(binding.EXPORTED) == set(declared_functions())
    assert binding.sox_abi_version() == 2


def _problem(n=4, N=8, tau=None, beta=5.0, kmesh=(1, 1, 1)):
    if tau is None:
        tau, w = synth.chebyshev_tau_grid(6, beta)
    else:
        w = np.ones_like(tau)
    keep = [np.ascontiguousarray(tau, dtype=np.float64), np.ascontiguousarray(w, dtype=np.float64)]
    pr = binding.sox_problem()
    pr.n_orb, pr.n_thc, pr.n_tau = n, N, len(tau)
    pr.kmesh[:] = list(kmesh)
    pr.beta = beta
    pr.tau = keep[0].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pr.weights = keep[1].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pr.n_omega = 0
    return pr, keep


def _create(pr, precision=1):
    h = ctypes.c_void_p()
    st = binding.load().sox_plan_create(ctypes.byref(pr), precision, ctypes.byref(h))
    return st, h


def test_plan_create_rejects_bad_problems_before_device_work():
    lib = binding.load()
    pr, keep = _problem(n=0)
    assert _create(pr)[0] == 2                      # SHAPE
    pr, keep = _problem(beta=-1.0)
    assert _create(pr)[0] == 1                      # INVALID_ARG
    pr, keep = _problem(tau=np.array([0.5, 1.0, 4.0]), beta=5.0)
    assert _create(pr)[0] == 3                      # GRID: not mirror symmetric
    assert b"mirror" in lib.sox_last_error()
    pr, keep = _problem(tau=np.array([1.0, 0.5, 4.0, 4.5]), beta=5.5)
    assert _create(pr)[0] == 3                      # GRID: not ascending
    pr, keep = _problem(kmesh=(3, 0, 3))
    assert _create(pr)[0] == 2                      # SHAPE: mesh entry < 1
    pr, keep = _problem(kmesh=(17, 1, 1))
    assert _create(pr)[0] == 2                      # SHAPE: mesh beyond the supported range
    pr, keep = _problem()
    assert _create(pr, precision=9)[0] == 1         # unknown precision
    h = ctypes.c_void_p()
    assert lib.sox_plan_create(None, 1, ctypes.byref(h)) == 1
    assert lib.sox_plan_create(ctypes.byref(pr), 1, None) == 1


def test_entry_points_reject_null_plan():
    lib = binding.load()
    out = ctypes.c_size_t()
    assert lib.sox_workspace_size(None, 0, ctypes.byref(out)) == 1
    assert lib.sox_sigma_bare(None, None, None, None, None, None, 0, None) == 1
    assert lib.sox_sigma_static(None, None, None, None, None, None, None, 0, None) == 1
    assert lib.sox_sigma_dynamic(None, None, None, None, None, None, None, 0, None) == 1
    assert lib.sox_sigma_vjp(None, 0, *([None] * 9), None, 0, None) == 1
    e = ctypes.c_double()
    assert lib.sox_energy_gm(None, None, None, ctypes.byref(e), None) == 1
    assert lib.sox_energy_gm_device(None, None, None, None, None) == 1
    assert lib.sox_build_g_tau(None, None, None, 0.0, None, None) == 1
    assert lib.sox_profile_select(None, 1) == 1
    assert lib.sox_plan_destroy(None) == 0
