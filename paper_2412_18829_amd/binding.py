"""ctypes binding of libsox.so with the C ABI's names (include/sox.h).

Argument marshalling only: tensors are torch CUDA (HIP) tensors on the
current device, passed by data pointer with the current torch stream.  No
arithmetic of the method runs here.  If the library has not been built the
first call raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsox.so")

SOX_OK = 0
STATUS_NAMES = {
    0: "SOX_OK", 1: "SOX_ERR_INVALID_ARG", 2: "SOX_ERR_SHAPE", 3: "SOX_ERR_GRID",
    4: "SOX_ERR_WORKSPACE", 5: "SOX_ERR_OOM", 6: "SOX_ERR_HIP", 7: "SOX_ERR_UNSUPPORTED",
}
SOX_FP64, SOX_FP32, SOX_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": SOX_FP64, "fp32": SOX_FP32, "bf16x3": SOX_BF16X3}
SOX_ENTRY_BARE, SOX_ENTRY_STATIC, SOX_ENTRY_DYNAMIC, SOX_ENTRY_VERTEX, SOX_ENTRY_GW = 0, 1, 2, 3, 4
ENTRIES = {"bare": SOX_ENTRY_BARE, "static": SOX_ENTRY_STATIC, "dynamic": SOX_ENTRY_DYNAMIC,
           "vertex": SOX_ENTRY_VERTEX, "gw": SOX_ENTRY_GW}
VERTEX_KINDS = {"sosex_stat": 0, "2sosex_stat": 1, "g3w2_stat": 2, "sosex_dyn": 3, "2sosex_dyn": 4}

EXPORTED = (
    "sox_plan_create", "sox_plan_destroy", "sox_workspace_size", "sox_sigma_bare",
    "sox_sigma_static", "sox_sigma_dynamic", "sox_sigma_vjp", "sox_build_g_tau",
    "sox_energy_gm", "sox_energy_gm_device", "sox_sync", "sox_last_error", "sox_abi_version", "sox_profile_enable",
    "sox_profile_read", "sox_profile_select", "sox_plan_set_graph", "sox_plan_describe",
    "sox_sigma_bare_noalloc", "sox_sigma_vertex", "sox_autotune", "sox_autotune_workspace_size",
    "sox_sigma_gw", "sox_ir_grid", "sox_ir_grid_fermion", "sox_scf_workspace_size", "sox_scf",
)
STAGES = ("gbuild", "utensor", "project", "astep", "fused", "back", "energy", "gg_ft", "wgemm",
          "ift", "split", "vjp", "kbc", "kd", "gw")


class SoxError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


class sox_problem(ctypes.Structure):
    _fields_ = [
        ("n_orb", ctypes.c_int32), ("n_thc", ctypes.c_int32), ("n_tau", ctypes.c_int32),
        ("kmesh", ctypes.c_int32 * 3), ("beta", ctypes.c_double),
        ("tau", ctypes.POINTER(ctypes.c_double)), ("weights", ctypes.POINTER(ctypes.c_double)),
        ("n_omega", ctypes.c_int32),
        ("t_fwd", ctypes.POINTER(ctypes.c_double)), ("t_bwd", ctypes.POINTER(ctypes.c_double)),
    ]


class sox_scf_params(ctypes.Structure):
    _fields_ = [
        ("n_elec", ctypes.c_double), ("mix", ctypes.c_double), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("terms", ctypes.c_int32), ("n_nu", ctypes.c_int32),
        ("nu", ctypes.POINTER(ctypes.c_double)), ("t_fwd", ctypes.POINTER(ctypes.c_double)),
        ("t_bwd", ctypes.POINTER(ctypes.c_double)), ("t_beta", ctypes.POINTER(ctypes.c_double)),
    ]


class sox_scf_result(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("e_inf", ctypes.c_double), ("e_dyn", ctypes.c_double),
                ("delta", ctypes.c_double), ("iterations", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsox.so once and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2412_18829_amd.build_lib` (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, sz, i32, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    L.sox_plan_create.argtypes = [ctypes.POINTER(sox_problem), i32, ctypes.POINTER(vp)]
    L.sox_plan_destroy.argtypes = [vp]
    L.sox_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.sox_sigma_bare.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_sigma_static.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_sigma_bare_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    L.sox_sigma_vertex.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_autotune.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_autotune_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    L.sox_sigma_dynamic.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_sigma_gw.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_ir_grid.argtypes = [dp, dp, dp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp,
                              vp, vp, vp, vp]
    L.sox_ir_grid_fermion.argtypes = [dp, dp, dp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      vp, vp, vp, vp, vp]
    L.sox_scf_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    L.sox_scf.argtypes = [vp, ctypes.POINTER(sox_scf_params), vp, vp, vp, vp, vp, vp,
                          ctypes.POINTER(sox_scf_result), vp, sz, vp]
    L.sox_sigma_vjp.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sox_build_g_tau.argtypes = [vp, vp, vp, dp, vp, vp]
    L.sox_energy_gm.argtypes = [vp, vp, vp, ctypes.POINTER(dp), vp]
    L.sox_energy_gm_device.argtypes = [vp, vp, vp, vp, vp]
    L.sox_sync.argtypes = [vp]
    L.sox_last_error.argtypes = []
    L.sox_last_error.restype = ctypes.c_char_p
    L.sox_abi_version.argtypes = []
    L.sox_profile_enable.argtypes = [vp, i32]
    L.sox_profile_select.argtypes = [vp, ctypes.c_uint32]
    L.sox_plan_set_graph.argtypes = [vp, i32]
    L.sox_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.sox_profile_read.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64), i32]
    for name in EXPORTED:
        if name not in ("sox_last_error",):
            getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def _check(status: int, where: str) -> None:
    if status != SOX_OK:
        msg = load().sox_last_error().decode(errors="replace")
        raise SoxError(status, where, msg)


def _ptr(t) -> int | None:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr()


def _f64(t, shape, name):
    import torch
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _ptr(t)


def _c128(t, shape, name):
    import torch
    if t is None:
        return None
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128 (k-point plans)")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _ptr(t)


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
class Plan:
    """Owns a sox_plan* and host copies of the grid it was built from."""

    def __init__(self, n_orb: int, n_thc: int, tau, weights, beta: float,
                 precision: str | int = "fp32", kmesh=(1, 1, 1), t_fwd=None, t_bwd=None):
        self.n, self.N = int(n_orb), int(n_thc)
        self.tau = np.ascontiguousarray(tau, dtype=np.float64)
        self.weights = np.ascontiguousarray(weights, dtype=np.float64)
        self.n_tau = int(self.tau.shape[0])
        self.beta = float(beta)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.kmesh = tuple(int(m) for m in kmesh)
        self.nk = int(np.prod(self.kmesh))
        pr = sox_problem()
        pr.n_orb, pr.n_thc, pr.n_tau = self.n, self.N, self.n_tau
        pr.kmesh[:] = list(kmesh)
        pr.beta = self.beta
        pr.tau = self.tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        pr.weights = self.weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._keep = []
        if t_fwd is not None:
            tf = np.ascontiguousarray(t_fwd, dtype=np.complex128)
            tb = np.ascontiguousarray(t_bwd, dtype=np.complex128)
            self._keep += [tf, tb]
            pr.n_omega = int(tf.shape[0])
            pr.t_fwd = tf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            pr.t_bwd = tb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            pr.n_omega = 0
        self.n_omega = int(pr.n_omega)
        h = ctypes.c_void_p()
        _check(load().sox_plan_create(ctypes.byref(pr), self.precision, ctypes.byref(h)),
               "sox_plan_create")
        self.handle = h
        self._ws = {}

    @property
    def solid(self) -> bool:
        return self.nk > 1

    def _t(self, t, shape, name):
        """Marshal a tensor: float64 `shape` for molecules, complex128
        [n_k, *shape] for k-point plans."""
        if self.solid:
            return _c128(t, (self.nk, *shape), name)
        return _f64(t, shape, name)

    def workspace_size(self, entry: str | int) -> int:
        e = ENTRIES[entry] if isinstance(entry, str) else int(entry)
        out = ctypes.c_size_t()
        _check(load().sox_workspace_size(self.handle, e, ctypes.byref(out)), "sox_workspace_size")
        return int(out.value)

    def autotune_workspace_size(self, entry: str | int, kind=0) -> int:
        e = ENTRIES[entry] if isinstance(entry, str) else int(entry)
        k = VERTEX_KINDS[kind] if isinstance(kind, str) else int(kind)
        out = ctypes.c_size_t()
        _check(load().sox_autotune_workspace_size(self.handle, e, k, ctypes.byref(out)),
               "sox_autotune_workspace_size")
        return int(out.value)

    def workspace(self, entry: str | int, nbytes: int | None = None):
        """A cached device workspace (torch uint8 tensor) for `entry`, of at
        least nbytes (default: the entry's size for the plan's choices)."""
        import torch
        e = ENTRIES[entry] if isinstance(entry, str) else int(entry)
        if nbytes is None:
            nbytes = self.workspace_size(e)
        ws = self._ws.get(e)
        if ws is None or ws.numel() < nbytes + 256:
            self._ws.pop(e, None)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            self._ws[e] = ws
        return ws

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().sox_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ws_args(plan: Plan, entry, ws):
    if ws is None:
        ws = plan.workspace(entry)
    p = ws.data_ptr()
    aligned = (p + 255) & ~255
    return aligned, ws.numel() - (aligned - p)


# ---------------------------------------------------------------------------
# entry points, same names as the C ABI
def sox_sigma_bare(plan: Plan, X, V, G, Sigma, ws=None, stream=None):
    n, N, nt = plan.n, plan.N, plan.n_tau
    w, wb = _ws_args(plan, "bare", ws)
    t = plan._t
    _check(load().sox_sigma_bare(plan.handle, t(X, (n, N), "X"), t(V, (N, N), "V"),
                                 t(G, (nt, n, n), "G"), t(Sigma, (nt, n, n), "Sigma"),
                                 w, wb, _stream(stream)), "sox_sigma_bare")
    return Sigma


def sox_sigma_bare_noalloc(plan: Plan, X, V, G, Sigma, stream=None):
    """sox_sigma_bare on the library's static scratch array (no workspace)."""
    n, N, nt = plan.n, plan.N, plan.n_tau
    t = plan._t
    _check(load().sox_sigma_bare_noalloc(plan.handle, t(X, (n, N), "X"), t(V, (N, N), "V"),
                                         t(G, (nt, n, n), "G"), t(Sigma, (nt, n, n), "Sigma"),
                                         _stream(stream)), "sox_sigma_bare_noalloc")
    return Sigma


def sox_sigma_vertex(plan: Plan, kind, X, V, W, G, Sigma, ws=None, stream=None):
    """Composite vertex self-energy; kind is a name of VERTEX_KINDS or its value.
    W is W0 [N, N] for the *_stat kinds and W_d(tau) [n_tau, N, N] for *_dyn."""
    n, N, nt = plan.n, plan.N, plan.n_tau
    k = VERTEX_KINDS[kind] if isinstance(kind, str) else int(kind)
    w, wb = _ws_args(plan, "vertex", ws)
    t = plan._t
    wshape = (nt, N, N) if k in (3, 4) else (N, N)
    _check(load().sox_sigma_vertex(plan.handle, k, t(X, (n, N), "X"), t(V, (N, N), "V"),
                                   t(W, wshape, "W"), t(G, (nt, n, n), "G"),
                                   t(Sigma, (nt, n, n), "Sigma"), w, wb, _stream(stream)),
           "sox_sigma_vertex")
    return Sigma


def sox_sigma_gw(plan: Plan, X, W_tau, G, Sigma, ws=None, stream=None):
    """THC-GW direct term Sigma = -G W_d (float64 whatever the plan's precision)."""
    n, N, nt = plan.n, plan.N, plan.n_tau
    w, wb = _ws_args(plan, "gw", ws)
    t = plan._t
    _check(load().sox_sigma_gw(plan.handle, t(X, (n, N), "X"), t(W_tau, (nt, N, N), "W_tau"),
                               t(G, (nt, n, n), "G"), t(Sigma, (nt, n, n), "Sigma"), w, wb,
                               _stream(stream)), "sox_sigma_gw")
    return Sigma


def sox_ir_grid(beta: float, lam: float, eps: float, capacity: int = 512) -> dict:
    """The library's IR grid: tau nodes, weights, Matsubara indices m, the
    transform pair T_fwd [n_omega, n_tau], T_bwd [n_tau, n_omega] (complex)
    and the singular values s_l / s_0 (host arrays)."""
    nt, nw = ctypes.c_int32(), ctypes.c_int32()
    tau = np.zeros(capacity)
    w = np.zeros(capacity)
    m = np.zeros(capacity, dtype=np.int64)
    tf = np.zeros(2 * capacity * capacity)
    tb = np.zeros(2 * capacity * capacity)
    sv = np.zeros(capacity)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(load().sox_ir_grid(float(beta), float(lam), float(eps), int(capacity), ctypes.byref(nt),
                              ctypes.byref(nw), p(tau), p(w), p(m), p(tf), p(tb), p(sv)),
           "sox_ir_grid")
    L, n = nt.value, nw.value
    return dict(tau=tau[:L].copy(), weights=w[:L].copy(), m=m[:n].copy(),
                T_fwd=tf[:2 * n * L].view(np.complex128).reshape(n, L).copy(),
                T_bwd=tb[:2 * L * n].view(np.complex128).reshape(L, n).copy(), s=sv[:L].copy())


def sox_ir_grid_fermion(beta: float, lam: float, eps: float, capacity: int = 512) -> dict:
    """The fermionic pair on the library's IR grid: tau, n (nu_n = (2n+1) pi /
    beta), T_fwd [n_nu, n_tau], T_bwd [n_tau, n_nu], t_beta [n_tau]."""
    nt, nw = ctypes.c_int32(), ctypes.c_int32()
    tau = np.zeros(capacity)
    m = np.zeros(capacity, dtype=np.int64)
    tf = np.zeros(2 * capacity * capacity)
    tb = np.zeros(2 * capacity * capacity)
    tbeta = np.zeros(capacity)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(load().sox_ir_grid_fermion(float(beta), float(lam), float(eps), int(capacity),
                                      ctypes.byref(nt), ctypes.byref(nw), p(tau), p(m), p(tf), p(tb),
                                      p(tbeta)), "sox_ir_grid_fermion")
    L, n = nt.value, nw.value
    return dict(tau=tau[:L].copy(), n=m[:n].copy(),
                T_fwd=tf[:2 * n * L].view(np.complex128).reshape(n, L).copy(),
                T_bwd=tb[:2 * L * n].view(np.complex128).reshape(L, n).copy(),
                t_beta=tbeta[:L].copy())


SCF_TERMS = {"gw": 1, "sox": 2}


def sox_scf(plan: Plan, fgrid: dict, X, V, W_tau, h, n_elec: float, G, terms=("gw",),
            mix: float = 0.5, tol: float = 1e-8, max_iter: int = 100, h_start=None, stream=None):
    """The minimal self-consistent loop on `plan` (its tau grid must be
    fgrid's).  G [n_tau, n, n] receives the converged G(tau); returns mu,
    e_inf, e_dyn, delta and iterations."""
    import torch
    n, N, nt = plan.n, plan.N, plan.n_tau
    bits = sum(SCF_TERMS[t] for t in terms)
    nu = np.ascontiguousarray((2 * fgrid["n"] + 1) * np.pi / plan.beta, dtype=np.float64)
    tf = np.ascontiguousarray(fgrid["T_fwd"], dtype=np.complex128)
    tb = np.ascontiguousarray(fgrid["T_bwd"], dtype=np.complex128)
    tbeta = np.ascontiguousarray(fgrid["t_beta"], dtype=np.float64)
    dptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    prm = sox_scf_params(float(n_elec), float(mix), float(tol), int(max_iter), int(bits),
                         int(len(nu)), dptr(nu), dptr(tf), dptr(tb), dptr(tbeta))
    nbytes = ctypes.c_size_t()
    _check(load().sox_scf_workspace_size(plan.handle, len(nu), bits, ctypes.byref(nbytes)),
           "sox_scf_workspace_size")
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) & ~255
    res = sox_scf_result()
    _check(load().sox_scf(plan.handle, ctypes.byref(prm), _f64(X, (n, N), "X"),
                          _f64(V, (N, N), "V"),
                          _f64(W_tau, (nt, N, N), "W_tau") if W_tau is not None else None,
                          _f64(h, (n, n), "h"),
                          _f64(h_start, (n, n), "h_start") if h_start is not None else None,
                          _f64(G, (nt, n, n), "G"), ctypes.byref(res), wp,
                          ws.numel() - (wp - ws.data_ptr()), _stream(stream)), "sox_scf")
    return dict(mu=res.mu, e_inf=res.e_inf, e_dyn=res.e_dyn, delta=res.delta,
                iterations=res.iterations)


def sox_autotune(plan: Plan, entry, X, U1, U2, G, Sigma, kind=0, ws=None, stream=None):
    """Time the plan's launch-choice candidates on these operands (one call of
    `entry` each) and keep the fastest.  U1, U2 as the entry takes them: bare
    V, None; static W0, V; dynamic W_tau, V; vertex V, W (kind as for
    sox_sigma_vertex).  Sigma receives the last candidate's result.  The
    default workspace is sized for every candidate."""
    n, N, nt = plan.n, plan.N, plan.n_tau
    e = ENTRIES[entry] if isinstance(entry, str) else int(entry)
    k = VERTEX_KINDS[kind] if isinstance(kind, str) else int(kind)
    if ws is None:
        ws = plan.workspace(e, plan.autotune_workspace_size(e, k))
    w, wb = _ws_args(plan, e, ws)
    t = plan._t
    s1 = (nt, N, N) if e == SOX_ENTRY_DYNAMIC else (N, N)
    s2 = (nt, N, N) if (e == SOX_ENTRY_VERTEX and k in (3, 4)) else (N, N)
    _check(load().sox_autotune(plan.handle, e, k, t(X, (n, N), "X"), t(U1, s1, "U1"),
                               t(U2, s2, "U2") if U2 is not None else None,
                               t(G, (nt, n, n), "G"), t(Sigma, (nt, n, n), "Sigma"), w, wb,
                               _stream(stream)), "sox_autotune")
    return Sigma


def sox_sigma_static(plan: Plan, X, W0, V, G, Sigma, ws=None, stream=None):
    n, N, nt = plan.n, plan.N, plan.n_tau
    w, wb = _ws_args(plan, "static", ws)
    t = plan._t
    _check(load().sox_sigma_static(plan.handle, t(X, (n, N), "X"), t(W0, (N, N), "W0"),
                                   t(V, (N, N), "V"), t(G, (nt, n, n), "G"),
                                   t(Sigma, (nt, n, n), "Sigma"), w, wb, _stream(stream)),
           "sox_sigma_static")
    return Sigma


def sox_sigma_dynamic(plan: Plan, X, W_tau, V, G, Sigma, ws=None, stream=None):
    n, N, nt = plan.n, plan.N, plan.n_tau
    w, wb = _ws_args(plan, "dynamic", ws)
    t = plan._t
    _check(load().sox_sigma_dynamic(plan.handle, t(X, (n, N), "X"),
                                    t(W_tau, (nt, N, N), "W_tau"), t(V, (N, N), "V"),
                                    t(G, (nt, n, n), "G"), t(Sigma, (nt, n, n), "Sigma"),
                                    w, wb, _stream(stream)), "sox_sigma_dynamic")
    return Sigma


def sox_sigma_vjp(plan: Plan, entry, X, U1, U2, G, R, dG=None, dX=None, dU1=None, dU2=None,
                  ws=None, stream=None):
    n, N, nt = plan.n, plan.N, plan.n_tau
    e = ENTRIES[entry] if isinstance(entry, str) else int(entry)
    u1_shape = (nt, N, N) if e == SOX_ENTRY_DYNAMIC else (N, N)
    w, wb = _ws_args(plan, e, ws)
    _check(load().sox_sigma_vjp(
        plan.handle, e, _f64(X, (n, N), "X"), _f64(U1, u1_shape, "U1"),
        _f64(U2, (N, N), "U2") if U2 is not None else None, _f64(G, (nt, n, n), "G"),
        _f64(R, (nt, n, n), "R"), _f64(dG, (nt, n, n), "dG"), _f64(dX, (n, N), "dX"),
        _f64(dU1, u1_shape, "dU1"), _f64(dU2, (N, N), "dU2"), w, wb, _stream(stream)),
        "sox_sigma_vjp")


def sox_build_g_tau(plan: Plan, Q, eps, mu: float, G, stream=None):
    n, nt = plan.n, plan.n_tau
    if plan.solid:
        q, e = _c128(Q, (plan.nk, n, n), "Q"), _f64(eps, (plan.nk, n), "eps")
    else:
        q, e = _f64(Q, (n, n), "Q"), _f64(eps, (n,), "eps")
    _check(load().sox_build_g_tau(plan.handle, q, e, float(mu), plan._t(G, (nt, n, n), "G"),
                                  _stream(stream)), "sox_build_g_tau")
    return G


def sox_energy_gm(plan: Plan, Sigma, G, stream=None) -> float:
    n, nt = plan.n, plan.n_tau
    e = ctypes.c_double()
    _check(load().sox_energy_gm(plan.handle, plan._t(Sigma, (nt, n, n), "Sigma"),
                                plan._t(G, (nt, n, n), "G"), ctypes.byref(e), _stream(stream)),
           "sox_energy_gm")
    return float(e.value)


def sox_energy_gm_device(plan: Plan, Sigma, G, E, stream=None):
    """Queue the energy into E (a one-element float64 device tensor, e.g. a
    row of a preallocated buffer) without synchronising."""
    import torch
    if E.dtype != torch.float64 or E.numel() != 1:
        raise ValueError("E must be a one-element float64 tensor")
    n, nt = plan.n, plan.n_tau
    _check(load().sox_energy_gm_device(plan.handle, plan._t(Sigma, (nt, n, n), "Sigma"),
                                       plan._t(G, (nt, n, n), "G"), _ptr(E), _stream(stream)),
           "sox_energy_gm_device")
    return E


def sox_sync(stream=None):
    _check(load().sox_sync(_stream(stream)), "sox_sync")


def sox_abi_version() -> int:
    return int(load().sox_abi_version())


def sox_profile_enable(plan: Plan, on: bool = True):
    _check(load().sox_profile_enable(plan.handle, 1 if on else 0), "sox_profile_enable")


def sox_profile_select(plan: Plan, stages=None):
    """Record only `stages` (names from STAGES; None: all) while profiling."""
    mask = 0xFFFFFFFF if stages is None else sum(1 << STAGES.index(s) for s in stages)
    _check(load().sox_profile_select(plan.handle, ctypes.c_uint32(mask)), "sox_profile_select")


def sox_profile_read(plan: Plan, reset: bool = True) -> dict:
    """{stage: (milliseconds, launches)} summed since the last reset, plus 'dropped'."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    dropped = ctypes.c_int64()
    _check(load().sox_profile_read(plan.handle, ms, cnt, ctypes.byref(dropped), 1 if reset else 0),
           "sox_profile_read")
    out = {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}
    out["dropped"] = int(dropped.value)
    return out


def sox_plan_set_graph(plan: Plan, enable: bool = True):
    _check(load().sox_plan_set_graph(plan.handle, 1 if enable else 0), "sox_plan_set_graph")


def sox_plan_describe(plan: Plan) -> dict:
    import json
    buf = ctypes.create_string_buffer(16384)
    _check(load().sox_plan_describe(plan.handle, buf, len(buf)), "sox_plan_describe")
    return json.loads(buf.value.decode())
