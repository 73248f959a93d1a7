"""Helpers shared by the GPU tests: device upload and the error metric.

The error metric of every parity check is max |GPU - oracle| / max |oracle|
over all tau (and k), the primary metric of the design notes.
"""
import numpy as np


def have_gpu() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref) -> float:
    got = np.asarray(got)
    ref = np.asarray(ref)
    s = np.abs(ref).max()
    return float(np.abs(got - ref).max() / s) if s > 0 else float(np.abs(got).max())


def log(msg: str) -> None:
    print(msg, flush=True)
