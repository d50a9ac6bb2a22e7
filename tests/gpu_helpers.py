"""Helpers shared by the GPU parity tests (moving arrays between NumPy and torch)."""
import numpy as np

TOL = {"c64": 2e-5, "c128": 1e-12}


def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    return _t


def to_dev(a: np.ndarray, dtype: str):
    t = torch()
    npdt = np.complex64 if dtype == "c64" else np.complex128
    return t.from_numpy(np.ascontiguousarray(a.astype(npdt))).cuda()


def to_np(x) -> np.ndarray:
    torch().cuda.synchronize()
    return x.cpu().numpy().astype(np.complex128) if x.is_complex() else x.cpu().numpy().astype(np.float64)


def rounded(a: np.ndarray, dtype: str) -> np.ndarray:
    """The oracle's view of a state stored in the kernel's precision."""
    return a.astype(np.complex64 if dtype == "c64" else np.complex128).astype(np.complex128)


def maxabs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
