"""Shared test utilities: the paper's relative-difference metric and device transfers."""
import numpy as np

TOL = 2e-6  # pixel tolerance against the FP64 oracle


def rel_err(gpu, ref) -> np.ndarray:
    """Relative difference of Section 3.1 (equation for Delta I), with a 1 ADU floor."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ref, dtype=np.float64)
    return np.abs(g - o) / np.maximum(np.abs(o), 1.0)


def err_summary(e: np.ndarray) -> str:
    e = np.asarray(e).ravel()
    if e.size == 0:
        return "empty"
    return (f"max {e.max():.3g}  p99.9 {np.quantile(e, 0.999):.3g}  "
            f"90% {np.quantile(e, 0.90):.3g}  95% {np.quantile(e, 0.95):.3g}")


def to_dev(a, dev="cuda:0"):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(dev)


def ulp32(x) -> np.ndarray:
    x = np.abs(np.asarray(x, dtype=np.float32))
    return np.spacing(x).astype(np.float64)
