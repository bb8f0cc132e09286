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


def assert_offsets_close(s_gpu, s_orc, label=""):
    """Sub-pixel offsets of the GPU within 2 float ulps of the oracle's (same FP64 scores up
    to summation order, then one rounding); returns the number of frames that differ at all."""
    g = np.asarray(s_gpu, dtype=np.float32).astype(np.float64)
    o = np.asarray(s_orc, dtype=np.float32).astype(np.float64)
    assert g.shape == o.shape, (label, g.shape, o.shape)
    d = np.abs(g - o)
    assert np.all(d <= 2 * ulp32(o)), f"{label}: offsets beyond 2 ulp:\n{g}\n{o}"
    return int(np.any(d > 0, axis=-1).sum())


def oracle_chain_at(orc, cal, s, rect, mask=None, missing=False, ksigma=3.0, max_iters=3):
    """The oracle's shift and clipped mean of its own calibrated frames cal [N][H][W] (FP64)
    at the given float32 offsets s [N][2] over rect: the end-to-end reference for a chain
    whose offsets are s.  Returns (out, near) with near [h][w] the pixels inside the
    threshold band of the clip (counted, not value-checked)."""
    al = orc.shift(cal, np.asarray(s, np.float32), rect, mask)
    out, _, _, near = orc.combine(al, ksigma, max_iters, missing=missing)
    return out, near.any(axis=0)


def assert_end_to_end(orc, cal, s_gpu, s_orc, rect, out_gpu, label, mask=None, missing=False):
    """End-to-end value check from raw that runs in every case: the GPU's combined image
    against the oracle's shift and clip at the GPU's own offsets (identical to the oracle's
    whole chain when the offsets agree bit for bit, which is counted and printed)."""
    n_diff = assert_offsets_close(s_gpu, s_orc, label)
    ref, near = oracle_chain_at(orc, cal, s_gpu, rect, mask, missing)
    g = np.asarray(out_gpu, dtype=np.float64)
    assert g.shape == ref.shape, (label, g.shape, ref.shape)
    assert np.array_equal(np.isnan(g), np.isnan(ref)), f"{label}: missing pixels differ"
    ok = ~np.isnan(ref) & ~near
    e = rel_err(g[ok], ref[ok])
    print(f"{label}: {n_diff} of {len(s_gpu)} frames with offsets differing from the oracle's "
          f"(within 2 ulp), {int(near.sum())} pixels in the clip's threshold band; {err_summary(e)}")
    assert e.size == 0 or e.max() <= TOL, f"{label}: {err_summary(e)}"
    return e
