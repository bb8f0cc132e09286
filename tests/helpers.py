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
    """Sub-pixel offsets of the GPU within 2 float ulps of the oracle's when both search the
    same calibrated frames (the same FP64 scores up to summation order, then one rounding);
    returns the number of frames that differ at all."""
    g = np.asarray(s_gpu, dtype=np.float32).astype(np.float64)
    o = np.asarray(s_orc, dtype=np.float32).astype(np.float64)
    assert g.shape == o.shape, (label, g.shape, o.shape)
    d = np.abs(g - o)
    assert np.all(d <= 2 * ulp32(o)), f"{label}: offsets beyond 2 ulp:\n{g}\n{o}"
    return int(np.any(d > 0, axis=-1).sum())


def offset_bound(cal_a, cal_b, ref_index, radius, offs_b, scores_b):
    """Largest change of each frame's parabola offset [N][2] (px) that the difference between
    two sets of calibrated frames can cause: the oracle searches cal_a from raw in FP64, the
    GPU searches its single-precision cal_b.  Each score S(d) = sum_T r'(x) f(x + d) then
    moves by at most b(d) = sum |r'||df| + sum |dr'||f| + sum |dr'||df| (+ the worst-case
    FP64 summation error of both sides), and the vertex delta = (S- - S+) / (2 (S- - 2 S0 + S+))
    by at most (b- + b+ + 2|delta| (b- + 2 b0 + b+)) / (2 |S- - 2 S0 + S+| - 2 (b- + 2 b0 + b+)),
    with the scores and offsets of either side (the bound is symmetric in the two)."""
    a = np.asarray(cal_a, np.float64)
    b = np.asarray(cal_b, np.float64)
    N, H, W = a.shape
    R = radius
    tw, th = W - 2 * R, H - 2 * R
    ra = a[ref_index, R:R + th, R:R + tw]
    rp = ra - ra.mean()
    dref = b[ref_index, R:R + th, R:R + tw] - ra
    drp = dref - dref.mean()
    eps_sum = 2.0 * tw * th * 2.0 ** -53
    side = 2 * R + 1
    out = np.zeros((N, 2))
    for k in range(N):
        dx, dy = int(offs_b["dx"][k]), int(offs_b["dy"][k])
        sc = np.asarray(scores_b[k]).reshape(side, side)

        def bnd(ex, ey):
            f = a[k, R + ey:R + ey + th, R + ex:R + ex + tw]
            df = b[k, R + ey:R + ey + th, R + ex:R + ex + tw] - f
            return (np.abs(rp * df).sum() + np.abs(drp * f).sum() + np.abs(drp * df).sum()
                    + eps_sum * np.abs(rp * f).sum())

        b0 = bnd(dx, dy)
        for ax, (ux, uy) in enumerate(((1, 0), (0, 1))):
            if not (-R < (dx if ax == 0 else dy) < R):
                continue  # on the window border: no vertex on this axis (exact integer on both sides)
            bm, bp = bnd(dx - ux, dy - uy), bnd(dx + ux, dy + uy)
            sm = sc[dy - uy + R, dx - ux + R]
            s0 = sc[dy + R, dx + R]
            sp = sc[dy + uy + R, dx + ux + R]
            den = 2.0 * (sm - 2.0 * s0 + sp)
            dd = 2.0 * (bm + 2.0 * b0 + bp)
            delta = (sm - sp) / den if den < 0 else 0.0
            out[k, ax] = (bm + bp + abs(delta) * dd) / (abs(den) - dd) if abs(den) > dd else np.inf
    return out


def assert_registration(orc, cal_orc, cal_gpu, offs_gpu, s_gpu, s_orc, radius, label, ref_index=0,
                        integer_mode=False):
    """Offsets of a chain from raw, checked in every case.  Stage-isolated: the oracle searches
    the GPU's own calibrated frames (promoted to FP64) and must find the same integer offsets,
    flags and, within 2 float ulps, sub-pixel offsets.  End to end: the oracle's search of its
    FP64 calibration must find the same integer offsets, and sub-pixel offsets within the
    bound that the single-precision calibration can move them (offset_bound) plus 2 ulps.
    Returns (frames whose offsets differ end to end, largest difference in px)."""
    cg = np.asarray(cal_gpu, np.float64)
    iso, scores = orc.register(cg[ref_index], cg, radius, want_scores=True)
    others = np.arange(len(cg)) != ref_index
    for key in ("dx", "dy"):
        assert np.array_equal(np.asarray(offs_gpu[key])[others], iso[key][others]), \
            f"{label}: stage-isolated integer offsets differ"
    assert np.array_equal(np.asarray(offs_gpu["flags"])[others] & 3, iso["flags"][others] & 3), \
        f"{label}: edge flags differ"
    s_iso = np.stack([iso["sx"], iso["sy"]], 1).astype(np.float32)
    if integer_mode:
        s_iso = np.stack([iso["dx"], iso["dy"]], 1).astype(np.float32)
    s_iso[ref_index] = 0.0
    assert_offsets_close(s_gpu, s_iso, label + " (stage-isolated)")
    g = np.asarray(s_gpu, np.float32).astype(np.float64)
    o = np.asarray(s_orc, np.float32).astype(np.float64)
    d = np.abs(g - o)
    if integer_mode:
        assert np.array_equal(g, o), f"{label}: integer offsets differ end to end"
    else:
        bound = offset_bound(cal_orc, cg, ref_index, radius, iso, scores)
        bound[ref_index] = 0.0
        tol = bound + 2 * ulp32(o)
        assert np.all(d <= tol), f"{label}: offsets beyond the calibration bound:\n{g}\n{o}\n{tol}"
    return int(np.any(d > 0, axis=-1).sum()), float(d.max())


def oracle_chain_at(orc, cal, s, rect, mask=None, missing=False, ksigma=3.0, max_iters=3):
    """The oracle's shift and clipped mean of its own calibrated frames cal [N][H][W] (FP64)
    at the given float32 offsets s [N][2] over rect: the end-to-end reference for a chain
    whose offsets are s.  Returns (out, near) with near [h][w] the pixels inside the
    threshold band of the clip (counted, not value-checked)."""
    al = orc.shift(cal, np.asarray(s, np.float32), rect, mask)
    out, _, _, near = orc.combine(al, ksigma, max_iters, missing=missing)
    return out, near.any(axis=0)


def assert_end_to_end(orc, cal, cal_gpu, offs_gpu, s_gpu, s_orc, rect, out_gpu, radius, label, ref_index=0,
                      integer_mode=False, mask=None, missing=False):
    """End-to-end value check from raw that runs in every case: the offsets as in
    assert_registration, then the GPU's combined image against the oracle's shift and clip
    of its own FP64 calibration at the GPU's offsets (the oracle's whole chain itself when
    the offsets agree bit for bit)."""
    n_diff, dmax = assert_registration(orc, cal, cal_gpu, offs_gpu, s_gpu, s_orc, radius, label, ref_index,
                                       integer_mode)
    ref, near = oracle_chain_at(orc, cal, s_gpu, rect, mask, missing)
    g = np.asarray(out_gpu, dtype=np.float64)
    assert g.shape == ref.shape, (label, g.shape, ref.shape)
    assert np.array_equal(np.isnan(g), np.isnan(ref)), f"{label}: missing pixels differ"
    ok = ~np.isnan(ref) & ~near
    e = rel_err(g[ok], ref[ok])
    print(f"{label}: {n_diff} of {len(s_gpu)} frames with offsets differing from the oracle's whole chain "
          f"(largest {dmax:.3g} px), {int(near.sum())} pixels in the clip's threshold band; {err_summary(e)}")
    assert e.size == 0 or e.max() <= TOL, f"{label}: {err_summary(e)}"
    return e
