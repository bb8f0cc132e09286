"""Bicubic-spline shift in FP64 -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The paper shifts frames by bicubic-spline interpolation and names the cost of its
tridiagonal systems, one per image row or column (Sec. 3.2.1).  Reading taken here: the
tensor-product natural cubic spline through the pixel values on the integer grid (zero
second derivative at both ends of every row and every column), evaluated at
(x + s_x, y + s_y) over the common overlap, like the bilinear shift.  Written from the
definition, along one line of values f[0..L-1]:

* second derivatives M solve  M[i-1] + 4 M[i] + M[i+1] = 6 (f[i+1] - 2 f[i] + f[i-1])
  for 0 < i < L-1, with M[0] = M[L-1] = 0 (forward elimination, back substitution);
* on [i, i+1], with t = x - i,
  S(x) = (1-t) f[i] + t f[i+1] + ((1-t)^3 - (1-t)) M[i] / 6 + (t^3 - t) M[i+1] / 6.

The 2-D interpolant is separable: the row splines are evaluated at the shifted x of every
output column for every row, then the column splines of that result at the shifted y.
"""
from __future__ import annotations

import numpy as np


def second_derivatives(f: np.ndarray) -> np.ndarray:
    """Natural-spline second derivatives along the last axis (FP64)."""
    f = np.asarray(f, dtype=np.float64)
    L = f.shape[-1]
    M = np.zeros_like(f)
    if L < 3:
        return M
    rhs = 6.0 * (f[..., 2:] - 2.0 * f[..., 1:-1] + f[..., :-2])  # equations i = 1 .. L-2
    n = L - 2
    c = np.empty(n)
    d = np.empty_like(rhs)
    c[0] = 1.0 / 4.0
    d[..., 0] = rhs[..., 0] / 4.0
    for i in range(1, n):
        den = 4.0 - c[i - 1]
        c[i] = 1.0 / den
        d[..., i] = (rhs[..., i] - d[..., i - 1]) / den
    x = np.empty_like(rhs)
    x[..., n - 1] = d[..., n - 1]
    for i in range(n - 2, -1, -1):
        x[..., i] = d[..., i] - c[i] * x[..., i + 1]
    M[..., 1:-1] = x
    return M


def evaluate(f: np.ndarray, M: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The splines of the lines of f (last axis) at positions x, clamped into [0, L-1]
    (positions inside the common overlap never need the clamp)."""
    f = np.asarray(f, dtype=np.float64)
    L = f.shape[-1]
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, L - 1.0)
    if L == 1:
        return np.broadcast_to(f[..., :1], f.shape[:-1] + x.shape).copy()
    i = np.clip(np.floor(x).astype(np.int64), 0, L - 2)
    t = x - i
    u = 1.0 - t
    return (u * f[..., i] + t * f[..., i + 1] + (u ** 3 - u) * M[..., i] / 6.0
            + (t ** 3 - t) * M[..., i + 1] / 6.0)


def shift_spline(frames: np.ndarray, offs: np.ndarray, rect) -> np.ndarray:
    """frames [N][H][W], offsets [N][2] (s_x, s_y; float32 values), rect (x0, y0, w, h)
    -> [N][h][w] FP64: out[k][v][u] = S_k(x0 + u + s_x, y0 + v + s_y)."""
    frames = np.asarray(frames, dtype=np.float64)
    if frames.ndim == 2:
        frames = frames[None]
    o = np.asarray(offs, dtype=np.float32).reshape(-1, 2)
    x0, y0, w, h = (int(v) for v in np.asarray(rect).reshape(4))
    N = frames.shape[0]
    out = np.empty((N, h, w))
    for k in range(N):
        xs = x0 + np.arange(w, dtype=np.float64) + float(o[k, 0])
        ys = y0 + np.arange(h, dtype=np.float64) + float(o[k, 1])
        rows = evaluate(frames[k], second_derivatives(frames[k]), xs)   # [H][w]
        cols = rows.T                                                    # [w][H]
        out[k] = evaluate(cols, second_derivatives(cols), ys).T
    return out
