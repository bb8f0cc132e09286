"""FP64 CPU oracle of the reduction hot path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle.so`` (plain C, built from ``oracle.c`` by
``build()``).  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg import this package; the product library never does, and this package imports
nothing from the product.

Every function takes and returns numpy arrays (float64 unless stated) and follows the
plain definitions written out in ``oracle.c``:

* ``calibrate``: (raw - dark) / flat (dark subtraction and flat fielding, Sec. 2.1-2.2);
* ``register``: zero-mean-template cross-correlation, argmax, 3-point parabola;
* ``valid_rect`` / ``shift``: common overlap and bilinear resampling (Sec. 3.1.2, 3.2.1);
* ``combine``: iterative sigma-clipped mean (Sec. 2.1, 3.1.2);
* ``shift_spline``: natural bicubic-spline resampling (``spline.py``, NumPy);
* ``downsample4``: 4x4 block mean;
* ``cnn_*``: the offset-proposal network (see ``oracle_cnn.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["oracle.c", "oracle_cnn.c"]

EDGE_X, EDGE_Y, NEAR_TIE, CLIPPED = 1, 2, 4, 16


class OracleOffset(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int32), ("dy", ctypes.c_int32),
                ("sx", ctypes.c_float), ("sy", ctypes.c_float),
                ("peak", ctypes.c_double), ("second", ctypes.c_double),
                ("margin", ctypes.c_double), ("flags", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


OFFSET_DTYPE = np.dtype([("dx", "<i4"), ("dy", "<i4"), ("sx", "<f4"), ("sy", "<f4"),
                         ("peak", "<f8"), ("second", "<f8"), ("margin", "<f8"),
                         ("flags", "<i4"), ("pad", "<i4")])
assert OFFSET_DTYPE.itemsize == ctypes.sizeof(OracleOffset) == 48


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: -O2, OpenMP, no FP contraction, no fast-math."""
    srcs = [os.path.join(_HERE, s) for s in SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(LIB_PATH) and all(
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(s) for s in srcs):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L: ctypes.CDLL) -> None:
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.oracle_num_threads.restype = ctypes.c_int
    L.oracle_set_num_threads.argtypes = [ctypes.c_int]
    L.oracle_set_num_threads.restype = None
    L.oracle_calibrate.argtypes = [P, I64, I64, P, P, P, I64, P, I32, I32, I32]
    L.oracle_register.argtypes = [P, P, I32, I32, I32, I32, I32, P, P, P, P]
    L.oracle_valid_rect.argtypes = [P, I32, I32, I32, P]
    L.oracle_shift.argtypes = [P, P, I32, I32, I32, P, P, P]
    L.oracle_combine.argtypes = [P, I32, I32, I32, D, I32, P, P, P, P, D, I32]
    L.oracle_downsample4.argtypes = [P, I32, I32, P]
    L.oracle_cnn_input.argtypes = [P, I32, I32, P]
    for name in ("oracle_calibrate", "oracle_register", "oracle_valid_rect", "oracle_shift",
                 "oracle_combine", "oracle_downsample4", "oracle_cnn_input"):
        getattr(L, name).restype = ctypes.c_int
    if hasattr(L, "oracle_cnn_forward"):
        L.oracle_bf16_round.argtypes = [P, P, I64]
        L.oracle_conv3x3s2_forward.argtypes = [P, I32, I32, I32, I32, P, P, I32, I32, P]
        L.oracle_conv3x3s2_backward.argtypes = [P, I32, I32, I32, I32, P, I32, P, I32, P, P, P, P]
        L.oracle_cnn_forward.argtypes = [P, I32, I32, I32, P, I32, P, P]
        L.oracle_cnn_loss_backward.argtypes = [P, I32, I32, I32, P, I32, P, D, P, P]
        L.oracle_cnn_num_params.restype = ctypes.c_int64
        L.oracle_cnn_act_size.argtypes = [I32, I32, I32]
        L.oracle_cnn_act_size.restype = ctypes.c_int64
        L.oracle_adamw.argtypes = [P, P, P, P, I64, D, D, D, D, D, I32]
        for name in ("oracle_bf16_round", "oracle_conv3x3s2_forward", "oracle_conv3x3s2_backward",
                     "oracle_cnn_forward", "oracle_cnn_loss_backward", "oracle_adamw"):
            getattr(L, name).restype = ctypes.c_int


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def calibrate(raw: np.ndarray, dark: np.ndarray, flat: np.ndarray, bias: Optional[np.ndarray] = None) -> np.ndarray:
    """raw uint16 [N][H][W] (any row/frame pitch via a view), bias (or None)/dark/flat [H][W]."""
    raw = np.asarray(raw)
    if raw.ndim == 2:
        raw = raw[None]
    assert raw.dtype == np.uint16
    N, H, W = raw.shape
    if raw.strides[2] != 2 or raw.strides[1] < 0 or raw.strides[0] < raw.strides[1] * H:
        raw = np.ascontiguousarray(raw)  # the C side takes nested row and frame pitches
    dark = np.ascontiguousarray(dark, dtype=np.float64)
    flat = np.ascontiguousarray(flat, dtype=np.float64)
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    if b is not None:
        assert b.shape == dark.shape
    out = np.empty((N, H, W), dtype=np.float64)
    _check(lib().oracle_calibrate(_p(raw), raw.strides[1] // 2, raw.strides[0] // 2,
                                  None if b is None else _p(b), _p(dark), _p(flat), dark.strides[0] // 8,
                                  _p(out), W, H, N),
           "oracle_calibrate")
    return out


def register(ref: np.ndarray, frames: np.ndarray, radius: int, radius_max: Optional[int] = None,
             centers: Optional[np.ndarray] = None, tmpl=None, want_scores: bool = False):
    """Returns a structured array of OFFSET_DTYPE [N] (and the score cube if asked)."""
    ref = _f64(ref)
    frames = _f64(frames)
    if frames.ndim == 2:
        frames = frames[None]
    N, H, W = frames.shape
    assert ref.shape == (H, W)
    rmax = radius if radius_max is None else radius_max
    c = None if centers is None else np.ascontiguousarray(centers, dtype=np.int32).reshape(N, 2)
    t = None if tmpl is None else np.ascontiguousarray(tmpl, dtype=np.int32).reshape(4)
    out = np.zeros(N, dtype=OFFSET_DTYPE)
    side = 2 * radius + 1
    scores = np.empty((N, side, side), dtype=np.float64) if want_scores else None
    _check(lib().oracle_register(_p(ref), _p(frames), W, H, N, radius, rmax, _p(c), _p(t),
                                 _p(out), _p(scores)), "oracle_register")
    return (out, scores) if want_scores else out


def valid_rect(offs: np.ndarray, W: int, H: int) -> np.ndarray:
    o = np.ascontiguousarray(offs, dtype=np.float32).reshape(-1, 2)
    rect = np.zeros(4, dtype=np.int32)
    _check(lib().oracle_valid_rect(_p(o), o.shape[0], W, H, _p(rect)), "oracle_valid_rect")
    return rect


def shift(frames: np.ndarray, offs: np.ndarray, rect, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Bilinear shift; mask: bad-pixel map uint8 [H][W] (nonzero = bad) or None."""
    frames = _f64(frames)
    if frames.ndim == 2:
        frames = frames[None]
    N, H, W = frames.shape
    o = np.ascontiguousarray(offs, dtype=np.float32).reshape(N, 2)
    r = np.ascontiguousarray(rect, dtype=np.int32).reshape(4)
    out = np.empty((N, int(r[3]), int(r[2])), dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    if m is not None:
        assert m.shape == (H, W)
    _check(lib().oracle_shift(_p(frames), _p(out), W, H, N, _p(o), _p(r), None if m is None else _p(m)),
           "oracle_shift")
    return out


def combine(aligned: np.ndarray, ksigma: float = 3.0, max_iters: int = 3,
            rel_band: float = 1e-6, missing: bool = False):
    """Returns (out [h][w], keep uint8 [N][h][w], n_rejected, near uint8 [N][h][w]); with
    missing, NaN values are left out (never kept, not counted as rejected)."""
    a = _f64(aligned)
    if a.ndim == 1:
        a = a.reshape(-1, 1, 1)
    N, h, w = a.shape
    out = np.empty((h, w), dtype=np.float64)
    keep = np.empty((N, h, w), dtype=np.uint8)
    near = np.empty((N, h, w), dtype=np.uint8)
    nrej = np.zeros(1, dtype=np.int64)
    _check(lib().oracle_combine(_p(a), w, h, N, float(ksigma), int(max_iters), _p(out), _p(keep),
                                _p(nrej), _p(near), float(rel_band), 1 if missing else 0), "oracle_combine")
    return out, keep, int(nrej[0]), near


def downsample4(img: np.ndarray) -> np.ndarray:
    img = _f64(img)
    H, W = img.shape
    out = np.empty((H // 4, W // 4), dtype=np.float64)
    _check(lib().oracle_downsample4(_p(img), W, H, _p(out)), "oracle_downsample4")
    return out


def cnn_input(img: np.ndarray) -> np.ndarray:
    """Block mean, standardisation, asinh, bfloat16 rounding (float64 [H/4][W/4])."""
    img = _f64(img)
    H, W = img.shape
    out = np.empty((H // 4, W // 4), dtype=np.float64)
    _check(lib().oracle_cnn_input(_p(img), W, H, _p(out)), "oracle_cnn_input")
    return out


def bf16_round(x) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _check(lib().oracle_bf16_round(_p(x), _p(out), x.size), "oracle_bf16_round")
    return out


CNN_CH = 32
CNN_CIN = (2, 32, 32, 32)


def cnn_num_params() -> int:
    return int(lib().oracle_cnn_num_params())


def cnn_split(params: np.ndarray) -> dict:
    """Views of the flat parameter vector: w1..w4 [9][cin][32], b1..b4, wl [2][32], bl [2]."""
    out, o = {}, 0
    for i, cin in enumerate(CNN_CIN):
        n = 9 * cin * CNN_CH
        out[f"w{i + 1}"] = params[o:o + n].reshape(9, cin, CNN_CH)
        o += n
        out[f"b{i + 1}"] = params[o:o + CNN_CH]
        o += CNN_CH
    out["wl"] = params[o:o + 2 * CNN_CH].reshape(2, CNN_CH)
    o += 2 * CNN_CH
    out["bl"] = params[o:o + 2]
    return out


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray, relu: bool = True) -> np.ndarray:
    """x [B][H][W][Cin], w [9][Cin][Cout] -> [B][ceil(H/2)][ceil(W/2)][Cout]."""
    x, w, b = _f64(x), _f64(w), _f64(b)
    B, H, W, Cin = x.shape
    Cout = w.shape[2]
    y = np.empty((B, (H + 1) // 2, (W + 1) // 2, Cout))
    _check(lib().oracle_conv3x3s2_forward(_p(x), B, Cin, H, W, _p(w), _p(b), Cout, 1 if relu else 0, _p(y)),
           "oracle_conv3x3s2_forward")
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, dz: np.ndarray, want_dx: bool = True):
    """Returns (dx or None, dw [9][Cin][Cout], db [Cout]) for dz = dLoss/dZ."""
    x, w, dz = _f64(x), _f64(w), _f64(dz)
    B, H, W, Cin = x.shape
    Cout = w.shape[2]
    dx = np.empty_like(x) if want_dx else None
    dw = np.empty_like(w)
    db = np.empty(Cout)
    _check(lib().oracle_conv3x3s2_backward(_p(x), B, Cin, H, W, _p(w), Cout, None, 1, _p(dz), _p(dx), _p(dw),
                                           _p(db)), "oracle_conv3x3s2_backward")
    return dx, dw, db


def cnn_forward(x: np.ndarray, params: np.ndarray, bf16: bool = True, want_acts: bool = False):
    """x [B][H][W][2] -> pred [B][2] (and the stored activations X1..X4 + pool, flat)."""
    x, params = _f64(x), _f64(params)
    B, H, W, _ = x.shape
    pred = np.empty((B, 2))
    acts = np.empty(int(lib().oracle_cnn_act_size(B, H, W))) if want_acts else None
    _check(lib().oracle_cnn_forward(_p(x), B, H, W, _p(params), 1 if bf16 else 0, _p(pred), _p(acts)),
           "oracle_cnn_forward")
    return (pred, acts) if want_acts else pred


def cnn_loss_backward(x: np.ndarray, params: np.ndarray, target: np.ndarray, huber_delta: float = 1.0,
                      bf16: bool = True):
    """(loss, grad of the flat parameters)."""
    x, params, target = _f64(x), _f64(params), _f64(target)
    B, H, W, _ = x.shape
    loss = np.zeros(1)
    grad = np.empty_like(params)
    _check(lib().oracle_cnn_loss_backward(_p(x), B, H, W, _p(params), 1 if bf16 else 0, _p(target),
                                          float(huber_delta), _p(loss), _p(grad)), "oracle_cnn_loss_backward")
    return float(loss[0]), grad


def adamw(params, m, v, grad, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
          eps: float = 1e-8, weight_decay: float = 0.0):
    """One AdamW step (FP64); returns the new (params, m, v), the inputs untouched."""
    p2, m2, v2 = (np.array(a, dtype=np.float64, copy=True).ravel() for a in (params, m, v))
    g = _f64(grad).ravel()
    assert p2.shape == m2.shape == v2.shape == g.shape
    _check(lib().oracle_adamw(_p(p2), _p(m2), _p(v2), _p(g), p2.size, float(lr), float(beta1), float(beta2),
                              float(eps), float(weight_decay), int(step)), "oracle_adamw")
    return p2, m2, v2


def reduce_stack(raw: np.ndarray, dark: np.ndarray, flat: np.ndarray, radius: int,
                 ref_index: int = 0, ksigma: float = 3.0, max_iters: int = 3,
                 integer_mode: bool = False, bias: Optional[np.ndarray] = None,
                 mask: Optional[np.ndarray] = None):
    """End-to-end chain from raw: calibrate, register to frame ref_index, shift, combine
    (with a bad-pixel mask, the outputs that read a bad pixel are missing in combine)."""
    cal = calibrate(raw, dark, flat, bias)
    offs = register(cal[ref_index], cal, radius)
    s = np.stack([offs["sx"], offs["sy"]], axis=1).astype(np.float32)
    if integer_mode:
        s = np.stack([offs["dx"], offs["dy"]], axis=1).astype(np.float32)
    s[ref_index] = 0.0
    rect = valid_rect(s, raw.shape[2], raw.shape[1])
    al = shift(cal, s, rect, mask)
    out, keep, nrej, near = combine(al, ksigma, max_iters, missing=mask is not None)
    return dict(cal=cal, offsets=offs, s=s, rect=rect, aligned=al, out=out, keep=keep,
                n_rej=nrej, near=near)


from .spline import shift_spline  # noqa: E402  (NumPy part of the oracle)
