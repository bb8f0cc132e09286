"""CCD frame reduction on MI355X: Python binding of libreduce (see include/reduce.h).

Argument marshalling only: every function passes device pointers of caller-owned
torch tensors and the current HIP stream to the C ABI.  All arithmetic runs in the
library's HIP kernels; there is no CPU fallback, and importing the binding fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreduce.so")

OK, ERR_NULL, ERR_SHAPE, ERR_RANGE, ERR_WORKSPACE, ERR_HIP, ERR_UNSUPPORTED = range(7)
EDGE_X, EDGE_Y, NEAR_TIE, FALLBACK, CLIPPED = 1, 2, 4, 8, 16

# reduce_offset_t
OFFSET_DTYPE = np.dtype([("dx", "<i4"), ("dy", "<i4"), ("sx", "<f4"), ("sy", "<f4"),
                         ("peak", "<f8"), ("second", "<f8"), ("margin", "<f8"),
                         ("flags", "<i4"), ("pad", "<i4")])
OFFSET_BYTES = 48


class ReduceError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"libreduce status {status}: {detail}")
        self.status = status


_lib: Optional[ctypes.CDLL] = None


def build(verbose: bool = False) -> str:
    from . import builder
    return builder.build(verbose=verbose)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2008_11486_amd.build()")
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    P, I32, I64, F, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                             ctypes.c_double, ctypes.c_size_t)
    L.reduce_status_str.restype = ctypes.c_char_p
    L.reduce_status_str.argtypes = [ctypes.c_int]
    L.reduce_last_error.restype = ctypes.c_char_p
    L.reduce_version.restype = ctypes.c_int
    L.reduce_calibrate.argtypes = [P, I64, I64, P, P, P, I64, P, I32, I32, I32, P]
    L.reduce_register_ws.argtypes = [I32, I32, I32, I32, I32]
    L.reduce_register_ws.restype = SZ
    L.reduce_register.argtypes = [P, P, I32, I32, I32, I32, I32, P, P, P, P, P, SZ, P]
    L.reduce_register_fft_ws.argtypes = [I32, I32, I32, I32]
    L.reduce_register_fft_ws.restype = SZ
    L.reduce_register_fft.argtypes = [P, P, I32, I32, I32, I32, P, P, P, P, SZ, P]
    L.reduce_register_fft.restype = ctypes.c_int
    L.reduce_tune_search.argtypes = [P, P, I32, I32, I32, I32, P, P, SZ, I32, P, P, P, P]
    L.reduce_tune_search.restype = ctypes.c_int
    L.reduce_register_static.argtypes = [P, P, I32, I32, I32, I32, I32, P, P, P, P, P]
    L.reduce_register_static.restype = ctypes.c_int
    L.reduce_register_static_max.restype = SZ
    L.reduce_valid_rect.argtypes = [P, I32, I32, I32, P]
    L.reduce_shift.argtypes = [P, P, I32, I32, I32, P, P, I32, P]
    L.reduce_shift_spline_ws.argtypes = [I32, I32, I32]
    L.reduce_shift_spline_ws.restype = SZ
    L.reduce_shift_spline.argtypes = [P, P, I32, I32, I32, P, P, P, SZ, P]
    L.reduce_shift_spline.restype = ctypes.c_int
    L.reduce_combine.argtypes = [P, I32, I32, I32, F, I32, P, P, P, I32, P]
    L.reduce_mask_shifted.argtypes = [P, P, I32, I32, I32, P, P, I32, P]
    L.reduce_register_plan.argtypes = [I32, I32, I32, I32, I32, P]
    L.reduce_register_plan.restype = ctypes.c_int
    L.reduce_tune_register.argtypes = [P, P, I32, I32, I32, I32, I32, P, P, SZ, I32, P, P]
    L.reduce_tune_register_ws.argtypes = [I32, I32, I32, I32, I32]
    L.reduce_tune_register_ws.restype = SZ
    L.reduce_tune_combine.argtypes = [P, I32, I32, I32, F, I32, P, I32, P, P]
    L.reduce_tune_save.argtypes = [ctypes.c_char_p]
    L.reduce_tune_load.argtypes = [ctypes.c_char_p]
    for n in ("reduce_tune_register", "reduce_tune_combine", "reduce_tune_save", "reduce_tune_load",
              "reduce_tune_clear"):
        getattr(L, n).restype = ctypes.c_int
    L.reduce_stack_batch_ws.argtypes = [P, I32]
    L.reduce_stack_batch_ws.restype = SZ
    L.reduce_stack_batch.argtypes = [P, I32, P, SZ, P]
    L.reduce_stack_batch.restype = ctypes.c_int
    L.reduce_cnn_input_ws.argtypes = [I32, I32, I32]
    L.reduce_cnn_input_ws.restype = SZ
    L.reduce_cnn_input.argtypes = [P, I32, I32, I32, P, P, SZ, P]
    L.reduce_cnn_num_params.restype = I64
    L.reduce_cnn_ws.argtypes = [I32, I32, I32]
    L.reduce_cnn_ws.restype = SZ
    L.reduce_cnn_ws_offsets.argtypes = [I32, I32, I32, P]
    L.reduce_cnn_forward.argtypes = [P, I64, P, I32, I32, I32, P, P, P, SZ, P]
    L.reduce_cnn_backward.argtypes = [P, I64, P, I32, I32, I32, P, P, P, F, P, P, P, SZ, P]
    L.reduce_cnn_adamw.argtypes = [P, P, P, P, I64, F, F, F, F, F, I32, P]
    L.reduce_cnn_centres.argtypes = [P, I32, F, I32, P, P]
    L.reduce_recentre.argtypes = [P, I32, I32, P, P]
    L.reduce_render_frames.argtypes = [P, I32, P, I32, I32, I32, F, F, F, I32, ctypes.c_uint64, P, P]
    L.reduce_propose_ws.argtypes = [I32, I32, I32, I32, I32]
    L.reduce_propose_ws.restype = SZ
    L.reduce_propose.argtypes = [P, P, I32, I32, I32, P, I32, I32, F, I32, P, P, P, P, SZ, P]
    L.reduce_propose.restype = ctypes.c_int
    for n in ("reduce_cnn_input", "reduce_cnn_ws_offsets", "reduce_cnn_forward", "reduce_cnn_backward",
              "reduce_cnn_adamw", "reduce_cnn_centres", "reduce_render_frames", "reduce_recentre"):
        getattr(L, n).restype = ctypes.c_int
    L.reduce_prof_enable.argtypes = [ctypes.c_int]
    L.reduce_prof_query.argtypes = [ctypes.c_char_p, P, P]
    for n in ("reduce_calibrate", "reduce_register", "reduce_valid_rect", "reduce_shift", "reduce_combine",
              "reduce_mask_shifted", "reduce_prof_enable", "reduce_prof_query"):
        getattr(L, n).restype = ctypes.c_int
    for n, args in _EXTRA_DECLS.items():
        if hasattr(L, n):
            fn = getattr(L, n)
            fn.argtypes, fn.restype = args


_EXTRA_DECLS: dict = {}


def exported_symbols() -> Sequence[str]:
    """Names declared in include/reduce.h that the binding knows about."""
    return ("reduce_status_str", "reduce_last_error", "reduce_version", "reduce_calibrate",
            "reduce_register_ws", "reduce_register", "reduce_valid_rect", "reduce_shift",
            "reduce_shift_spline_ws", "reduce_shift_spline", "reduce_mask_shifted",
            "reduce_combine", "reduce_prof_enable", "reduce_prof_query", "reduce_register_plan",
            "reduce_tune_register", "reduce_tune_register_ws", "reduce_tune_combine", "reduce_tune_save",
            "reduce_tune_load",
            "reduce_tune_clear", "reduce_stack_batch_ws", "reduce_stack_batch",
            "reduce_cnn_input_ws", "reduce_cnn_input", "reduce_cnn_num_params", "reduce_cnn_ws",
            "reduce_cnn_ws_offsets", "reduce_cnn_forward", "reduce_cnn_backward", "reduce_cnn_adamw",
            "reduce_cnn_centres", "reduce_render_frames", "reduce_recentre", "reduce_propose_ws",
            "reduce_propose", "reduce_register_static_max", "reduce_register_static", "reduce_register_fft_ws",
            "reduce_register_fft", "reduce_tune_search")


def _check(rc: int) -> None:
    if rc != OK:
        raise ReduceError(rc, lib().reduce_last_error().decode())


def prof_enable(on: bool = True) -> None:
    _check(lib().reduce_prof_enable(1 if on else 0))


def prof_query(kernel: str):
    """(total milliseconds, launches) of one kernel since prof_enable(True)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().reduce_prof_query(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return t


def _raw_view(raw: torch.Tensor) -> torch.Tensor:
    if raw.dtype not in (torch.uint16, torch.int16):
        raise TypeError("raw must be uint16 (or int16 carrying the same bits)")
    return raw


# ---------------------------------------------------------------------------- calibrate
def calibrate(raw: torch.Tensor, dark: torch.Tensor, flat: torch.Tensor,
              out: Optional[torch.Tensor] = None, stream=None, bias: Optional[torch.Tensor] = None) -> torch.Tensor:
    """raw [N][H][W] uint16 (row/frame strides honoured), bias (or None)/dark/flat [H][W] float32."""
    raw = _raw_view(_dev(raw, "raw"))
    if raw.dim() == 2:
        raw = raw.unsqueeze(0)
    N, H, W = raw.shape
    if raw.stride(2) != 1 or dark.stride(1) != 1 or flat.stride() != dark.stride():
        raise ValueError("x must be contiguous and dark/flat must share strides")
    if dark.dtype != torch.float32 or flat.dtype != torch.float32:
        raise TypeError("dark and flat must be float32")
    if bias is not None and (bias.dtype != torch.float32 or bias.stride() != dark.stride()):
        raise ValueError("bias must be float32 with the strides of dark")
    if out is None:
        out = torch.empty((N, H, W), dtype=torch.float32, device=raw.device)
    _check(lib().reduce_calibrate(_ptr(raw), raw.stride(1), raw.stride(0), _ptr(bias), _ptr(dark), _ptr(flat),
                                  dark.stride(0), _ptr(out), W, H, N, _stream(stream)))
    return out


# ---------------------------------------------------------------------------- register
def register_ws_bytes(W: int, H: int, N: int, radius: int, radius_max: Optional[int] = None) -> int:
    return int(lib().reduce_register_ws(W, H, N, radius, radius if radius_max is None else radius_max))


def register_fft_ws_bytes(W: int, H: int, N: int, radius: int) -> int:
    return int(lib().reduce_register_fft_ws(W, H, N, radius))


def register_fft(ref: torch.Tensor, frames: torch.Tensor, radius: int, want_scores: bool = False,
                 want_info: bool = False, ws: Optional[torch.Tensor] = None, stream=None):
    """Full-window search with the scores evaluated from row spectra and the offsets from
    exact direct sums (reduce_register_fft).  Returns the offsets (device uint8 [N][48]),
    and the spectral score cube and the per-frame decision codes if asked."""
    _dev(ref, "ref")
    _dev(frames, "frames")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    if not (ref.is_contiguous() and frames.is_contiguous()):
        raise ValueError("ref and frames must be contiguous")
    need = register_fft_ws_bytes(W, H, N, radius)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=frames.device)
    out = torch.empty((N, OFFSET_BYTES), dtype=torch.uint8, device=frames.device)
    D = 2 * radius + 1
    scores = torch.empty((N, D, D), dtype=torch.float64, device=frames.device) if want_scores else None
    info = torch.empty(N, dtype=torch.int32, device=frames.device) if want_info else None
    _check(lib().reduce_register_fft(_ptr(ref), _ptr(frames), W, H, N, radius, _ptr(out), _ptr(scores), _ptr(info),
                                     _ptr(ws), ws.numel(), _stream(stream)))
    res = [out]
    if want_scores:
        res.append(scores)
    if want_info:
        res.append(info)
    return res[0] if len(res) == 1 else tuple(res)


def register_static(ref: torch.Tensor, frames: torch.Tensor, radius: int, radius_max: Optional[int] = None,
                    centers: Optional[torch.Tensor] = None, tmpl: Optional[Sequence[int]] = None,
                    out: Optional[torch.Tensor] = None, scores: Optional[torch.Tensor] = None, stream=None):
    """register() through the entry point that allocates nothing (its workspace is the
    library's fixed per-device array): out (and scores, if given) must be caller-provided
    device tensors, [N][48] uint8 and float64 [N][2R+1][2R+1]."""
    _dev(ref, "ref")
    _dev(frames, "frames")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    rmax = radius if radius_max is None else radius_max
    if not (ref.is_contiguous() and frames.is_contiguous()):
        raise ValueError("ref and frames must be contiguous")
    if out is None or out.shape != (N, OFFSET_BYTES) or out.dtype != torch.uint8:
        raise ValueError("out must be a device uint8 tensor [N][48]")
    if scores is not None and (scores.dtype != torch.float64 or scores.shape != (N, 2 * radius + 1, 2 * radius + 1)):
        raise ValueError("scores must be a device float64 tensor [N][2R+1][2R+1]")
    if centers is not None:
        centers = _dev(centers, "centers")
        if centers.dtype != torch.int32 or not centers.is_contiguous():
            raise TypeError("centers must be a contiguous int32 device tensor [N][2]")
    t = None if tmpl is None else (ctypes.c_int32 * 4)(*[int(v) for v in tmpl])
    _check(lib().reduce_register_static(_ptr(ref), _ptr(frames), W, H, N, radius, rmax, _ptr(centers), t,
                                        _ptr(out), _ptr(scores), _stream(stream)))
    return out


def register(ref: torch.Tensor, frames: torch.Tensor, radius: int, radius_max: Optional[int] = None,
             centers: Optional[torch.Tensor] = None, tmpl: Optional[Sequence[int]] = None,
             want_scores: bool = False, ws: Optional[torch.Tensor] = None, stream=None):
    """Returns a device uint8 tensor [N][48] of reduce_offset_t (decode with offsets_to_numpy)
    and, if asked, the score cube float64 [N][2R+1][2R+1]."""
    _dev(ref, "ref")
    _dev(frames, "frames")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    rmax = radius if radius_max is None else radius_max
    if not (ref.is_contiguous() and frames.is_contiguous()):
        raise ValueError("ref and frames must be contiguous")
    need = register_ws_bytes(W, H, N, radius, rmax)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=frames.device)
    out = torch.empty((N, OFFSET_BYTES), dtype=torch.uint8, device=frames.device)
    scores = (torch.empty((N, 2 * radius + 1, 2 * radius + 1), dtype=torch.float64, device=frames.device)
              if want_scores else None)
    if centers is not None:
        centers = _dev(centers, "centers")
        if centers.dtype != torch.int32 or not centers.is_contiguous():
            raise TypeError("centers must be a contiguous int32 device tensor [N][2]")
    t = None
    if tmpl is not None:
        t = (ctypes.c_int32 * 4)(*[int(v) for v in tmpl])
    _check(lib().reduce_register(_ptr(ref), _ptr(frames), W, H, N, radius, rmax, _ptr(centers),
                                 t, _ptr(out), _ptr(scores), _ptr(ws), ws.numel(), _stream(stream)))
    return (out, scores) if want_scores else out


PLAN_FIELDS = ("D", "K", "NBX", "C", "G", "CW", "S", "threads", "TX", "TY", "BR", "JS", "FR", "FC",
               "lds", "n_tiles")


def register_plan(W: int, H: int, N: int, radius: int, radius_max: Optional[int] = None) -> dict:
    f = (ctypes.c_int32 * 16)()
    _check(lib().reduce_register_plan(W, H, N, radius, radius if radius_max is None else radius_max, f))
    return dict(zip(PLAN_FIELDS, list(f)))


def tune_register(ref: torch.Tensor, frames: torch.Tensor, radius: int, radius_max: Optional[int] = None,
                  reps: int = 3, stream=None) -> dict:
    """Time candidate launch shapes of the search on these frames; caches and returns the winner."""
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    rmax = radius if radius_max is None else radius_max
    ws = torch.empty(max(int(lib().reduce_tune_register_ws(W, H, N, radius, rmax)), 1), dtype=torch.uint8,
                     device=frames.device)
    out = torch.empty((N, OFFSET_BYTES), dtype=torch.uint8, device=frames.device)
    f = (ctypes.c_int32 * 16)()
    _check(lib().reduce_tune_register(_ptr(ref), _ptr(frames), W, H, N, radius, rmax, _ptr(out), _ptr(ws),
                                      ws.numel(), reps, _stream(stream), f))
    return dict(zip(PLAN_FIELDS, list(f)))


def tune_combine(aligned: torch.Tensor, ksigma: float = 3.0, max_iters: int = 3, reps: int = 3,
                 stream=None) -> int:
    N, h, w = aligned.shape
    out = torch.empty((h, w), dtype=torch.float32, device=aligned.device)
    lanes = ctypes.c_int32(0)
    _check(lib().reduce_tune_combine(_ptr(aligned), w, h, N, float(ksigma), int(max_iters), _ptr(out), reps,
                                     _stream(stream), ctypes.byref(lanes)))
    return lanes.value


def tune_save(path: str) -> None:
    _check(lib().reduce_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _check(lib().reduce_tune_load(path.encode()))


def tune_search(ref: torch.Tensor, frames: torch.Tensor, radius: int, reps: int = 3, stream=None) -> dict:
    """Times the full-window search with direct sums and through row spectra on these
    frames; returns {"search": "direct" | "spectral", "ms_direct", "ms_spectral"}."""
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    need = max(register_ws_bytes(W, H, N, radius), register_fft_ws_bytes(W, H, N, radius))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=frames.device)
    out = torch.empty((N, OFFSET_BYTES), dtype=torch.uint8, device=frames.device)
    srch = ctypes.c_int32(0)
    md, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().reduce_tune_search(_ptr(ref.contiguous()), _ptr(frames.contiguous()), W, H, N, radius, _ptr(out),
                                    _ptr(ws), ws.numel(), int(reps), _stream(stream), ctypes.byref(srch),
                                    ctypes.byref(md), ctypes.byref(ms)))
    return {"search": "spectral" if srch.value == SEARCH_SPECTRAL else "direct", "ms_direct": md.value,
            "ms_spectral": ms.value}


def tune_clear() -> None:
    _check(lib().reduce_tune_clear())


def offsets_to_numpy(raw_offsets: torch.Tensor) -> np.ndarray:
    """Device reduce_offset_t bytes -> host structured array (a copy; synchronises)."""
    b = raw_offsets.detach().cpu().numpy().reshape(-1)
    return b.view(OFFSET_DTYPE).copy()


# ---------------------------------------------------------------------------- overlap / shift
def valid_rect(offs: np.ndarray, W: int, H: int) -> np.ndarray:
    o = np.ascontiguousarray(offs, dtype=np.float32).reshape(-1, 2)
    rect = np.zeros(4, dtype=np.int32)
    _check(lib().reduce_valid_rect(o.ctypes.data_as(ctypes.c_void_p), o.shape[0], W, H,
                                   rect.ctypes.data_as(ctypes.c_void_p)))
    return rect


def shift(frames: torch.Tensor, offs: torch.Tensor, rect: Sequence[int], integer_mode: bool = False,
          out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """frames float32 [N][H][W], offs float32 device [N][2], rect host (x0, y0, w, h)."""
    _dev(frames, "frames")
    _dev(offs, "offs")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    if offs.dtype != torch.float32 or not offs.is_contiguous() or offs.numel() != 2 * N:
        raise TypeError("offs must be a contiguous float32 device tensor [N][2]")
    r = (ctypes.c_int32 * 4)(*[int(v) for v in rect])
    if out is None:
        out = torch.empty((N, int(rect[3]), int(rect[2])), dtype=torch.float32, device=frames.device)
    _check(lib().reduce_shift(_ptr(frames.contiguous()), _ptr(out), W, H, N, _ptr(offs), r,
                              1 if integer_mode else 0, _stream(stream)))
    return out


def shift_spline(frames: torch.Tensor, offs: torch.Tensor, rect: Sequence[int], out: Optional[torch.Tensor] = None,
                 ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Bicubic-spline shift: frames float32 [N][H][W], offs float32 device [N][2], rect host
    (x0, y0, w, h) -> [N][h][w]."""
    _dev(frames, "frames")
    _dev(offs, "offs")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    if offs.dtype != torch.float32 or not offs.is_contiguous() or offs.numel() != 2 * N:
        raise TypeError("offs must be a contiguous float32 device tensor [N][2]")
    r = (ctypes.c_int32 * 4)(*[int(v) for v in rect])
    if out is None:
        out = torch.empty((N, int(rect[3]), int(rect[2])), dtype=torch.float32, device=frames.device)
    if ws is None:
        ws = torch.empty(max(int(lib().reduce_shift_spline_ws(W, H, N)), 1), dtype=torch.uint8, device=frames.device)
    _check(lib().reduce_shift_spline(_ptr(frames.contiguous()), _ptr(out), W, H, N, _ptr(offs), r, _ptr(ws),
                                     ws.numel(), _stream(stream)))
    return out


# ---------------------------------------------------------------------------- combine
def combine(aligned: torch.Tensor, ksigma: float = 3.0, max_iters: int = 3, want_keep: bool = False,
            want_nrej: bool = False, out: Optional[torch.Tensor] = None, stream=None, missing: bool = False):
    """Returns (out [h][w] float32, keep uint8 [N][h][w] or None, n_rej int64 [1] or None);
    with missing, NaN values are left out."""
    _dev(aligned, "aligned")
    N, h, w = aligned.shape
    if not aligned.is_contiguous():
        raise ValueError("aligned must be contiguous")
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=aligned.device)
    elif out.dtype != torch.float32 or out.numel() != h * w or not out.is_contiguous():
        raise ValueError("out must be contiguous float32 [h][w]")
    keep = torch.empty((N, h, w), dtype=torch.uint8, device=aligned.device) if want_keep else None
    nrej = torch.empty(1, dtype=torch.int64, device=aligned.device) if want_nrej else None
    _check(lib().reduce_combine(_ptr(aligned), w, h, N, float(ksigma), int(max_iters), _ptr(out),
                                _ptr(keep), _ptr(nrej), 1 if missing else 0, _stream(stream)))
    return out, keep, nrej


def mask_shifted(mask: torch.Tensor, out: torch.Tensor, offs: torch.Tensor, rect: Sequence[int], W: int, H: int,
                 integer_mode: bool = False, stream=None) -> torch.Tensor:
    """Sets to NaN the values of shift()'s output out [N][h][w] that read a bad pixel of
    mask uint8 [H][W] (nonzero = bad)."""
    _dev(mask, "mask")
    _dev(out, "out")
    if mask.dtype != torch.uint8 or not mask.is_contiguous() or tuple(mask.shape) != (H, W):
        raise ValueError("mask must be a contiguous uint8 device tensor [H][W]")
    if out.dim() == 2:
        out = out.unsqueeze(0)
    N = out.shape[0]
    if not out.is_contiguous() or offs.numel() != 2 * N:
        raise ValueError("out must be contiguous [N][h][w] with offs [N][2]")
    r = (ctypes.c_int32 * 4)(*[int(v) for v in rect])
    _check(lib().reduce_mask_shifted(_ptr(mask), _ptr(out), W, H, N, _ptr(offs), r, 1 if integer_mode else 0,
                                     _stream(stream)))
    return out


# ---------------------------------------------------------------------------- batched stacks
class StackDesc(ctypes.Structure):
    """reduce_stack_t"""
    _fields_ = [("raw", ctypes.c_void_p), ("raw_row_pitch", ctypes.c_int64), ("raw_frame_pitch", ctypes.c_int64),
                ("dark", ctypes.c_void_p), ("flat", ctypes.c_void_p), ("cal_row_pitch", ctypes.c_int64),
                ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("N", ctypes.c_int32), ("ref_index", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("ksigma", ctypes.c_float),
                ("integer_mode", ctypes.c_int32), ("out", ctypes.c_void_p), ("out_rect", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("n_rej", ctypes.c_void_p), ("bias", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("search", ctypes.c_int32), ("pad", ctypes.c_int32)]


SEARCH_DIRECT, SEARCH_SPECTRAL = 0, 1


class StackBatch:
    """Device buffers and descriptors of a batch of stacks (caller-owned torch tensors).

    Each stack is (raw uint16 [N][H][W], dark [H][W], flat [H][W], radius) or that tuple
    followed by bias [H][W] (or None) and a bad-pixel map uint8 [H][W] (or None); search
    is "direct" or "spectral" (per stack with a list); outputs
    are allocated here once: out [H*W] float32 (the image is out[:h*w] as [h][w]),
    rect int32 [4], offsets [N][48] bytes, n_rej int64 [1].
    """

    def __init__(self, stacks, ksigma: float = 3.0, max_iters: int = 3, ref_index=0, integer_mode=False,
                 search="direct"):
        self.items = []
        descs = []
        for i, st in enumerate(stacks):
            raw, dark, flat, radius = st[:4]
            bias = st[4] if len(st) > 4 else None
            mask = st[5] if len(st) > 5 else None
            if mask is not None and (mask.dtype != torch.uint8 or not mask.is_contiguous()):
                raise ValueError("mask must be a contiguous uint8 tensor [H][W]")
            raw = _raw_view(_dev(raw, "raw"))
            N, H, W = raw.shape
            dev = raw.device
            ref = ref_index[i] if isinstance(ref_index, (list, tuple)) else ref_index
            imode = integer_mode[i] if isinstance(integer_mode, (list, tuple)) else integer_mode
            srch = search[i] if isinstance(search, (list, tuple)) else search
            if srch not in ("direct", "spectral"):
                raise ValueError("search must be 'direct' or 'spectral'")
            out = torch.empty(H * W, dtype=torch.float32, device=dev)
            rect = torch.zeros(4, dtype=torch.int32, device=dev)
            offs = torch.zeros((N, OFFSET_BYTES), dtype=torch.uint8, device=dev)
            nrej = torch.zeros(1, dtype=torch.int64, device=dev)
            d = StackDesc(raw.data_ptr(), raw.stride(1), raw.stride(0), dark.data_ptr(), flat.data_ptr(),
                          dark.stride(0), W, H, N, int(ref), int(radius), int(max_iters), float(ksigma),
                          1 if imode else 0, out.data_ptr(), rect.data_ptr(), offs.data_ptr(), nrej.data_ptr(),
                          0 if bias is None else bias.data_ptr(), 0 if mask is None else mask.data_ptr(),
                          SEARCH_SPECTRAL if srch == "spectral" else SEARCH_DIRECT, 0)
            descs.append(d)
            self.items.append(dict(raw=raw, dark=dark, flat=flat, bias=bias, mask=mask, out=out, rect=rect,
                                   offsets=offs, n_rej=nrej,
                                   W=W, H=H, N=N))
        self.descs = (StackDesc * len(descs))(*descs)
        self.n = len(descs)
        self.ws = None

    def ws_bytes(self) -> int:
        return int(lib().reduce_stack_batch_ws(self.descs, self.n))

    def run(self, stream=None) -> None:
        need = self.ws_bytes()
        if need == 0:
            raise ReduceError(ERR_SHAPE, "invalid batch: " + lib().reduce_last_error().decode())
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.items[0]["raw"].device)
        _check(lib().reduce_stack_batch(self.descs, self.n, _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def result(self, i: int):
        """(image [h][w] float32 tensor, rect numpy, offsets structured numpy, n_rej int)."""
        it = self.items[i]
        rect = it["rect"].cpu().numpy()
        h, w = int(rect[3]), int(rect[2])
        return it["out"][: h * w].view(h, w), rect, offsets_to_numpy(it["offsets"]), int(it["n_rej"].cpu()[0])


# ---------------------------------------------------------------------------- proposal network
def cnn_num_params() -> int:
    return int(lib().reduce_cnn_num_params())


def cnn_input_ws_bytes(W: int, H: int, N: int) -> int:
    return int(lib().reduce_cnn_input_ws(W, H, N))


def cnn_input(frames: torch.Tensor, out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
    """frames float32 [N][H][W] -> bfloat16 bits as int16 [N][H/4][W/4]."""
    _dev(frames, "frames")
    if frames.dim() == 2:
        frames = frames.unsqueeze(0)
    N, H, W = frames.shape
    if ws is None:
        ws = torch.empty(max(cnn_input_ws_bytes(W, H, N), 1), dtype=torch.uint8, device=frames.device)
    if out is None:
        out = torch.empty((N, H // 4, W // 4), dtype=torch.int16, device=frames.device)
    _check(lib().reduce_cnn_input(_ptr(frames.contiguous()), W, H, N, _ptr(out), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return out


def bf16_bits_to_float(t: torch.Tensor) -> torch.Tensor:
    """int16 tensor of bfloat16 bits -> float32 (a view change, no arithmetic)."""
    return t.contiguous().view(torch.bfloat16).float()


class CnnWorkspace:
    """Device workspace of the network for a batch shape (activations, gradients)."""

    def __init__(self, B: int, h: int, w: int, device="cuda:0"):
        self.B, self.h, self.w = B, h, w
        n = int(lib().reduce_cnn_ws(B, h, w))
        if n == 0:
            raise ReduceError(ERR_SHAPE, "bad network shape")
        self.buf = torch.empty(n, dtype=torch.uint8, device=device)
        off = (ctypes.c_int64 * 6)()
        _check(lib().reduce_cnn_ws_offsets(B, h, w, off))
        self.offsets = list(off)

    def activation(self, layer: int) -> torch.Tensor:
        """bfloat16 bits (int16) [B][h_l][w_l][32] of layer 1..4 after the last forward."""
        hl, wl = self.h, self.w
        for _ in range(layer):
            hl, wl = (hl + 1) // 2, (wl + 1) // 2
        n = self.B * hl * wl * 32
        o = self.offsets[layer - 1]
        return self.buf[o:o + 2 * n].view(torch.int16).view(self.B, hl, wl, 32)

    def grad_z(self, layer: int) -> torch.Tensor:
        """bfloat16 bits of dLoss/dZ of layer 1 or 2 after the last backward."""
        if layer not in (1, 2):
            raise ValueError("only the gradients of layers 1 and 2 stay in the workspace")
        shape = self.activation(layer).shape
        n = shape[0] * shape[1] * shape[2] * 32
        o = self.offsets[5 if layer == 1 else 4]
        return self.buf[o:o + 2 * n].view(torch.int16).view(shape)


def cnn_forward(ref_in: torch.Tensor, img_in: torch.Tensor, params: torch.Tensor, cws: CnnWorkspace,
                ref_shared: bool = True, pred: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """ref_in int16 [h][w] (shared) or [B][h][w]; img_in int16 [B][h][w]; params float32 -> pred [B][2]."""
    B, h, w = img_in.shape
    if pred is None:
        pred = torch.empty((B, 2), dtype=torch.float32, device=img_in.device)
    stride = 0 if ref_shared else h * w
    _check(lib().reduce_cnn_forward(_ptr(ref_in), stride, _ptr(img_in), B, h, w, _ptr(params), _ptr(pred),
                                    _ptr(cws.buf), cws.buf.numel(), _stream(stream)))
    return pred


def cnn_backward(ref_in: torch.Tensor, img_in: torch.Tensor, params: torch.Tensor, pred: torch.Tensor,
                 target: torch.Tensor, cws: CnnWorkspace, huber_delta: float = 1.0, ref_shared: bool = True,
                 grad: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None, stream=None):
    """(loss [1], grad [n]) after cnn_forward on the same inputs; all device float32."""
    B, h, w = img_in.shape
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    stride = 0 if ref_shared else h * w
    _check(lib().reduce_cnn_backward(_ptr(ref_in), stride, _ptr(img_in), B, h, w, _ptr(params), _ptr(pred),
                                     _ptr(target), float(huber_delta), _ptr(loss), _ptr(grad), _ptr(cws.buf),
                                     cws.buf.numel(), _stream(stream)))
    return loss, grad


def cnn_adamw(params, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, stream=None):
    _check(lib().reduce_cnn_adamw(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), float(lr),
                                  float(beta1), float(beta2), float(eps), float(weight_decay), int(step),
                                  _stream(stream)))


def cnn_centres(pred: torch.Tensor, scale: float = 4.0, radius_max: int = 64, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """int32 [B][2] window centres from a [B][2] prediction."""
    B = pred.shape[0]
    if out is None:
        out = torch.empty((B, 2), dtype=torch.int32, device=pred.device)
    _check(lib().reduce_cnn_centres(_ptr(pred), B, float(scale), int(radius_max), _ptr(out), _stream(stream)))
    return out


def render_frames(stars: torch.Tensor, keys: torch.Tensor, W: int, H: int, sky: float = 1000.0,
                  fwhm: float = 3.0, read_noise: float = 10.0, noise: bool = True, seed: int = 0,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """stars device float32 [F][S][4], keys device int64 [F] -> frames float32 [F][H][W]."""
    F_, S = stars.shape[0], stars.shape[1]
    if stars.dtype != torch.float32 or stars.shape[2] != 4 or not stars.is_contiguous():
        raise ValueError("stars must be contiguous float32 [F][S][4]")
    if keys.dtype != torch.int64 or keys.numel() != F_:
        raise ValueError("keys must be int64 [F]")
    if out is None:
        out = torch.empty((F_, H, W), dtype=torch.float32, device=stars.device)
    _check(lib().reduce_render_frames(_ptr(stars), S, _ptr(keys), F_, W, H, float(sky), float(fwhm),
                                      float(read_noise), 1 if noise else 0, int(seed) & (2 ** 64 - 1), _ptr(out),
                                      _stream(stream)))
    return out


def recentre(offsets: torch.Tensor, centres: torch.Tensor, radius_max: int, stream=None) -> torch.Tensor:
    """Move the centres of frames whose window maximum is on the border (in place)."""
    N = centres.shape[0]
    if offsets.numel() != N * OFFSET_BYTES or centres.dtype != torch.int32 or not centres.is_contiguous():
        raise ValueError("offsets [N][48] bytes and contiguous int32 centres [N][2] needed")
    _check(lib().reduce_recentre(_ptr(offsets), N, int(radius_max), _ptr(centres), _stream(stream)))
    return centres


def propose_ws_bytes(W: int, H: int, N: int, refine_radius: int = 2, radius_max: int = 64) -> int:
    return int(lib().reduce_propose_ws(W, H, N, refine_radius, radius_max))


def propose(ref: torch.Tensor, frames: torch.Tensor, params: torch.Tensor, radius_max: int = 64,
            refine_radius: int = 2, peak_ratio: float = 0.5, max_moves: int = 4, ws: Optional[torch.Tensor] = None,
            out: Optional[torch.Tensor] = None, centres: Optional[torch.Tensor] = None,
            info: Optional[torch.Tensor] = None, stream=None):
    """Network proposal, narrowed search, window moves and full-search fallback in one call:
    ref [H][W], frames [N][H][W] float32, params float32 -> (offsets [N][48] bytes, centres
    int32 [N][2], info int32 [N]), all on the device."""
    _dev(ref, "ref")
    _dev(frames, "frames")
    N, H, W = frames.shape
    if not (ref.is_contiguous() and frames.is_contiguous() and params.is_contiguous()):
        raise ValueError("ref, frames and params must be contiguous")
    if params.dtype != torch.float32 or params.numel() != cnn_num_params():
        raise ValueError("params must be the network's float32 parameter vector")
    need = propose_ws_bytes(W, H, N, refine_radius, radius_max)
    if need == 0:
        raise ReduceError(ERR_SHAPE, "reduce_propose: unsupported sizes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=frames.device)
    if out is None:
        out = torch.empty((N, OFFSET_BYTES), dtype=torch.uint8, device=frames.device)
    if centres is None:
        centres = torch.empty((N, 2), dtype=torch.int32, device=frames.device)
    if info is None:
        info = torch.empty(N, dtype=torch.int32, device=frames.device)
    _check(lib().reduce_propose(_ptr(ref), _ptr(frames), W, H, N, _ptr(params), int(refine_radius), int(radius_max),
                                float(peak_ratio), int(max_moves), _ptr(out), _ptr(centres), _ptr(info), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return out, centres, info
