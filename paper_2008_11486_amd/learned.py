"""Offset proposals from the small convolutional network.

* ``pair_catalogues`` / ``stack_catalogue`` draw star catalogues and true offsets for
  training pairs and evaluation stacks; the frames themselves are rendered on the GPU
  (``render_frames``), converted to the network input on the GPU (``cnn_input``), so
  the network learns from what the pipeline produces.
* ``ProposalTrainer`` runs forward, Huber-loss backward and AdamW, all in the
  library's kernels, on freshly rendered pairs.
* ``LearnedRegistrar`` marshals ``reduce_propose``: the network proposes an offset per
  frame, the search runs only in a small window around it with the same template as
  the full search (a window whose maximum lies on its border moves onto that maximum,
  a few times at most), and the full window replaces the result when the narrowed one
  cannot be trusted (its maximum still on a window border inside the search limit, or
  a peak far below the reference's own zero-offset score); all of it on the device.

The registration problem itself (score, argmax, sub-pixel vertex) is the one of
``reduce_register``; the network only moves the window.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import (CLIPPED, FALLBACK, OFFSET_BYTES, CnnWorkspace, cnn_adamw, cnn_backward, cnn_forward, cnn_input,
               cnn_input_ws_bytes, cnn_num_params, offsets_to_numpy, propose, propose_ws_bytes, register,
               render_frames)

SEED_ROOT = 20081148
STAR_DENSITY = 200.0 / (1024 * 1024)     # stars per pixel, as in the 1024x1024 stacks
AMP_RANGE = (2.0e3, 5.0e4)               # peak amplitude, log-uniform
SKY, FWHM, READ_NOISE = 1000.0, 3.0, 10.0
DOWNSAMPLE = 4
CNN_CIN = (2, 32, 32, 32)
CNN_CH = 32
TRAIN_SET, EVAL_SET = 0, 1


def _rng(*words) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 4, *[int(w) for w in words]])))


def _draw_stars(rng, n, W, H, pad):
    x = rng.uniform(-pad, W - 1 + pad, n)
    y = rng.uniform(-pad, H - 1 + pad, n)
    amp = np.exp(rng.uniform(math.log(AMP_RANGE[0]), math.log(AMP_RANGE[1]), n))
    return x, y, amp


def n_stars(W: int, H: int) -> int:
    return max(1, int(round(STAR_DENSITY * W * H)))


def _key(set_id, index, frame):
    return (int(set_id) << 48) | (int(index) << 8) | int(frame)


def pair_catalogues(indices: Sequence[int], W: int, H: int, shift_bound: float, set_id: int = TRAIN_SET):
    """Catalogues of B pairs: stars float32 [2B][S][4] (B references, then the B shifted
    frames), keys int64 [2B], true offsets float64 [B][2] with frame(x + t) = ref(x)."""
    B, S = len(indices), n_stars(W, H)
    stars = np.zeros((2 * B, S, 4), np.float32)
    keys = np.zeros(2 * B, np.int64)
    t = np.zeros((B, 2))
    for j, i in enumerate(indices):
        rng = _rng(set_id, i)
        x, y, amp = _draw_stars(rng, S, W, H, shift_bound + 8)
        t[j] = rng.uniform(-shift_bound, shift_bound, 2)
        stars[j, :, 0], stars[j, :, 1], stars[j, :, 2] = x, y, amp
        stars[B + j, :, 0], stars[B + j, :, 1], stars[B + j, :, 2] = x + t[j, 0], y + t[j, 1], amp
        keys[j], keys[B + j] = _key(set_id, i, 0), _key(set_id, i, 1)
    return stars, keys, t


def stack_catalogue(index: int, n_frames: int, W: int, H: int, shift_bound: float, set_id: int = EVAL_SET):
    """One reference (frame 0, offset 0) and n_frames - 1 shifted frames of one sky."""
    S = n_stars(W, H)
    rng = _rng(set_id, index)
    x, y, amp = _draw_stars(rng, S, W, H, shift_bound + 8)
    t = np.zeros((n_frames, 2))
    t[1:] = rng.uniform(-shift_bound, shift_bound, (n_frames - 1, 2))
    stars = np.zeros((n_frames, S, 4), np.float32)
    for k in range(n_frames):
        stars[k, :, 0], stars[k, :, 1], stars[k, :, 2] = x + t[k, 0], y + t[k, 1], amp
    keys = np.array([_key(set_id, index, k) for k in range(n_frames)], np.int64)
    return stars, keys, t


def render_stack(index: int, n_frames: int, W: int, H: int, shift_bound: float, set_id: int = EVAL_SET,
                 device="cuda:0", seed: int = SEED_ROOT):
    """Device frames [n_frames][H][W] of stack_catalogue and the true offsets."""
    stars, keys, t = stack_catalogue(index, n_frames, W, H, shift_bound, set_id)
    frames = render_frames(torch.from_numpy(stars).to(device), torch.from_numpy(keys).to(device), W, H,
                           sky=SKY, fwhm=FWHM, read_noise=READ_NOISE, seed=seed)
    return frames, t


def param_slices() -> dict:
    """Slices of the flat parameter vector (W1 b1 ... W4 b4 Wl bl)."""
    out, o = {}, 0
    for i, cin in enumerate(CNN_CIN):
        n = 9 * cin * CNN_CH
        out[f"w{i + 1}"] = (slice(o, o + n), (9, cin, CNN_CH))
        o += n
        out[f"b{i + 1}"] = (slice(o, o + CNN_CH), (CNN_CH,))
        o += CNN_CH
    out["wl"] = (slice(o, o + 2 * CNN_CH), (2, CNN_CH))
    o += 2 * CNN_CH
    out["bl"] = (slice(o, o + 2), (2,))
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal convolution weights, zero biases, a small linear head."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(cnn_num_params(), np.float32)
    sl = param_slices()
    for i, cin in enumerate(CNN_CIN):
        s, shape = sl[f"w{i + 1}"]
        p[s] = rng.normal(0.0, math.sqrt(2.0 / (9 * cin)), int(np.prod(shape)))
    s, shape = sl["wl"]
    p[s] = rng.normal(0.0, 1.0 / math.sqrt(CNN_CH), int(np.prod(shape)))
    return p


def save_params(path: str, params) -> None:
    p = params.detach().cpu().numpy() if isinstance(params, torch.Tensor) else np.asarray(params)
    np.save(path, p.astype(np.float32), allow_pickle=False)


def load_params(path: str) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (cnn_num_params(),):
        raise ValueError(f"{path}: expected float32 [{cnn_num_params()}]")
    return p


class ProposalTrainer:
    """AdamW training of the proposal network on rendered pairs (targets: t / 4)."""

    def __init__(self, W: int, H: int, batch: int, shift_bound: float, lr: float = 1e-3,
                 weight_decay: float = 1e-4, huber_delta: float = 1.0, seed: int = 0,
                 params: Optional[np.ndarray] = None, device="cuda:0"):
        if W % DOWNSAMPLE or H % DOWNSAMPLE:
            raise ValueError("frame sides must be multiples of 4")
        self.W, self.H, self.B, self.bound = W, H, batch, shift_bound
        self.lr, self.wd, self.delta = lr, weight_decay, huber_delta
        self.dev = torch.device(device)
        self.h, self.w = H // DOWNSAMPLE, W // DOWNSAMPLE
        p0 = init_params(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p0.copy()).to(self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.empty_like(self.params)
        self.loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        self.pred = torch.empty((batch, 2), dtype=torch.float32, device=self.dev)
        self.frames = torch.empty((2 * batch, H, W), dtype=torch.float32, device=self.dev)
        self.inp = torch.empty((2 * batch, self.h, self.w), dtype=torch.int16, device=self.dev)
        self.in_ws = torch.empty(max(cnn_input_ws_bytes(W, H, 2 * batch), 1), dtype=torch.uint8, device=self.dev)
        self.cws = CnnWorkspace(batch, self.h, self.w, device=self.dev)
        self.steps = 0

    def step(self, indices: Sequence[int], lr: Optional[float] = None) -> torch.Tensor:
        if len(indices) != self.B:
            raise ValueError("one index per batch item")
        stars, keys, t = pair_catalogues(indices, self.W, self.H, self.bound, TRAIN_SET)
        render_frames(torch.from_numpy(stars).to(self.dev), torch.from_numpy(keys).to(self.dev), self.W, self.H,
                      sky=SKY, fwhm=FWHM, read_noise=READ_NOISE, seed=SEED_ROOT, out=self.frames)
        cnn_input(self.frames, out=self.inp, ws=self.in_ws)
        B = self.B
        ref, img = self.inp[:B], self.inp[B:]
        cnn_forward(ref, img, self.params, self.cws, ref_shared=False, pred=self.pred)
        target = torch.from_numpy((t / DOWNSAMPLE).astype(np.float32)).to(self.dev)
        cnn_backward(ref, img, self.params, self.pred, target, self.cws, huber_delta=self.delta,
                     ref_shared=False, grad=self.grad, loss=self.loss)
        self.steps += 1
        cnn_adamw(self.params, self.m, self.v, self.grad, self.lr if lr is None else lr, self.steps,
                  weight_decay=self.wd)
        return self.loss

    def train(self, n_pairs: int, epochs: int, warmup: int = 100, min_lr_frac: float = 0.01,
              log_every: int = 50, shuffle_seed: int = 1, log=None, time_budget: Optional[float] = None) -> list:
        """Cosine schedule over epochs x n_pairs / B steps (or over time_budget seconds,
        stopping when it is spent); returns (step, loss) pairs."""
        per_epoch = n_pairs // self.B
        total = per_epoch * epochs
        rng = np.random.Generator(np.random.PCG64(shuffle_seed))
        history = []
        s = 0
        t0 = time.perf_counter()
        for _ in range(epochs):
            order = rng.permutation(n_pairs)
            for k in range(per_epoch):
                if time_budget is not None:
                    frac = (time.perf_counter() - t0) / time_budget
                    if frac >= 1.0:
                        break
                else:
                    frac = s / max(total - 1, 1)
                lr = self.lr * (min_lr_frac + (1 - min_lr_frac) * 0.5 * (1 + math.cos(math.pi * frac)))
                if s < warmup:
                    lr *= (s + 1) / warmup
                loss = self.step(order[k * self.B:(k + 1) * self.B], lr=lr)
                if s % log_every == 0 or s == total - 1:
                    history.append((s, float(loss.item())))
                    if log:
                        log(f"step {s}/{total} loss {history[-1][1]:.4f} lr {lr:.2e} "
                            f"{time.perf_counter() - t0:.0f} s")
                s += 1
            else:
                continue
            break
        if history and history[-1][0] != s - 1:
            history.append((s - 1, float(loss.item())))
        return history


@dataclass
class LearnedResult:
    offsets: np.ndarray            # reduce_offset_t records (FALLBACK set where the full window ran)
    centres: np.ndarray            # int32 [M][2] window centres from the network
    fallback: np.ndarray           # bool [M]
    reason: dict = field(default_factory=dict)


class LearnedRegistrar:
    """Network proposal -> narrowed search -> window moves -> full-window fallback, for
    frames [M][H][W] against one reference [H][W] (all device float32): one
    ``reduce_propose`` call, every decision taken on the device."""

    def __init__(self, params, W: int, H: int, M: int, radius_max: int = 64, refine_radius: int = 2,
                 peak_ratio: float = 0.5, moves: int = 4, device="cuda:0"):
        self.W, self.H, self.M = W, H, M
        self.rmax, self.r = radius_max, refine_radius
        self.moves = moves
        self.peak_ratio = peak_ratio
        self.dev = torch.device(device)
        p = params if isinstance(params, torch.Tensor) else torch.from_numpy(np.asarray(params, np.float32))
        self.params = p.to(self.dev).contiguous()
        self.ws = torch.empty(max(propose_ws_bytes(W, H, M, refine_radius, radius_max), 1), dtype=torch.uint8,
                              device=self.dev)
        self.out = torch.empty((M, OFFSET_BYTES), dtype=torch.uint8, device=self.dev)
        self.centres = torch.empty((M, 2), dtype=torch.int32, device=self.dev)
        self.info = torch.empty(M, dtype=torch.int32, device=self.dev)

    def enqueue(self, ref: torch.Tensor, frames: torch.Tensor) -> torch.Tensor:
        """Enqueue the whole learned registration; returns the device offsets."""
        if frames.shape != (self.M, self.H, self.W):
            raise ValueError(f"frames must be [{self.M}][{self.H}][{self.W}]")
        propose(ref, frames, self.params, radius_max=self.rmax, refine_radius=self.r, peak_ratio=self.peak_ratio,
                max_moves=self.moves, ws=self.ws, out=self.out, centres=self.centres, info=self.info)
        return self.out

    def register(self, ref: torch.Tensor, frames: torch.Tensor) -> LearnedResult:
        self.enqueue(ref, frames)
        o = offsets_to_numpy(self.out)
        info = self.info.cpu().numpy()
        fb = (o["flags"] & FALLBACK) != 0
        return LearnedResult(offsets=o, centres=self.centres.cpu().numpy(), fallback=fb,
                             reason=dict(border=int(((info >> 8) & 1).sum()), weak=int(((info >> 9) & 1).sum()),
                                         moves=int((info & 255).sum()),
                                         clipped=int(((o["flags"] & CLIPPED) != 0).sum())))


def full_search(ref: torch.Tensor, frames: torch.Tensor, radius_max: int = 64, ws=None) -> torch.Tensor:
    """The plain full-window search (device offsets)."""
    return register(ref, frames, radius_max, radius_max, ws=ws)


def time_call(fn, reps: int = 3) -> float:
    """Median wall time (s) of fn() with a device sync on both sides."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))
