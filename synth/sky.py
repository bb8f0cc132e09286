"""Seeded synthetic CCD frames standing in for the paper's telescope data.

The paper reduces 16-bit frames from three-band CCD cameras (Section 2.1) and, for
its scaling runs, frames of random values (Section 3.2.2).  Neither data set is
available, so every test and benchmark draws frames from this generator.  It holds
none of the reduction arithmetic: it only renders a sky, a dark and a flat and
quantises the result to uint16.

Recipe (all seeded through numpy's PCG64 from ``SeedSequence([20081148, cfg])``):

* sky background B = 1000 ADU, gain 1 e-/ADU;
* circular Gaussian stars, FWHM 3 px, evaluated at integer pixel centres inside a
  square box of half-width ceil(6 sigma); peak amplitude log-uniform on
  [2e3, 5e4] ADU; positions uniform on the reference canvas padded by the shift
  bound plus the stamp radius;
* frame k renders every star at p + t_k with t_0 = 0, so that
  frame(x + t_k) = ref(x) holds for the noiseless image at any sub-pixel t_k;
* raw = clip(round(Poisson(flat * S_k) + dark + N(0, 10^2) [+ cosmic rays]), 0, 65535);
* dark = 100 + N(0, 3^2) ADU and flat ~ U[0.95, 1.05], both fixed per stack;
* cosmic rays (wide-field case): round(1e-4 W H / 2.5) tracks per frame, each of
  length U{1..4} in one of 8 directions, each hit pixel adding U(5e3, 6e4) ADU.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ENTROPY = 20081148
SKY_ADU = 1000.0
READ_NOISE_ADU = 10.0
DARK_MEAN_ADU = 100.0
DARK_SIGMA_ADU = 3.0
FWHM_PX = 3.0
STAR_SIGMA_PX = FWHM_PX / (2.0 * math.sqrt(2.0 * math.log(2.0)))
STAMP_HALF = int(math.ceil(6.0 * STAR_SIGMA_PX))
AMP_RANGE = (2.0e3, 5.0e4)

_DIRECTIONS = ((1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1))


@dataclasses.dataclass(frozen=True)
class StackSpec:
    """Shape and sky model of one stack of frames.

    shift_kind is "int" (integer shifts U{-b..b}), "float" (continuous U(-b, b)),
    or "zero".  radius is the registration search radius used with this stack.
    """

    N: int
    W: int
    H: int
    n_stars: int
    shift_kind: str
    shift_bound: float
    radius: int
    cosmic: bool
    seed: tuple

    @property
    def pixels(self) -> int:
        return self.N * self.W * self.H


@dataclasses.dataclass
class Stack:
    spec: StackSpec
    raw: np.ndarray      # uint16 [N][H][W]
    dark: np.ndarray     # float32 [H][W]
    flat: np.ndarray     # float32 [H][W]
    shifts: np.ndarray   # float64 [N][2], (tx, ty) with frame(x + t) = ref(x)


def _stack_seq(seed: tuple) -> np.random.SeedSequence:
    return np.random.SeedSequence(list(seed))


def config_specs(cfg: int, *, n_stacks: Optional[int] = None) -> List[StackSpec]:
    """Stack specifications of the five benchmark workloads.

    0: one stack, 5 frames 512x512, 20 stars, integer shifts within +-8, R = 8.
    1: three bands x 10 frames 1024x1024, 200 stars, sub-pixel +-20, R = 21.
    2: 64 stacks, N ~ U{3..30}, side ~ {512, 1024, 2048, 4096}, sub-pixel +-16,
       R = 17, star density of workload 1.
    3: 16 frames 6144x6160, 5000 stars, cosmic rays, sub-pixel +-64, R = 65.
    4: learned-registration pairs 4096x4096 (N = 2), 3200 stars, +-64, R = 64.
    """
    base = (ENTROPY, cfg)
    if cfg == 0:
        return [StackSpec(5, 512, 512, 20, "int", 8, 8, False, base + (0,))]
    if cfg == 1:
        return [StackSpec(10, 1024, 1024, 200, "float", 20.0, 21, False, base + (b,))
                for b in range(3)]
    if cfg == 2:
        rng = np.random.Generator(np.random.PCG64(_stack_seq(base + (9999,))))
        count = 64 if n_stacks is None else n_stacks
        out = []
        for s in range(count):
            n = int(rng.integers(3, 31))
            side = int(rng.choice([512, 1024, 2048, 4096]))
            stars = int(round(200 * side * side / (1024 * 1024)))
            out.append(StackSpec(n, side, side, stars, "float", 16.0, 17, False, base + (s,)))
        return out
    if cfg == 3:
        return [StackSpec(16, 6144, 6160, 5000, "float", 64.0, 65, True, base + (0,))]
    if cfg == 4:
        count = 1 if n_stacks is None else n_stacks
        return [StackSpec(2, 4096, 4096, 3200, "float", 64.0, 64, False, base + (p,))
                for p in range(count)]
    raise ValueError(f"unknown workload {cfg}")


def small_spec(N: int, W: int, H: int, *, n_stars: int = 20, shift_kind: str = "float",
               shift_bound: float = 4.0, radius: Optional[int] = None,
               cosmic: bool = False, seed: Sequence[int] = (0,)) -> StackSpec:
    """A reduced stack for tests; same sky model, caller-chosen shape."""
    r = int(math.ceil(shift_bound)) + (1 if shift_kind == "float" else 0) if radius is None else radius
    return StackSpec(N, W, H, n_stars, shift_kind, float(shift_bound), r, cosmic,
                     (ENTROPY, 100) + tuple(seed))


def _draw_shifts(spec: StackSpec, rng: np.random.Generator) -> np.ndarray:
    t = np.zeros((spec.N, 2), dtype=np.float64)
    if spec.N > 1:
        if spec.shift_kind == "int":
            b = int(spec.shift_bound)
            t[1:] = rng.integers(-b, b + 1, size=(spec.N - 1, 2)).astype(np.float64)
        elif spec.shift_kind == "float":
            t[1:] = rng.uniform(-spec.shift_bound, spec.shift_bound, size=(spec.N - 1, 2))
        elif spec.shift_kind != "zero":
            raise ValueError(spec.shift_kind)
    return t


def _gauss_1d(centre: float, lo: int, hi: int) -> np.ndarray:
    x = np.arange(lo, hi, dtype=np.float64)
    return np.exp(-0.5 * ((x - centre) / STAR_SIGMA_PX) ** 2)


def render_sky(W: int, H: int, stars: np.ndarray, t: Sequence[float]) -> np.ndarray:
    """Noiseless sky in ADU (float64 [H][W]) with every star moved by t = (tx, ty)."""
    img = np.full((H, W), SKY_ADU, dtype=np.float64)
    tx, ty = float(t[0]), float(t[1])
    for px, py, amp in stars:
        cx, cy = px + tx, py + ty
        ix, iy = int(math.floor(cx + 0.5)), int(math.floor(cy + 0.5))
        x0, x1 = max(ix - STAMP_HALF, 0), min(ix + STAMP_HALF + 1, W)
        y0, y1 = max(iy - STAMP_HALF, 0), min(iy + STAMP_HALF + 1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        img[y0:y1, x0:x1] += amp * np.outer(_gauss_1d(cy, y0, y1), _gauss_1d(cx, x0, x1))
    return img


def cosmic_ray_hits(W: int, H: int, rng: np.random.Generator):
    """Pixels of one frame hit by cosmic-ray tracks and the ADU each hit adds:
    round(1e-4 W H / 2.5) tracks, each of length U{1..4} from a uniform start pixel in one
    of 8 directions, every hit pixel inside the frame adding U(5e3, 6e4).  Returns
    (ys, xs, adu) in draw order (a pixel may appear more than once)."""
    n_tracks = int(round(1e-4 * W * H / 2.5))
    lengths = rng.integers(1, 5, size=n_tracks)
    dirs = rng.integers(0, 8, size=n_tracks)
    xs = rng.integers(0, W, size=n_tracks)
    ys = rng.integers(0, H, size=n_tracks)
    hy, hx, adu = [], [], []
    for L, d, x, y in zip(lengths, dirs, xs, ys):
        ddx, ddy = _DIRECTIONS[d]
        for step in range(int(L)):
            px, py = int(x) + ddx * step, int(y) + ddy * step
            if 0 <= px < W and 0 <= py < H:
                hy.append(py)
                hx.append(px)
                adu.append(rng.uniform(5.0e3, 6.0e4))
    return np.array(hy, dtype=np.int64), np.array(hx, dtype=np.int64), np.array(adu, dtype=np.float64)


def _cosmic_rays(raw_f: np.ndarray, rng: np.random.Generator) -> None:
    H, W = raw_f.shape
    ys, xs, adu = cosmic_ray_hits(W, H, rng)
    np.add.at(raw_f, (ys, xs), adu)


def _stack_setup(spec: StackSpec):
    ss = _stack_seq(spec.seed)
    stack_ss, frames_ss = ss.spawn(2)
    rng = np.random.Generator(np.random.PCG64(stack_ss))
    dark = (DARK_MEAN_ADU + rng.normal(0.0, DARK_SIGMA_ADU, size=(spec.H, spec.W))).astype(np.float32)
    flat = rng.uniform(0.95, 1.05, size=(spec.H, spec.W)).astype(np.float32)
    pad = spec.shift_bound + STAMP_HALF
    stars = np.empty((spec.n_stars, 3), dtype=np.float64)
    stars[:, 0] = rng.uniform(-pad, spec.W + pad, size=spec.n_stars)
    stars[:, 1] = rng.uniform(-pad, spec.H + pad, size=spec.n_stars)
    lo, hi = np.log(AMP_RANGE[0]), np.log(AMP_RANGE[1])
    stars[:, 2] = np.exp(rng.uniform(lo, hi, size=spec.n_stars))
    shifts = _draw_shifts(spec, rng)
    return dark, flat, stars, shifts, frames_ss.spawn(spec.N)


def render_frame(spec: StackSpec, dark: np.ndarray, flat: np.ndarray, stars: np.ndarray,
                 t: np.ndarray, frame_ss: np.random.SeedSequence) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(frame_ss))
    sky = render_sky(spec.W, spec.H, stars, t)
    raw_f = rng.poisson(flat.astype(np.float64) * sky).astype(np.float64)
    raw_f += dark.astype(np.float64)
    raw_f += rng.normal(0.0, READ_NOISE_ADU, size=raw_f.shape)
    if spec.cosmic:
        _cosmic_rays(raw_f, rng)
    return np.clip(np.rint(raw_f), 0, 65535).astype(np.uint16)


def _frame_job(args):
    spec, k = args
    dark, flat, stars, shifts, frame_ss = _stack_setup(spec)
    return render_frame(spec, dark, flat, stars, shifts[k], frame_ss[k])


def make_stack(spec: StackSpec, workers: int = 1) -> Stack:
    """Render every frame of a stack; the result does not depend on ``workers``."""
    dark, flat, stars, shifts, frame_ss = _stack_setup(spec)
    raw = np.empty((spec.N, spec.H, spec.W), dtype=np.uint16)
    if workers > 1 and spec.N > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(min(workers, spec.N)) as pool:
            for k, frame in enumerate(pool.map(_frame_job, [(spec, k) for k in range(spec.N)])):
                raw[k] = frame
    else:
        for k in range(spec.N):
            raw[k] = render_frame(spec, dark, flat, stars, shifts[k], frame_ss[k])
    return Stack(spec, raw, dark, flat, shifts)


def make_config(cfg: int, *, n_stacks: Optional[int] = None, workers: int = 1) -> List[Stack]:
    return [make_stack(s, workers=workers) for s in config_specs(cfg, n_stacks=n_stacks)]
