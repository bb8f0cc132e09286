#!/usr/bin/env python
"""Throughput of the CCD reduction hot path on one MI355X.

One step = one pass of the whole path (dark subtraction + flat division, registration
against frame 0 of each stack, bilinear shift onto the common overlap, sigma-clipped
mean) over one batch of synthetic frames already resident in HBM.  The default
workload is three bands x 10 frames of 1024x1024 uint16 with sub-pixel shifts within
+-20 px (search radius 21) and a 3-sigma, 3-iteration clip.

Prints one JSON line: stacked Mpix/s (input pixels of all frames per second), the
roofline position of the dominant kernel (timed with HIP events on its own stream
over the timed steps), the streaming kernels' HBM fractions, and the FP64 CPU oracle
timed on this host as a baseline.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector FMA: 256 CUs x 64 lanes x 2 flop x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
METRIC = "stacked Mpix/s & % HBM peak; learned vs full-search registration speedup"

WORKLOADS = {
    1: "3 bands x 10 frames 1024x1024 uint16, 200 stars, sub-pixel shifts +-20 px, search radius 21, "
       "bilinear shift, 3-sigma clipped mean (3 iterations)",
    0: "5 frames 512x512 uint16, 20 stars, integer shifts +-8 px, search radius 8, integer shift, "
       "3-sigma clipped mean (3 iterations)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=1, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the cost-model launch shapes")
    ap.add_argument("--path", choices=("stagewise", "batched"), default="batched",
                    help="one batched call for all stacks (default), or the stage-wise entry points per stack")
    ap.add_argument("--tune-cache", default=None,
                    help="load tuned launch shapes from this file if it exists, else tune and save them here")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device copy (read 512 MiB + write 512 MiB per launch) "
                         "to calibrate the HBM byte counters")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch from rocprofv3 counters (JSON), if present")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE runs of this benchmark "
                         "and of --copy-probe): write the --traffic JSON and exit")
    ap.add_argument("--traffic-kernels", default=",".join(("batch_score", "batch_cal", "batch_shift", "batch_comb",
                                                           "score_tiles", "calibrate", "shift", "combine")),
                    help="with --traffic-from: the kernels to record (those unchanged since the counter runs)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2008_11486_amd", "weights",
                                                      "proposal_4096.npy"),
                    help="trained proposal network (float32 .npy); untrained weights if missing")
    ap.add_argument("--learned-frames", type=int, default=16)
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the streaming kernels at the wide-field size (16 frames of 6144x6160)")
    ap.add_argument("--no-many", action="store_true",
                    help="skip the batched leg over 64 stacks of 3-30 frames, sides 512-4096")
    ap.add_argument("--sweep", action="store_true",
                    help="only the sweeps over image size and frame count (one JSON line)")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the wide-field streaming kernels (for counter runs) and print their figures")
    ap.add_argument("--traffic-key", default="kernels",
                    help="with --traffic-from: the section of the traffic file to write (kernels, wide)")
    return ap.parse_args()


# Sources each timed kernel is built from: recorded counter values are used only
# while these files are unchanged.
KERNEL_SOURCES = {
    "score_tiles": ("register.hip", "register_core.h", "register_plan.h", "plan.cpp"),
    "batch_score": ("batch.hip", "register_core.h", "register_plan.h", "plan.cpp"),
    "batch_shift": ("batch.hip", "shift_core.h", "common.h"),
    "batch_comb": ("batch.hip", "combine_core.h"),
    "batch_cal": ("batch.hip", "calibrate_core.h", "common.h"),
    "calibrate": ("calibrate.hip", "calibrate_core.h", "common.h"),
    "shift": ("shift.hip", "shift_core.h", "common.h"),
    "combine": ("combine.hip", "combine_core.h"),
    "combine_deep": ("combine.hip", "combine_core.h"),
    "combine_missing": ("combine.hip", "combine_core.h"),
    "mask_shifted": ("shift.hip", "shift_core.h", "common.h"),
    "shift_spline": ("spline.hip", "common.h", "shift_core.h"),
}
KERNEL_SYMBOLS = {"batch_score": "batch_score", "batch_shift": "batch_shift", "batch_comb": "batch_comb",
                  "batch_cal": "batch_cal", "score_tiles": "score_tiles", "calibrate": "calibrate_",
                  "shift": "shift_kernel",
                  # a list: every part must appear in the kernel name
                  "combine": ["combine_cols<", "false>"], "combine_deep": "combine_deep<false>",
                  "combine_missing": ["combine_cols<", "true>"], "mask_shifted": "mask_shifted",
                  "shift_spline": ("spline_rows", "spline_cols")}  # one call = both passes


def source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2008_11486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_rows(folder, counter):
    rows = []
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {folder}")
    return rows


def traffic_from(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, kernels):
    """Per-launch HBM bytes of the timed kernels from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for a plain device copy."""
    copy_bytes = 128 << 22  # --copy-probe moves 512 MiB in and 512 MiB out per launch
    cf = max(v for _, v in _counter_rows(copy_fetch_dir, "FETCH_SIZE")) * 1024
    cw = max(v for _, v in _counter_rows(copy_write_dir, "WRITE_SIZE")) * 1024
    fs, ws = copy_bytes / cf, copy_bytes / cw
    out = {"workload": WORKLOADS[workload], "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
           "copy_probe_bytes": copy_bytes, "kernels": {}}
    fr, wr = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")
    for k, syms in KERNEL_SYMBOLS.items():
        if k not in kernels:
            continue
        syms = syms if isinstance(syms, tuple) else (syms,)  # a call of several kernels: their sum
        fetch = write = 0.0
        dispatches = None
        for sym in syms:
            parts = sym if isinstance(sym, list) else [sym]
            fv = [v for n, v in fr if all(q in n for q in parts)]
            wv = [v for n, v in wr if all(q in n for q in parts)]
            if not fv or not wv:
                break
            fetch += sum(fv) / len(fv) * 1024 * fs
            write += sum(wv) / len(wv) * 1024 * ws
            dispatches = len(fv) if dispatches is None else dispatches
        else:
            out["kernels"][k] = {"fetch_bytes": round(fetch), "write_bytes": round(write),
                                 "bytes": round(fetch + write), "dispatches": dispatches,
                                 "source_sha256": source_hash(k)}
    return out


def recorded_traffic(path, kernel, section=None):
    """Bytes per launch recorded for kernel, or None if absent or the kernel changed since."""
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if section:
        d = d.get(section, {})
    rec = d.get("kernels", {}).get(kernel)
    if rec is None or rec.get("source_sha256") != source_hash(kernel):
        return None
    return rec["bytes"]


class StagePipeline:
    """Stage-wise chain over several stacks through the C ABI."""

    def __init__(self, rd, torch, stacks, integer_mode):
        self.rd, self.torch = rd, torch
        self.integer_mode = integer_mode
        dev = torch.device("cuda:0")
        self.items = []
        for st in stacks:
            sp = st.spec
            raw = torch.from_numpy(st.raw.view(np.int16)).to(dev)
            dark = torch.from_numpy(st.dark).to(dev)
            flat = torch.from_numpy(st.flat).to(dev)
            cal = torch.empty((sp.N, sp.H, sp.W), dtype=torch.float32, device=dev)
            ws = torch.empty(max(rd.register_ws_bytes(sp.W, sp.H, sp.N - 1, sp.radius), 1),
                             dtype=torch.uint8, device=dev)
            self.items.append(dict(spec=sp, raw=raw, dark=dark, flat=flat, cal=cal, ws=ws))
        self.pixels = sum(st.spec.pixels for st in stacks)

    def step(self):
        rd = self.rd
        offs = []
        for it in self.items:
            sp = it["spec"]
            rd.calibrate(it["raw"], it["dark"], it["flat"], out=it["cal"])
            offs.append(rd.register(it["cal"][0], it["cal"][1:], sp.radius, ws=it["ws"]))
        host = [rd.offsets_to_numpy(o) for o in offs]  # one device->host sync per step
        outs = []
        for it, o in zip(self.items, host):
            sp = it["spec"]
            key = ("dx", "dy") if self.integer_mode else ("sx", "sy")
            s = np.zeros((sp.N, 2), np.float32)
            s[1:, 0], s[1:, 1] = o[key[0]], o[key[1]]
            rect = rd.valid_rect(s, sp.W, sp.H)
            al = rd.shift(it["cal"], self.torch.from_numpy(s).to(it["cal"].device, non_blocking=True), rect,
                          integer_mode=self.integer_mode)
            outs.append(rd.combine(al)[0])
        return outs


class BatchedPipeline:
    """All stacks through one reduce_stack_batch call per step (one launch per phase)."""

    def __init__(self, rd, torch, stacks, integer_mode):
        dev = torch.device("cuda:0")
        self.items = []
        for st in stacks:
            self.items.append((torch.from_numpy(st.raw.view(np.int16)).to(dev), torch.from_numpy(st.dark).to(dev),
                               torch.from_numpy(st.flat).to(dev), st.spec.radius))
        self.batch = rd.StackBatch(self.items, integer_mode=integer_mode)
        self.pixels = sum(st.spec.pixels for st in stacks)

    def step(self):
        self.batch.run()


def register_flops_per_launch(spec, frames):
    R = spec.radius
    tw, th = spec.W - 2 * R, spec.H - 2 * R
    return 2.0 * frames * tw * th * (2 * R + 1) ** 2


def streaming_bytes(spec):
    N, W, H, R = spec.N, spec.W, spec.H, spec.radius
    hw = (W - 2 * R) * (H - 2 * R)  # upper bound of the overlap used for the byte count
    return {
        "calibrate": N * W * H * (2 + 4) + 8 * W * H,
        "shift": N * hw * (4 + 4),
        "combine": N * hw * 4 + hw * 4,
    }


def cpu_baseline(stacks, integer_mode, min_seconds=10.0, max_reps=20):
    """The FP64 C oracle on this host's cores, from raw frames, over the whole workload,
    repeated until about min_seconds of CPU work have been timed."""
    import oracle
    t0 = time.perf_counter()
    pix = 0
    reps = 0
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < min_seconds):
        for st in stacks:
            oracle.reduce_stack(st.raw, st.dark, st.flat, st.spec.radius, integer_mode=integer_mode)
            pix += st.spec.pixels
        reps += 1
    dt = time.perf_counter() - t0
    return {"value": pix / dt / 1e6, "unit": "Mpix/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the full workload ({len(stacks)} stacks, {pix / reps / 1e6:.1f} Mpix) {reps} times, "
                      f"FP64 C oracle from raw frames (calibrate, search, shift, combine), {dt:.1f} s"}


def many_stack_inputs(torch, rd, specs, on_frames=None):
    """Device inputs of the many-stack workload: per stack (raw int16 [N][H][W] holding the
    uint16 counts, dark, flat, radius), frames rendered on the GPU at the star density of
    the 1024x1024 bands with sub-pixel shifts within +-16 px, and the true shifts
    [N][2] (frame(x + t) = ref(x)).  on_frames(i, spec, frames) sees each stack's float
    frames before they become raw counts."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(20081148)
    stacks, shifts = [], []
    for i, sp in enumerate(specs):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20081148, 2, 7, i])))
        x = rng.uniform(-24, sp.W + 24, sp.n_stars)
        y = rng.uniform(-24, sp.H + 24, sp.n_stars)
        amp = np.exp(rng.uniform(np.log(2e3), np.log(5e4), sp.n_stars))
        t = np.zeros((sp.N, 2))
        t[1:] = rng.uniform(-16, 16, (sp.N - 1, 2))
        stars = np.zeros((sp.N, sp.n_stars, 4), np.float32)
        for k in range(sp.N):
            stars[k, :, 0], stars[k, :, 1], stars[k, :, 2] = x + t[k, 0], y + t[k, 1], amp
        frames = rd.render_frames(torch.from_numpy(stars).to(dev),
                                  torch.arange(sp.N, dtype=torch.int64, device=dev) + 64 * i, sp.W, sp.H,
                                  sky=1000.0, fwhm=3.0, read_noise=10.0, seed=2)
        if on_frames is not None:
            on_frames(i, sp, frames)
        dark = 100.0 + 3.0 * torch.randn((sp.H, sp.W), generator=g, device=dev)
        flat = 0.95 + 0.1 * torch.rand((sp.H, sp.W), generator=g, device=dev)
        raw = frames.mul_(flat).add_(dark).round_().clamp_(0, 65535).to(torch.int32).to(torch.int16)
        del frames
        stacks.append((raw, dark, flat, sp.radius))
        shifts.append(t)
    return stacks, shifts


def tune_many_stacks(torch, rd, specs, stacks_frames):
    """Search shapes per frame size, timed on up to 32 frames of that size (the batched
    search runs all frames of a size in one launch, so the candidates see a full grid).
    stacks_frames: {W: (reference frame, [frame blocks])} gathered by many_stack_inputs'
    on_frames hook; emptied here."""
    plans = {}
    for W in sorted(stacks_frames):
        ref, blocks = stacks_frames.pop(W)
        fr = torch.cat(blocks)
        p = rd.tune_register(ref.contiguous(), fr, specs[0].radius)
        plans[str(W)] = {k: p[k] for k in ("K", "G", "S", "TY", "BR", "threads", "n_tiles")}
        del fr, ref, blocks
    torch.cuda.empty_cache()
    return plans


def tuning_hook(store, limit=32):
    """on_frames hook that keeps up to `limit` non-reference frames per frame size."""
    def hook(i, sp, frames):
        ref, blocks = store.get(sp.W, (None, []))
        have = sum(int(b.shape[0]) for b in blocks)
        if have < limit:
            store[sp.W] = (frames[0].clone() if ref is None else ref, blocks + [frames[1:1 + limit - have].clone()])
    return hook


def many_stacks(torch, rd, reps=2):
    """64 stacks (frame counts 3-30, square sides 512-4096, sub-pixel shifts within +-16 px,
    search radius 17) through one batched call: the stack shapes of the many-stack
    workload, frames rendered on the GPU (star density of the 1024x1024 stacks)."""
    import synth
    specs = synth.config_specs(2)
    store = {}
    stacks, _ = many_stack_inputs(torch, rd, specs, tuning_hook(store))
    pix = sum(sp.N * sp.W * sp.H for sp in specs)
    plans = tune_many_stacks(torch, rd, specs, store)
    batch = rd.StackBatch(stacks)
    batch.run()
    torch.cuda.synchronize()
    rd.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ms, n = rd.prof_query("batch_score")
    rd.prof_enable(False)
    flops = sum(2.0 * (sp.N - 1) * (sp.W - 2 * sp.radius) * (sp.H - 2 * sp.radius) * (2 * sp.radius + 1) ** 2
                for sp in specs)
    frames_n = [sp.N for sp in specs]
    res = {"workload": f"{len(specs)} stacks, N in {min(frames_n)}-{max(frames_n)} ({sum(frames_n)} frames), "
                       f"sides 512-4096, shifts +-16 px, R=17, one batched call",
           "Mpix/s": round(pix / dt / 1e6, 1), "ms_per_call": round(dt * 1e3, 2), "input_pixels": pix,
           "search_ms": round(ms / n, 2), "search_TFLOP/s": round(flops / (ms / n / 1e3) / 1e12, 2),
           "search_frac_fp64": round(flops / (ms / n / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4),
           "search_plans": plans}
    del batch, stacks
    torch.cuda.empty_cache()
    return res


def sweep(torch, rd, reps=3):
    """Time of the batched path while the image side N grows at n = 300 frames (three
    stacks of 100), and while the frame count n grows at N = 1020 (stacks of at most 100
    frames), as the two sweeps of the paper's Section 3.2.2; frames rendered on the GPU
    at the star density of the 1024x1024 stacks, shifts within +-16 px, search radius 17,
    the search shapes the library picks without tuning."""
    from collections import namedtuple
    Spec = namedtuple("Spec", "N W H n_stars radius")

    def run(side, counts):
        specs = [Spec(c, side, side, max(8, round(200 * side * side / 1024 ** 2)), 17) for c in counts]
        stacks, _ = many_stack_inputs(torch, rd, specs)
        batch = rd.StackBatch(stacks)
        batch.run()
        torch.cuda.synchronize()
        rd.prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ms, n = rd.prof_query("batch_score")
        rd.prof_enable(False)
        pix = sum(c * side * side for c in counts)
        res = {"N": side, "n": sum(counts), "stacks": len(counts), "ms_per_call": round(dt * 1e3, 3),
               "Mpix/s": round(pix / dt / 1e6, 1), "search_share": round(ms / n / 1e3 / dt, 3)}
        del batch, stacks
        torch.cuda.empty_cache()
        return res

    out = {"sizes": [run(side, [100, 100, 100]) for side in (256, 512, 1020, 2048, 4096)], "counts": []}
    for n in (30, 90, 300, 600, 900, 1500):
        per = min(100, n // 3)
        out["counts"].append(run(1020, [per] * (n // per)))
    return out


def learned_comparison(torch, rd, weights_path, M):
    """Full +-64 px search vs network proposal + +-2 px search + fallbacks on one stack of
    4096x4096 frames (a reference and M shifted frames, shifts uniform in +-64 px)."""
    from paper_2008_11486_amd import learned
    W = H = 4096
    trained = os.path.exists(weights_path)
    params = learned.load_params(weights_path) if trained else learned.init_params(0)
    frames, t = learned.render_stack(0, M + 1, W, H, 64.0)
    ref, rest = frames[0], frames[1:].contiguous()
    # both searches run with tuned launch shapes (tuned on four frames; the shape does not depend on N)
    rd.tune_register(ref, rest[:4].contiguous(), 64, 64)
    rd.tune_register(ref, rest, 2, 64)
    ws = torch.empty(rd.register_ws_bytes(W, H, M, 64, 64), dtype=torch.uint8, device=frames.device)
    reg = learned.LearnedRegistrar(params, W, H, M, radius_max=64, refine_radius=2)
    full_s = learned.time_call(lambda: learned.full_search(ref, rest, 64, ws=ws), reps=3)
    full = rd.offsets_to_numpy(learned.full_search(ref, rest, 64, ws=ws))
    res = {}
    learned_s = learned.time_call(lambda: res.setdefault("r", reg.register(ref, rest)), reps=1)
    learned_s = min(learned_s, learned.time_call(lambda: reg.register(ref, rest), reps=3))
    r = res["r"]
    torch.cuda.synchronize()
    rd.prof_enable(True)
    reg.register(ref, rest)
    torch.cuda.synchronize()
    parts = {}
    for name in ("cnn_input", "cnn_forward", "register", "score_tiles"):
        ms, n = rd.prof_query(name)
        parts[name] = {"ms": round(ms, 3), "launches": n}
    rd.prof_enable(False)
    same = np.mean((r.offsets["dx"] == full["dx"]) & (r.offsets["dy"] == full["dy"]))
    err = np.abs(r.centres - np.stack([full["dx"], full["dy"]], 1)).max(axis=1)
    return {"workload": f"a reference and {M} frames of {W}x{H}, shifts uniform in +-64 px, full search R=64 "
                        f"vs network proposal + R=2 search (same template) + full-search fallback",
            "weights": "trained" if trained else "untrained", "full_ms": round(full_s * 1e3, 3),
            "learned_ms": round(learned_s * 1e3, 3), "speedup": round(full_s / learned_s, 3),
            "identical_integer_offsets": float(same), "fallback_rate": float(r.fallback.mean()),
            "centre_error_px_median": float(np.median(err)), "centre_error_px_max": float(err.max()),
            "true_offset_max_abs_px": float(np.abs(t).max()), "learned_breakdown": parts}


def streaming_wide(torch, rd, reps=5, traffic_path=os.path.join(ROOT, "profiles", "traffic.json")):
    """calibrate, shift (bilinear, and the bicubic spline timed alone) and combine over 16
    frames of 6144x6160 (working sets of 1.2-2.4 GB, far beyond the 256 MB last-level
    cache), bad-pixel masking with the missing-value combine, and the combine of a
    97-frame stack (the deepest co-adding set of the paper) of 2040x2040, timed with
    HIP events on their stream."""
    from paper_2008_11486_amd import learned
    N, W, H, bound = 16, 6144, 6160, 64.0
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(20081148)
    # input preparation: rendered sky (5000 stars per frame), then dark, flat, single-pixel
    # cosmic-ray hits on 0.01% of pixels, rounding to uint16
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20081148, 3])))
    S = 5000
    x = rng.uniform(-bound - 8, W + bound + 8, S)
    y = rng.uniform(-bound - 8, H + bound + 8, S)
    amp = np.exp(rng.uniform(np.log(2e3), np.log(5e4), S))
    t = np.zeros((N, 2))
    t[1:] = rng.uniform(-bound, bound, (N - 1, 2))
    stars = np.zeros((N, S, 4), np.float32)
    for k in range(N):
        stars[k, :, 0], stars[k, :, 1], stars[k, :, 2] = x + t[k, 0], y + t[k, 1], amp
    cal = torch.empty((N, H, W), dtype=torch.float32, device=dev)
    rd.render_frames(torch.from_numpy(stars).to(dev), torch.arange(N, dtype=torch.int64, device=dev), W, H,
                     sky=1000.0, fwhm=3.0, read_noise=10.0, seed=3, out=cal)
    dark = 100.0 + 3.0 * torch.randn((H, W), generator=g, device=dev)
    flat = 0.95 + 0.1 * torch.rand((H, W), generator=g, device=dev)
    hits = torch.rand((N, H, W), generator=g, device=dev) < 1e-4
    cal.mul_(flat).add_(dark).add_(hits * (5e3 + 5.5e4 * torch.rand((N, H, W), generator=g, device=dev)))
    raw = cal.round_().clamp_(0, 65535).to(torch.int32).to(torch.int16)  # two's-complement bits of uint16
    del hits
    s = torch.from_numpy(t.astype(np.float32)).to(dev)
    rect = rd.valid_rect(t.astype(np.float32), W, H)
    w, h = int(rect[2]), int(rect[3])
    al = torch.empty((N, h, w), dtype=torch.float32, device=dev)
    al_spline = torch.empty((N, h, w), dtype=torch.float32, device=dev)
    spline_ws = torch.empty(rd.lib().reduce_shift_spline_ws(W, H, N), dtype=torch.uint8, device=dev)
    out = torch.empty((h, w), dtype=torch.float32, device=dev)
    # deep stack: aligned values N(1000, 30) with outliers on 0.01% of them
    ND, SD = 97, 2040
    deep = 1000.0 + 30.0 * torch.randn((ND, SD, SD), generator=g, device=dev)
    dh = torch.rand((ND, SD, SD), generator=g, device=dev) < 1e-4
    deep.add_(dh * (5e3 + 5.5e4 * torch.rand((ND, SD, SD), generator=g, device=dev)))
    del dh
    deep_out = torch.empty((SD, SD), dtype=torch.float32, device=dev)
    # bad-pixel map: 0.1% of the detector's pixels
    bad = (torch.rand((H, W), generator=g, device=dev) < 1e-3).to(torch.uint8)
    out_miss = torch.empty((h, w), dtype=torch.float32, device=dev)

    def chain():
        rd.calibrate(raw, dark, flat, out=cal)
        rd.shift(cal, s, rect, out=al)
        rd.combine(al, out=out)
        rd.mask_shifted(bad, al, s, rect, W, H)  # bad-pixel masking, then the missing-value combine
        rd.combine(al, out=out_miss, missing=True)
        rd.shift_spline(cal, s, rect, out=al_spline, ws=spline_ws)  # the paper's interpolation, timed alone
        rd.combine(deep, out=deep_out)

    for _ in range(2):
        chain()
    torch.cuda.synchronize()
    rd.prof_enable(True)
    for _ in range(reps):
        chain()
    torch.cuda.synchronize()
    res = {"workload": f"{N} frames {W}x{H}, 5000 stars, cosmic-ray hits on 0.01% of pixels, shifts +-64 px, "
                       f"overlap {w}x{h}, bad pixels 0.1%; deep combine: {ND} frames {SD}x{SD}"}
    byts = {"calibrate": N * W * H * (2 + 4) + 8 * W * H, "shift": N * w * h * (4 + 4), "combine": N * w * h * 4 + w * h * 4,
            # rows: frame read, row-pass result written; columns: that result read, output written
            "shift_spline": N * 4 * (H * W + 2 * H * w + h * w), "combine_deep": (ND + 1) * SD * SD * 4,
            # the map (from L2 after the first frame) and the marked values
            "mask_shifted": H * W + int(torch.isnan(al).sum()) * 4, "combine_missing": N * w * h * 4 + w * h * 4}
    for name in ("calibrate", "shift", "combine", "shift_spline", "combine_deep", "mask_shifted", "combine_missing"):
        ms, n = rd.prof_query(name)
        gbs = byts[name] / (ms / n / 1e3) / 1e9
        res[name] = {"avg_launch_ms": round(ms / n, 4), "bytes": byts[name], "GB/s": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(traffic_path, name, "wide")}
    rd.prof_enable(False)
    del raw, cal, al, al_spline, spline_ws, deep, deep_out, bad, out_miss
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.traffic_from:
        rec = traffic_from(*args.traffic_from, workload=args.workload, kernels=args.traffic_kernels.split(","))
        old = json.load(open(args.traffic)) if os.path.exists(args.traffic) else {}
        if args.traffic_key == "kernels":
            kernels = dict(old.get("kernels", {}))
            kernels.update(rec["kernels"])
            old.update(rec)
            old["kernels"] = kernels
        else:
            old[args.traffic_key] = {"workload": "16 frames 6144x6160 (wide field)", "kernels": rec["kernels"],
                                     "fetch_scale": rec["fetch_scale"], "write_scale": rec["write_scale"]}
        with open(args.traffic, "w") as fh:
            json.dump(old, fh, indent=1)
        print(json.dumps(old))
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; sharding stacks over several GPUs is a design "
              "note, not a measured path. Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    import paper_2008_11486_amd as rd
    import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    if args.copy_probe:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": dst.numel() * 4,
                          "ms": round(ms, 4), "GB/s": round(2 * src.numel() * 4 / (ms / 1e3) / 1e9, 1)}))
        return 0
    if args.wide_only:
        rd.lib()
        print(json.dumps({"streaming_wide": streaming_wide(torch, rd)}))
        return 0
    if args.sweep:
        rd.lib()
        print(json.dumps({"sweep": sweep(torch, rd)}))
        return 0
    rd.lib()
    stacks = synth.make_config(args.workload)
    integer_mode = args.workload == 0
    pipe = (BatchedPipeline if args.path == "batched" else StagePipeline)(rd, torch, stacks, integer_mode)
    tuned = None
    if args.tune_cache and os.path.exists(args.tune_cache):
        rd.tune_load(args.tune_cache)
        tuned = "loaded"
    elif not args.no_tune:
        # timed on the frames one search launch covers: every stack's in the batched path
        # (one launch for all stacks), one stack's in the stage-wise path
        cals = [rd.calibrate(torch.from_numpy(st.raw.view(np.int16)).to("cuda:0"),
                             torch.from_numpy(st.dark).to("cuda:0"), torch.from_numpy(st.flat).to("cuda:0"))
                for st in (stacks if args.path == "batched" else stacks[:1])]
        tuned = rd.tune_register(cals[0][0].contiguous(), torch.cat([c[1:] for c in cals]),
                                 stacks[0].spec.radius)
        del cals
        if args.tune_cache:
            rd.tune_save(args.tune_cache)

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()

    rd.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    kern = {name: rd.prof_query(name) for name in ("score_tiles", "calibrate", "shift", "combine", "batch_score",
                                                   "batch_out")}
    if args.path == "batched":
        kern["score_tiles"] = kern["batch_score"]
    rd.prof_enable(False)

    spec0 = stacks[0].spec
    score_ms, score_n = kern["score_tiles"]
    score_avg_s = score_ms / score_n / 1e3
    # one stage-wise launch searches one stack; one batched launch searches all of them
    flops = sum(register_flops_per_launch(st.spec, st.spec.N - 1)
                for st in (stacks if args.path == "batched" else stacks[:1]))
    achieved = flops / score_avg_s / 1e12
    traffic = recorded_traffic(args.traffic, "batch_score" if args.path == "batched" else "score_tiles")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(FP64_VALU_PEAK_TFLOPS, 3),
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "batch_score" if args.path == "batched" else "score_tiles",
                "avg_launch_ms": round(score_avg_s * 1e3, 4),
                "flops_per_launch": flops}

    sbytes = streaming_bytes(spec0)
    streaming = {}
    for name in ("calibrate", "shift", "combine"):
        ms, n = kern[name]
        if n and args.path == "stagewise":
            gbs = sbytes[name] / (ms / n / 1e3) / 1e9
            streaming[name] = {"avg_launch_ms": round(ms / n, 4), "GB/s": round(gbs, 1),
                               "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": sbytes[name],
                               "traffic": recorded_traffic(args.traffic, name)}

    value = pipe.pixels / (ms_per_step / 1e3) / 1e6
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "stacks": len(stacks),
                   "frames": [s.spec.N for s in stacks], "size": [spec0.W, spec0.H],
                   "path": args.path, "pixel_storage": "uint16 in, f32 between stages",
                   "search_plan": rd.register_plan(spec0.W, spec0.H, spec0.N - 1, spec0.radius)},
        "roofline": roofline, "streaming": streaming,
    }
    if not args.no_wide:
        line["streaming_wide"] = streaming_wide(torch, rd)
    if not args.no_many:
        line["many_stacks"] = many_stacks(torch, rd)
    if not args.no_learned:
        line["learned"] = learned_comparison(torch, rd, args.weights, args.learned_frames)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(stacks, integer_mode)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
