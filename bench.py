#!/usr/bin/env python
"""Throughput of the CCD reduction hot path on one MI355X.

One step = one pass of the whole path (dark subtraction + flat division, registration
against frame 0 of each stack, bilinear shift onto the common overlap, sigma-clipped
mean) over one batch of synthetic frames already resident in HBM.  The default
workload is the largest one that runs as one call on one GPU: 64 independent stacks of
3-30 frames with square sides from 512 to 4096 (6.56 Gpix of uint16 frames), sub-pixel
shifts within +-16 px (search radius 17), all stacks in one batched call.

Prints one JSON line: stacked Mpix/s (input pixels of all frames per second), the
roofline position of the dominant kernel (timed with HIP events on its own stream over
the timed steps), the FP64 CPU oracle timed on this host on a stated sample of the same
workload (and the parity of the GPU's results on that sample), and extra legs: the three
1024x1024 bands, the wide-field chain of 16 frames of 6144x6160 with the +-65 px search,
the streaming kernels at that size, and the learned proposal against the full search.
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
    2: "64 stacks, N uniform in 3-30, square sides from {512, 1024, 2048, 4096} (6.56 Gpix of uint16 frames), "
       "200 stars per 1024x1024, sub-pixel shifts +-16 px, search radius 17, bilinear shift, 3-sigma clipped "
       "mean (3 iterations), all stacks in one batched call",
    1: "3 bands x 10 frames 1024x1024 uint16, 200 stars, sub-pixel shifts +-20 px, search radius 21, "
       "bilinear shift, 3-sigma clipped mean (3 iterations)",
    0: "5 frames 512x512 uint16, 20 stars, integer shifts +-8 px, search radius 8, integer shift, "
       "3-sigma clipped mean (3 iterations)",
}
REDUCE_NEAR_TIE = 4


def log(msg):
    """A progress line on stderr as each leg of the run ends (the JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, choices=sorted(WORKLOADS))
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
    ap.add_argument("--no-bands", action="store_true",
                    help="skip the leg over three bands of 10 frames of 1024x1024 (with --workload 2)")
    ap.add_argument("--no-wide-chain", action="store_true",
                    help="skip the end-to-end wide-field chain with the +-65 px search")
    ap.add_argument("--no-autotuned-search", action="store_true",
                    help="skip the 64-stack leg with the search of each frame size chosen by timing")
    ap.add_argument("--sweep", action="store_true",
                    help="only the sweeps over image size and frame count (one JSON line)")
    ap.add_argument("--no-alone", action="store_true",
                    help="skip the back-to-back timing of each streaming kernel alone (for counter runs)")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the wide-field streaming kernels (for counter runs) and print their figures")
    ap.add_argument("--traffic-key", default=None,
                    help="with --traffic-from: the section of the traffic file to write (many, kernels, wide); "
                         "default: many for workload 2, kernels otherwise")
    return ap.parse_args()


# Sources each timed kernel is built from: recorded counter values are used only
# while these files are unchanged.
KERNEL_SOURCES = {
    "score_tiles": ("register.hip", "register_core.h", "register_plan.h", "plan.cpp", "common.h"),
    "batch_score": ("batch.hip", "register_core.h", "register_plan.h", "plan.cpp", "common.h"),
    "batch_shift": ("batch.hip", "shift_core.h", "common.h"),
    "batch_comb": ("batch.hip", "combine_core.h", "common.h"),
    "batch_cal": ("batch.hip", "calibrate_core.h", "common.h"),
    "batch_fused": ("batch.hip", "shift_core.h", "combine_core.h", "common.h"),
    "calibrate": ("calibrate.hip", "calibrate_core.h", "common.h"),
    "shift": ("shift.hip", "shift_core.h", "common.h"),
    "combine": ("combine.hip", "combine_core.h"),
    "combine_deep": ("combine.hip", "combine_core.h"),
    "combine_missing": ("combine.hip", "combine_core.h"),
    "mask_shifted": ("shift.hip", "shift_core.h", "common.h"),
    "shift_spline": ("spline.hip", "common.h", "shift_core.h"),
}
KERNEL_SYMBOLS = {"batch_score": "batch_score", "batch_shift": "batch_shift", "batch_comb": "batch_comb",
                  "batch_cal": "batch_cal", "batch_fused": "batch_fused", "score_tiles": "score_tiles",
                  "calibrate": "calibrate_",
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
    """(kernel name, value) of every dispatch's counter in a rocprofv3 --pmc output folder:
    CSV output (*counter_collection.csv) or the SQLite database rocprofv3 writes by default
    (*_results.db, its counters_collection view)."""
    import sqlite3
    rows = []
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    for f in glob.glob(os.path.join(folder, "**", "*_results.db"), recursive=True):
        db = sqlite3.connect(f"file:{f}?mode=ro", uri=True)
        try:
            rows += [(n, float(v)) for n, v in db.execute(
                "select kernel_name, value from counters_collection where counter_name = ? order by dispatch_id",
                (counter,))]
        finally:
            db.close()
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


def tune_many_stacks(torch, rd, specs, stacks_frames, searches=None):
    """Search shapes per frame size, timed on up to 32 frames of that size (the batched
    search runs all frames of a size in one launch, so the candidates see a full grid);
    with a dict `searches`, also the faster search (direct sums or row spectra) per frame
    size on the same frames.  stacks_frames: {W: (reference frame, [frame blocks])}
    gathered by many_stack_inputs' on_frames hook; emptied here."""
    plans = {}
    for W in sorted(stacks_frames):
        ref, blocks = stacks_frames.pop(W)
        fr = torch.cat(blocks)
        p = rd.tune_register(ref.contiguous(), fr, specs[0].radius)
        plans[str(W)] = {k: p[k] for k in ("K", "G", "S", "TY", "BR", "threads", "n_tiles")}
        if searches is not None:
            searches[W] = rd.tune_search(ref.contiguous(), fr, specs[0].radius)
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


def search_flops(specs):
    """Algorithmic flops of the full-window search of every non-reference frame: one FMA
    (2 flop) per template pixel (the interior shrunk by the radius) per candidate offset."""
    return sum(2.0 * (sp.N - 1) * (sp.W - 2 * sp.radius) * (sp.H - 2 * sp.radius) * (2 * sp.radius + 1) ** 2
               for sp in specs)


class ManyStackPipeline:
    """The 64-stack workload (frame counts 3-30, square sides 512-4096, sub-pixel shifts
    within +-16 px, search radius 17): frames rendered on the GPU at the star density of the
    1024x1024 stacks, search shapes tuned per frame size, all stacks in one batched call
    per step."""

    def __init__(self, rd, torch, tune=True, tune_cache=None):
        import synth
        self.specs = synth.config_specs(2)
        store = {}
        cached = tune_cache is not None and os.path.exists(tune_cache)
        if cached:
            rd.tune_load(tune_cache)
        tune = tune and not cached
        self.stacks, self.shifts = many_stack_inputs(torch, rd, self.specs, tuning_hook(store) if tune else None)
        log("64-stack inputs rendered")
        self.searches = {}
        self.plans = (tune_many_stacks(torch, rd, self.specs, store, self.searches) if tune
                      else ("loaded" if cached else None))
        if tune and tune_cache:
            rd.tune_save(tune_cache)
        self.batch = rd.StackBatch(self.stacks)
        self.pixels = sum(sp.N * sp.W * sp.H for sp in self.specs)

    def step(self):
        self.batch.run()


def autotuned_search_leg(torch, rd, pipe, steps=10, warmup=2):
    """The 64-stack workload with the search of each frame size chosen by timing (direct
    sums or row spectra, on the tuning frames of that size): same stacks, one batched call
    per step, and the per-size choices and times."""
    if not pipe.searches:
        return None
    choice = [pipe.searches[sp.W]["search"] for sp in pipe.specs]
    batch = rd.StackBatch(pipe.stacks, search=choice)
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    rd.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    parts = {k: round(rd.prof_query(k)[0] / steps, 3)
             for k in ("batch_cal", "batch_score", "batch_spectral", "spec_corr", "fft_rows", "spec_eval",
                       "fft_refine", "batch_fused")}
    rd.prof_enable(False)
    res = {"workload": WORKLOADS[2] + "; the search of each frame size chosen by timing",
           "Mpix/s": round(pipe.pixels / dt / 1e6, 1), "ms_per_step": round(dt * 1e3, 3), "steps": steps,
           "search_by_size": {str(W): {"search": v["search"], "ms_direct": round(v["ms_direct"], 3),
                                       "ms_spectral": round(v["ms_spectral"], 3)}
                              for W, v in sorted(pipe.searches.items())},
           "ms_per_step_by_phase": parts}
    del batch
    torch.cuda.empty_cache()
    return res


def many_sample(pipe, min_frames=5):
    """Host copies for the CPU leg: per frame size, the stack with the fewest frames (at
    least min_frames), its raw counts, dark, flat and the GPU's results; the GPU's offsets
    of every stack (for the near-tie count)."""
    specs = pipe.specs
    picks = []
    for W in sorted({sp.W for sp in specs}):
        cand = [i for i, sp in enumerate(specs) if sp.W == W and sp.N >= min_frames]
        picks.append(min(cand, key=lambda i: (specs[i].N, i)))
    sample = []
    for i in picks:
        raw, dark, flat, R = pipe.stacks[i]
        img, rect, offs, nrej = pipe.batch.result(i)
        sample.append(dict(index=i, spec=specs[i], raw=raw.cpu().numpy().view(np.uint16), dark=dark.cpu().numpy(),
                           flat=flat.cpu().numpy(), img=img.cpu().numpy(), rect=np.asarray(rect), offs=offs,
                           n_rej=nrej))
    all_offs = [pipe.batch.result(i)[2] for i in range(len(specs))]
    return sample, all_offs


def err_stats(e):
    e = np.asarray(e, np.float64).ravel()
    if e.size == 0:
        return {"max": None, "p99.9": None, "p95": None, "p90": None}
    return {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)), "p95": float(np.quantile(e, 0.95)),
            "p90": float(np.quantile(e, 0.90))}


def _oracle_chain_timed(oracle, raw, dark, flat, R):
    """The oracle's chain from raw, stage by stage, with the time of each stage."""
    t = {}
    t0 = time.perf_counter()
    cal = oracle.calibrate(raw, dark, flat)
    t["calibrate"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    offs = oracle.register(cal[0], cal, R)
    t["register"] = time.perf_counter() - t0
    s = np.stack([offs["sx"], offs["sy"]], axis=1).astype(np.float32)
    s[0] = 0.0
    rect = oracle.valid_rect(s, raw.shape[2], raw.shape[1])
    t0 = time.perf_counter()
    al = oracle.shift(cal, s, rect)
    t["shift"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    out, keep, nrej, near = oracle.combine(al)
    t["combine"] = time.perf_counter() - t0
    return dict(cal=cal, offsets=offs, s=s, rect=rect, out=out, near=near, n_rej=nrej), t


def cpu_baseline_many(sample, all_offs, specs, one_thread_sides=(512, 1024)):
    """The FP64 C oracle on this host's cores, from raw frames, on the sampled stacks (one
    per frame size), stage by stage; the whole workload's time extrapolated from it (the
    search by its FMA count per frame size, calibrate + shift + combine by pixel count),
    at all threads and at one thread (one thread: the stacks of the sides named, larger
    sides at the per-FMA rate of the largest of them).  The same oracle outputs give the
    parity of the GPU's results on the sample: offsets from raw (integer offsets must be
    identical), and the combined images against the oracle's shift and clip at the GPU's
    offsets (pixels inside the clip's threshold band are counted, not value-checked)."""
    import oracle
    all_threads = oracle.num_threads()

    def fma(sp):
        return (sp.N - 1) * (sp.W - 2 * sp.radius) * (sp.H - 2 * sp.radius) * (2 * sp.radius + 1) ** 2

    def extrapolate(times):
        """times: {side: (t_register, t_stream, sample fma, sample pixels)} -> workload seconds."""
        stream_rate = sum(v[1] for v in times.values()) / sum(v[3] for v in times.values())
        top = max(times)
        total = 0.0
        for sp in specs:
            key = sp.W if sp.W in times else top
            total += fma(sp) * times[key][0] / times[key][2] + sp.N * sp.W * sp.H * stream_rate
        return total

    pix_all = sum(sp.N * sp.W * sp.H for sp in specs)
    t_all, parity_rows = {}, []
    wall0 = time.perf_counter()
    for smp in sample:
        sp = smp["spec"]
        o, t = _oracle_chain_timed(oracle, smp["raw"], smp["dark"], smp["flat"], sp.radius)
        t_all[sp.W] = (t["register"], t["calibrate"] + t["shift"] + t["combine"], fma(sp), sp.N * sp.W * sp.H)
        parity_rows.append(_parity_row(oracle, smp, o))
        del o
    wall_all = time.perf_counter() - wall0
    t_one = {}
    oracle.set_num_threads(1)
    wall0 = time.perf_counter()
    try:
        for smp in sample:
            sp = smp["spec"]
            if sp.W in one_thread_sides:
                _, t = _oracle_chain_timed(oracle, smp["raw"], smp["dark"], smp["flat"], sp.radius)
                t_one[sp.W] = (t["register"], t["calibrate"] + t["shift"] + t["combine"], fma(sp),
                               sp.N * sp.W * sp.H)
    finally:
        oracle.set_num_threads(all_threads)
    wall_one = time.perf_counter() - wall0
    T_all, T_one = extrapolate(t_all), extrapolate(t_one)
    desc = ", ".join(f"{smp['spec'].N} x {smp['spec'].W}x{smp['spec'].H} (stack {smp['index']})" for smp in sample)
    baseline = {"value": round(pix_all / T_all / 1e6, 3), "unit": "Mpix/s", "cores": all_threads, "kind": "oracle",
                "sample": f"FP64 C oracle from raw frames (calibrate, full-window search, shift, combine) on one "
                          f"stack per frame size: {desc}; {wall_all:.1f} s at {all_threads} threads; the workload's "
                          f"{pix_all / 1e6:.0f} Mpix extrapolated per frame size (search by FMA count, the other "
                          f"stages by pixel count): {T_all:.0f} s",
                "value_1_thread": round(pix_all / T_one / 1e6, 4),
                "sample_1_thread": f"the {', '.join(str(w) for w in sorted(t_one))} stacks of the sample at 1 "
                                   f"thread ({wall_one:.1f} s); larger sides at the per-FMA search rate of the "
                                   f"{max(t_one)} stack: {T_one:.0f} s for the workload"}
    return baseline, _parity_summary(parity_rows, all_offs, specs)


def _parity_row(oracle, smp, o):
    """One sampled stack: GPU results against the oracle's chain from raw."""
    sp, offs = smp["spec"], smp["offs"]
    s_gpu = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
    same_int = (offs["dx"][1:] == o["offsets"]["dx"][1:]) & (offs["dy"][1:] == o["offsets"]["dy"][1:])
    ds = np.abs(s_gpu.astype(np.float64) - o["s"].astype(np.float64))[1:]
    rect_same = bool(np.array_equal(smp["rect"], o["rect"]))
    if np.array_equal(s_gpu[1:], o["s"][1:]) and rect_same:
        ref, near = o["out"], o["near"].any(axis=0)
    else:  # the oracle's shift and clip of its own calibration at the GPU's offsets
        al = oracle.shift(o["cal"], s_gpu, smp["rect"])
        ref, _, _, nb = oracle.combine(al)
        near = nb.any(axis=0)
        del al
    g = smp["img"].astype(np.float64)
    ok = ~near
    e = np.abs(g[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), 1.0)
    return dict(index=smp["index"], N=sp.N, W=sp.W, frames=int(sp.N - 1), same_int=int(same_int.sum()),
                s_diff_frames=int(np.any(ds > 0, axis=1).sum()), s_diff_max=float(ds.max()) if ds.size else 0.0,
                rect_same=rect_same, pixels=int(g.size), band=int(near.sum()), err=e, n_rej=smp["n_rej"])


def _parity_summary(rows, all_offs, specs, tol=2e-6):
    e = np.concatenate([r["err"] for r in rows])
    frames = sum(r["frames"] for r in rows)
    near_ties = sum(int(np.sum((o["flags"][1:] & REDUCE_NEAR_TIE) != 0)) for o in all_offs)
    st = err_stats(e)
    ok = all(r["same_int"] == r["frames"] and r["rect_same"] for r in rows) and (st["max"] or 0.0) <= tol
    return {"stacks": [r["index"] for r in rows], "frames_searched": frames,
            "identical_integer_offsets": round(sum(r["same_int"] for r in rows) / max(frames, 1), 6),
            "frames_with_subpixel_offset_difference": sum(r["s_diff_frames"] for r in rows),
            "max_subpixel_offset_difference_px": max(r["s_diff_max"] for r in rows),
            "rects_identical": all(r["rect_same"] for r in rows),
            "pixels_checked": int(e.size), "threshold_band_pixels": sum(r["band"] for r in rows),
            "rel_err": st, "tolerance": tol,
            "near_tie_frames_all_stacks": near_ties,
            "frames_all_stacks": sum(sp.N - 1 for sp in specs), "within_tolerance": bool(ok)}


def bands_leg(torch, rd, steps=20, warmup=3):
    """The three 1024x1024 bands of 10 frames (search radius 21) through one batched call."""
    import synth
    stacks = synth.make_config(1)
    pipe = BatchedPipeline(rd, torch, stacks, False)
    cals = [rd.calibrate(torch.from_numpy(st.raw.view(np.int16)).to("cuda:0"),
                         torch.from_numpy(st.dark).to("cuda:0"), torch.from_numpy(st.flat).to("cuda:0"))
            for st in stacks]
    rd.tune_register(cals[0][0].contiguous(), torch.cat([c[1:] for c in cals]), stacks[0].spec.radius)
    del cals
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    rd.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms, n = rd.prof_query("batch_score")
    rd.prof_enable(False)
    flops = search_flops([st.spec for st in stacks]) / (n / steps)
    res = {"workload": WORKLOADS[1], "Mpix/s": round(pipe.pixels / dt / 1e6, 1), "ms_per_step": round(dt * 1e3, 4),
           "search_avg_launch_ms": round(ms / n, 4),
           "search_frac_fp64": round(flops / (ms / n / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4)}
    del pipe
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
    """Full +-64 px search (direct sums, and through row spectra) vs network proposal +
    +-2 px search + fallbacks on one stack of 4096x4096 frames (a reference and M shifted
    frames, shifts uniform in +-64 px)."""
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
    # the full window through row spectra (same offsets)
    wsf = torch.empty(rd.register_fft_ws_bytes(W, H, M, 64), dtype=torch.uint8, device=frames.device)
    spec_s = learned.time_call(lambda: rd.register_fft(ref, rest, 64, ws=wsf), reps=3)
    spec = rd.offsets_to_numpy(rd.register_fft(ref, rest, 64, ws=wsf))
    del wsf
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
            "full_spectral_ms": round(spec_s * 1e3, 3), "speedup_vs_full_spectral": round(spec_s / learned_s, 3),
            "spectral_identical_integer_offsets": bool(np.array_equal(spec["dx"], full["dx"]) and
                                                       np.array_equal(spec["dy"], full["dy"])),
            "spectral_max_subpixel_difference_px": float(max(np.abs(spec["sx"] - full["sx"]).max(),
                                                             np.abs(spec["sy"] - full["sy"]).max())),
            "identical_integer_offsets": float(same), "fallback_rate": float(r.fallback.mean()),
            "centre_error_px_median": float(np.median(err)), "centre_error_px_max": float(err.max()),
            "true_offset_max_abs_px": float(np.abs(t).max()), "learned_breakdown": parts}


def wide_inputs(torch, rd):
    """The wide-field stack: 16 frames of 6144x6160 rendered on the GPU (5000 stars, sky
    1000 ADU, read noise 10 ADU), shifts uniform in +-64 px, dark 100 +- 3 ADU, flat
    1 +- 0.05, cosmic-ray tracks of 1-4 px on 0.01% of the pixels of every frame (5e3-6e4
    ADU per hit pixel), rounded to uint16."""
    import synth
    N, W, H, bound = 16, 6144, 6160, 64.0
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(20081148)
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
    cal.mul_(flat).add_(dark)
    hit_pixels = 0
    for k in range(N):
        ys, xs, adu = synth.cosmic_ray_hits(W, H, np.random.Generator(np.random.PCG64(
            np.random.SeedSequence([20081148, 3, 1, k]))))
        idx = (torch.full((len(ys),), k, dtype=torch.int64, device=dev), torch.from_numpy(ys).to(dev),
               torch.from_numpy(xs).to(dev))
        cal.index_put_(idx, torch.from_numpy(adu.astype(np.float32)).to(dev), accumulate=True)
        hit_pixels += len(ys)
    raw = cal.round_().clamp_(0, 65535).to(torch.int32).to(torch.int16)  # two's-complement bits of uint16
    del cal
    return dict(N=N, W=W, H=H, raw=raw, dark=dark, flat=flat, t=t, g=g, hit_fraction=hit_pixels / (N * W * H))


def wide_chain(torch, rd, inp, reps=3):
    """The wide-field stack end to end from raw through one batched call: calibrate, the
    full +-65 px search of all 15 frames against frame 0 (template shrunk by 65), shift and
    the clipped mean; search shapes tuned on two frames."""
    N, W, H, R = inp["N"], inp["W"], inp["H"], 65
    cal = rd.calibrate(inp["raw"][:3], inp["dark"], inp["flat"])
    plan = rd.tune_register(cal[0].contiguous(), cal[1:3].contiguous(), R)
    del cal
    torch.cuda.empty_cache()
    batch = rd.StackBatch([(inp["raw"], inp["dark"], inp["flat"], R)])
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
    _, rect, offs, nrej = batch.result(0)
    del batch
    torch.cuda.empty_cache()
    # the same chain with the search through row spectra
    sbatch = rd.StackBatch([(inp["raw"], inp["dark"], inp["flat"], R)], search="spectral")
    sbatch.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sbatch.run()
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / reps
    _, rect_s, offs_s, _ = sbatch.result(0)
    same = bool(np.array_equal(rect, rect_s) and np.array_equal(offs["dx"], offs_s["dx"]) and
                np.array_equal(offs["dy"], offs_s["dy"]) and np.array_equal(offs["flags"], offs_s["flags"]))
    ds = float(max(np.abs(offs["sx"] - offs_s["sx"]).max(), np.abs(offs["sy"] - offs_s["sy"]).max()))
    s = np.stack([offs["sx"], offs["sy"]], 1)
    flops = 2.0 * (N - 1) * (W - 2 * R) * (H - 2 * R) * (2 * R + 1) ** 2
    res = {"workload": f"{N} frames {W}x{H}, 5000 stars, cosmic-ray tracks of 1-4 px on "
                       f"{100 * inp['hit_fraction']:.4f}% of pixels, shifts +-64 px, search radius 65, one batched call",
           "Mpix/s": round(N * W * H / dt / 1e6, 1), "ms_per_call": round(dt * 1e3, 2),
           "search_ms": round(ms / reps, 2), "search_share": round(ms / reps / 1e3 / dt, 4),
           "search_frac_fp64": round(flops / (ms / reps / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4),
           "rect": [int(v) for v in rect], "rejected_values": int(nrej),
           "max_offset_error_vs_truth_px": round(float(np.abs(s[1:] - inp["t"][1:]).max()), 4),
           "spectral_search": {"Mpix/s": round(N * W * H / dt_s / 1e6, 1), "ms_per_call": round(dt_s * 1e3, 2),
                               "same_integer_offsets_flags_and_overlap": same,
                               "max_subpixel_offset_difference_px": ds},
           "search_plan": {k: plan[k] for k in ("K", "G", "S", "TY", "BR", "threads", "n_tiles")}}
    del sbatch
    torch.cuda.empty_cache()
    return res


def streaming_wide(torch, rd, inp, reps=10, traffic_path=os.path.join(ROOT, "profiles", "traffic.json"), alone=True):
    """calibrate, shift (bilinear, and the bicubic spline timed alone) and combine over the
    wide-field stack at its true shifts (working sets of 1.2-2.4 GB, far beyond the 256 MB
    last-level cache), bad-pixel masking with the missing-value combine, and the combine of
    a 97-frame stack (the deepest co-adding set of the paper) of 2040x2040, timed with HIP
    events on their stream."""
    N, W, H = inp["N"], inp["W"], inp["H"]
    raw, dark, flat, t, g = inp["raw"], inp["dark"], inp["flat"], inp["t"], inp["g"]
    dev = raw.device
    cal = torch.empty((N, H, W), dtype=torch.float32, device=dev)
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

    # the device reaches its steady clocks only after tens of milliseconds of back-to-back
    # work (a 0.5 ms kernel runs 20-40% longer in its first launches after an idle
    # second), so the chain runs for half a second before the timed repetitions
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < 0.5:
        for _ in range(8):
            chain()
        torch.cuda.synchronize()
    rd.prof_enable(True)
    for _ in range(reps):
        chain()
    torch.cuda.synchronize()
    res = {"workload": f"{N} frames {W}x{H} at their true shifts (+-64 px), overlap {w}x{h}, bad pixels 0.1%; "
                       f"deep combine: {ND} frames {SD}x{SD}; timed after 0.5 s of warm-up"}
    byts = {"calibrate": N * W * H * (2 + 4) + 8 * W * H, "shift": N * w * h * (4 + 4), "combine": N * w * h * 4 + w * h * 4,
            # rows: frame read, row-pass result written; columns: that result read, output written
            "shift_spline": N * 4 * (H * W + 2 * H * w + h * w), "combine_deep": (ND + 1) * SD * SD * 4,
            # the map (from L2 after the first frame) and the marked values
            "mask_shifted": H * W + int(torch.isnan(al).sum()) * 4, "combine_missing": N * w * h * 4 + w * h * 4}
    names = ("calibrate", "shift", "combine", "shift_spline", "combine_deep", "mask_shifted", "combine_missing")
    for name in names:
        ms, n = rd.prof_query(name)
        gbs = byts[name] / (ms / n / 1e3) / 1e9
        res[name] = {"avg_launch_ms": round(ms / n, 4), "bytes": byts[name], "GB/s": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(traffic_path, name, "wide")}
    rd.prof_enable(False)
    # each kernel alone, launched back to back for 0.2 s and then timed over 20 launches:
    # the rate it keeps when the stage runs over many stacks in a row (the device settles
    # at other clocks under one memory-bound kernel than under the mixed chain)
    single = {"calibrate": lambda: rd.calibrate(raw, dark, flat, out=cal),
             "shift": lambda: rd.shift(cal, s, rect, out=al),
             "combine": lambda: rd.combine(al, out=out),
             "mask_shifted": lambda: rd.mask_shifted(bad, al, s, rect, W, H),
             "combine_missing": lambda: rd.combine(al, out=out_miss, missing=True),
             "shift_spline": lambda: rd.shift_spline(cal, s, rect, out=al_spline, ws=spline_ws),
             "combine_deep": lambda: rd.combine(deep, out=deep_out)}
    for name in ("calibrate", "shift", "combine", "mask_shifted", "combine_missing", "shift_spline", "combine_deep"):
        if not alone:
            break
        fn = single[name]
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.2:
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
        rd.prof_enable(True)
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        ms, n = rd.prof_query(name)
        rd.prof_enable(False)
        res[name]["alone_ms"] = round(ms / n, 4)
        res[name]["alone_frac"] = round(byts[name] / (ms / n / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    del cal, al, al_spline, spline_ws, deep, deep_out, bad, out_miss
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.traffic_from:
        rec = traffic_from(*args.traffic_from, workload=args.workload, kernels=args.traffic_kernels.split(","))
        old = json.load(open(args.traffic)) if os.path.exists(args.traffic) else {}
        key = args.traffic_key or ("many" if args.workload == 2 else "kernels")
        if key == "kernels":
            kernels = dict(old.get("kernels", {}))
            kernels.update(rec["kernels"])
            old.update(rec)
            old["kernels"] = kernels
        else:
            old[key] = {"workload": WORKLOADS[args.workload] if key == "many" else "16 frames 6144x6160 (wide field)",
                        "kernels": rec["kernels"], "fetch_scale": rec["fetch_scale"],
                        "write_scale": rec["write_scale"]}
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
        print(json.dumps({"streaming_wide": streaming_wide(torch, rd, wide_inputs(torch, rd), alone=not args.no_alone)}))
        return 0
    if args.sweep:
        rd.lib()
        print(json.dumps({"sweep": sweep(torch, rd)}))
        return 0
    rd.lib()
    tuned = None
    if args.workload == 2:
        if args.path != "batched":
            print("bench.py: the 64-stack workload runs as one batched call", file=sys.stderr)
            return 2
        pipe = ManyStackPipeline(rd, torch, tune=not args.no_tune, tune_cache=args.tune_cache)
        log(f"64-stack inputs rendered and search shapes tuned: {pipe.plans}")
        specs = pipe.specs
        tuned = pipe.plans
    else:
        stacks = synth.make_config(args.workload)
        specs = [st.spec for st in stacks]
        integer_mode = args.workload == 0
        pipe = (BatchedPipeline if args.path == "batched" else StagePipeline)(rd, torch, stacks, integer_mode)
        if args.tune_cache and os.path.exists(args.tune_cache):
            rd.tune_load(args.tune_cache)
            tuned = "loaded"
        elif not args.no_tune:
            # timed on the frames one search launch covers
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
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms per step")

    kern = {name: rd.prof_query(name) for name in ("score_tiles", "calibrate", "shift", "combine", "batch_score",
                                                   "batch_fused", "batch_comb", "batch_shift")}
    batched = args.path == "batched"
    rd.prof_enable(False)

    score_ms, score_n = kern["batch_score" if batched else "score_tiles"]
    score_avg_s = score_ms / score_n / 1e3
    launches_per_step = score_n / args.steps
    # batched: the flops of the step's searches spread over its search dispatches (one per
    # group of stacks that share a launch shape); stage-wise: one stack's search per launch
    flops = search_flops(specs) / launches_per_step if batched else search_flops(specs[:1])
    achieved = flops / score_avg_s / 1e12
    kname = "batch_score" if batched else "score_tiles"
    traffic = recorded_traffic(args.traffic, kname, "many" if args.workload == 2 else None)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(FP64_VALU_PEAK_TFLOPS, 3),
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": kname, "avg_launch_ms": round(score_avg_s * 1e3, 4),
                "launches_per_step": round(launches_per_step, 3), "flops_per_launch": flops,
                "search_share_of_step": round(score_ms / args.steps / ms_per_step, 4)}
    # the other timed phases of a batched step (HIP events, ms per step)
    phases = {k: round(kern[k][0] / args.steps, 3) for k in ("batch_fused", "batch_comb", "batch_shift")
              if batched and kern[k][1]}

    streaming = {}
    if not batched:
        sbytes = streaming_bytes(specs[0])
        for name in ("calibrate", "shift", "combine"):
            ms, n = kern[name]
            if n:
                gbs = sbytes[name] / (ms / n / 1e3) / 1e9
                streaming[name] = {"avg_launch_ms": round(ms / n, 4), "GB/s": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": sbytes[name],
                                   "traffic": recorded_traffic(args.traffic, name)}

    value = pipe.pixels / (ms_per_step / 1e3) / 1e6
    frames = [sp.N for sp in specs]
    config = {"workload": WORKLOADS[args.workload], "stacks": len(specs), "frames_total": sum(frames),
              "input_pixels": pipe.pixels, "sizes": sorted({sp.W for sp in specs}), "path": args.path,
              "pixel_storage": "uint16 in, f32 between stages, f32 out", "search": "FP64 FMA of the float frame values and the FP64 mean-free reference",
              "search_plans": tuned if args.workload == 2 else rd.register_plan(specs[0].W, specs[0].H,
                                                                               specs[0].N - 1, specs[0].radius)}
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": config,
        "roofline": roofline,
    }
    if streaming:
        line["streaming"] = streaming
    if phases:
        line["phases_ms_per_step"] = phases
    sample = None
    if args.workload == 2:
        if not args.no_cpu_baseline:
            sample = many_sample(pipe)
        pipe.batch = None  # the direct-search workspace
        if not args.no_autotuned_search:
            line["autotuned_search"] = autotuned_search_leg(torch, rd, pipe)
            log(f"autotuned search: {line['autotuned_search']}")
        del pipe
        torch.cuda.empty_cache()
        if not args.no_bands:
            line["bands"] = bands_leg(torch, rd)
            log(f"bands: {line['bands']}")
    if not args.no_wide or not args.no_wide_chain:
        inp = wide_inputs(torch, rd)
        log("wide-field inputs rendered")
        if not args.no_wide_chain:
            line["wide_field_chain"] = wide_chain(torch, rd, inp)
            log(f"wide-field chain: {line['wide_field_chain']}")
        if not args.no_wide:
            line["streaming_wide"] = streaming_wide(torch, rd, inp)
            log("wide-field streaming kernels timed")
        del inp
        torch.cuda.empty_cache()
    if not args.no_learned:
        line["learned"] = learned_comparison(torch, rd, args.weights, args.learned_frames)
        log(f"learned: speed-up {line['learned']['speedup']}")
    if not args.no_cpu_baseline:
        if args.workload == 2:
            line["cpu_baseline"], line["parity"] = cpu_baseline_many(*sample, specs)
        else:
            line["cpu_baseline"] = cpu_baseline(stacks, integer_mode)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
