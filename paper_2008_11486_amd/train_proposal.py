"""Train the offset-proposal network on rendered 4096x4096 pairs and evaluate it.

    python -m paper_2008_11486_amd.train_proposal --pairs 20000 --epochs 4 \
        --out paper_2008_11486_amd/weights/proposal_4096.npy --summary run_summary.json

Training pairs are (reference, shifted frame) with offsets uniform in +-64 px, rendered
on the GPU and reduced to the network input on the GPU; the targets are the offsets in
downsampled pixels.  The evaluation uses stacks from a separate seed set: for each
frame the narrowed search around the trained and the untrained network's proposal is
compared with the full +-64 px search (fallback rate, centre error, identical integer
offsets).  The zero-offset score ratio that triggers a fallback is checked on
training pairs only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--bound", type=float, default=64.0)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-decay", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-budget", type=float, default=None,
                    help="seconds of training; the learning-rate schedule runs over this time")
    ap.add_argument("--eval-stacks", type=int, default=2)
    ap.add_argument("--eval-frames", type=int, default=16)
    ap.add_argument("--out", required=True)
    ap.add_argument("--summary", default=None)
    args = ap.parse_args(argv)

    from . import lib, offsets_to_numpy
    from . import learned
    lib()
    if not torch.cuda.is_available():
        print("train_proposal: no GPU visible", file=sys.stderr)
        return 2
    W = H = args.size
    rmax = int(round(args.bound))

    def log(msg):
        print(msg, flush=True)

    tr = learned.ProposalTrainer(W, H, args.batch, args.bound, lr=args.lr, weight_decay=args.weight_decay,
                                 seed=args.seed)
    untrained = tr.params.clone()
    t0 = time.perf_counter()
    hist = tr.train(args.pairs, args.epochs, warmup=100, log_every=20, log=log, time_budget=args.time_budget)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    learned.save_params(args.out, tr.params)
    log(f"trained {tr.steps} steps in {train_s:.1f} s -> {args.out}")

    # zero-offset score ratio at the true peak, on training pairs only
    ratios = []
    for i in range(8):
        stars, keys, _ = learned.pair_catalogues([i], W, H, args.bound, learned.TRAIN_SET)
        fr = torch.empty((2, H, W), dtype=torch.float32, device="cuda:0")
        from . import render_frames, register
        render_frames(torch.from_numpy(stars).cuda(), torch.from_numpy(keys).cuda(), W, H, sky=learned.SKY,
                      fwhm=learned.FWHM, read_noise=learned.READ_NOISE, seed=learned.SEED_ROOT, out=fr)
        full = offsets_to_numpy(register(fr[0], fr[1:2], rmax, rmax))
        auto = offsets_to_numpy(register(fr[0], fr[0:1], 0, rmax))
        ratios.append(float(full["peak"][0] / auto["peak"][0]))
    log(f"true-peak / zero-offset score on training pairs: min {min(ratios):.3f} max {max(ratios):.3f}")

    evals = []
    for s in range(args.eval_stacks):
        frames, t = learned.render_stack(s, args.eval_frames + 1, W, H, args.bound)
        ref, rest = frames[0], frames[1:].contiguous()
        full = offsets_to_numpy(learned.full_search(ref, rest, rmax))
        for name, p in (("untrained", untrained), ("trained", tr.params)):
            reg = learned.LearnedRegistrar(p, W, H, args.eval_frames, radius_max=rmax)
            r = reg.register(ref, rest)
            same = bool(np.all((r.offsets["dx"] == full["dx"]) & (r.offsets["dy"] == full["dy"])))
            err = np.abs(r.centres - np.stack([full["dx"], full["dy"]], 1)).max(axis=1)
            evals.append(dict(stack=s, weights=name, fallbacks=int(r.fallback.sum()), frames=args.eval_frames,
                              identical=same, centre_err_median=float(np.median(err)),
                              centre_err_max=float(err.max()), reasons=r.reason))
            log(json.dumps(evals[-1]))
        del frames, rest
    summary = dict(size=W, bound=args.bound, pairs=args.pairs, batch=args.batch, epochs=args.epochs,
                   time_budget=args.time_budget,
                   steps=tr.steps, lr=args.lr, weight_decay=args.weight_decay, train_seconds=round(train_s, 1),
                   loss_first=hist[0][1], loss_last=hist[-1][1], loss_history=hist,
                   true_peak_ratio_train=dict(min=min(ratios), max=max(ratios)), eval=evals)
    if args.summary:
        with open(args.summary, "w") as fh:
            json.dump(summary, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
