"""Distil the student context model from the full model on generated latents.

Usage (one GPU):
  python paper_2605_20977_amd/distill.py --crops 2000 --size 48 --epochs 4 \
      --out student.npz --report report.json

Steps: generate `crops` latent crops (half I-frames, half P-frames with two
previous latents) with the seeded generator, label them with the full
model's mean and log-scale (FP32 encode form), train the student with the
library's FP32 training kernels (AdamW, I and P batches alternating), then
measure on held-out 4K-shaped frames the bits of the full model, of the
untrained and of the trained student (FP32 and BF16 inference), and the
per-frame fallback decision. Writes the trained weights (npz) and a JSON
report.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--crops", type=int, default=2000)
    ap.add_argument("--size", type=int, default=48)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--wd", type=float, default=0.01)
    ap.add_argument("--eval-frames", default="135x240", help="HxW of the held-out frames")
    ap.add_argument("--out", default="")
    ap.add_argument("--report", default="")
    args = ap.parse_args()

    import torch
    import synth
    from paper_2605_20977_amd import pswa

    full, stud = synth.FULL, synth.STUDENT
    teacher_w = synth.model_weights(full, synth.CONFIG_SEEDS["4k_student"][1])
    init_w = synth.model_weights(stud, 51)
    teacher = pswa.Model(full, teacher_w)
    S = args.size
    t0 = time.time()

    # ---- data: generated crops labelled by the full model
    data = {0: [], 2: []}
    for k in range(args.crops):
        n_prev = 0 if k % 2 == 0 else 2
        y, z, prev = synth.frame_inputs(full, synth.FrameCfg(S, S, n_prev), 1000 + k)
        o = pswa.pswa_encode_params(teacher, y, z, prev, total_bits=False)
        data[n_prev].append((y, z, prev, o["mean"], torch.log(o["scale"].double()).float()))
        if (k + 1) % 250 == 0:
            print(f"labelled {k + 1}/{args.crops} crops ({time.time() - t0:.0f} s)", flush=True)

    def stack(items, n_prev):
        ys = torch.as_tensor(np.stack([c[0] for c in items])).cuda()
        zs = torch.as_tensor(np.stack([c[1] for c in items])).cuda()
        ps = torch.as_tensor(np.stack([c[2] for c in items])).cuda() if n_prev else None
        mus = torch.stack([c[3] for c in items]).contiguous()
        lss = torch.stack([c[4] for c in items]).contiguous()
        return ys, zs, ps, mus, lss

    # ---- training
    tr = pswa.Trainer(stud, init_w, max_crops=args.batch, H=S, W=S)
    rng = np.random.default_rng(0)
    curve = []
    steps_per_epoch = args.crops // args.batch
    for ep in range(args.epochs):
        order = {n: rng.permutation(len(data[n])) for n in data}
        losses = []
        for it in range(steps_per_epoch):
            n_prev = 0 if it % 2 == 0 else 2
            half = it // 2
            idx = order[n_prev][(half * args.batch) % len(data[n_prev]):][:args.batch]
            if len(idx) < args.batch:
                idx = order[n_prev][:args.batch]
            ys, zs, ps, mus, lss = stack([data[n_prev][i] for i in idx], n_prev)
            lr = args.lr * 0.5 * (1 + math.cos(math.pi * (ep * steps_per_epoch + it)
                                                 / (args.epochs * steps_per_epoch)))
            losses.append(tr.step(ys, zs, mus, lss, prev=ps, lr=lr, weight_decay=args.wd))
        curve.append(float(np.mean(losses)))
        print(f"epoch {ep + 1}/{args.epochs}: mean loss {curve[-1]:.4f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    trained_w = tr.read("weights")

    # ---- evaluation on held-out frames
    Hf, Wf = (int(v) for v in args.eval_frames.split("x"))
    models = {"full": teacher,
              "student_untrained": pswa.Model(stud, init_w),
              "student_trained": pswa.Model(stud, trained_w),
              "student_trained_bf16": pswa.Model(stud, trained_w, "bf16")}
    evals = []
    for k, n_prev in enumerate((0, 2)):
        y, z, prev = synth.frame_inputs(full, synth.FrameCfg(Hf, Wf, n_prev),
                                        synth.CONFIG_SEEDS["4k_student"][0] + k)
        bits = {n: pswa.pswa_encode_params(m, y, z, prev)["total_bits"] for n, m in models.items()}
        rec = {"frame": f"{Hf}x{Wf}x{full.C} {'P' if n_prev else 'I'}", "bits": bits,
               "overhead_vs_full": {n: bits[n] / bits["full"] - 1.0 for n in bits if n != "full"},
               "student_kept": pswa.pswa_student_accept(bits["student_trained_bf16"],
                                                        bits["full"], 0.01)}
        evals.append(rec)
        print(json.dumps(rec), flush=True)
    report = {"crops": args.crops, "crop": f"{S}x{S}x{full.C}", "batch": args.batch,
              "epochs": args.epochs, "steps": tr.steps, "lr": args.lr, "weight_decay": args.wd,
              "loss_per_epoch": curve, "eval": evals, "seconds": time.time() - t0}
    if args.out:
        np.savez(args.out, **trained_w)
    if args.report:
        json.dump(report, open(args.report, "w"), indent=1)
    print(json.dumps({"loss_per_epoch": curve, "seconds": report["seconds"]}), flush=True)


if __name__ == "__main__":
    main()
