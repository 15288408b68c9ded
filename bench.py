"""Throughput of wavefront decoding of a 1080p-shaped I-frame on one MI355X.

One step = one whole frame decoded diagonal by diagonal (T = 455 steps of
accumulator, 6 layers and head, symbols taken from device memory), with the
inputs resident in HBM. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(cfg, Wt, y, z):
    """The FP64 oracle (parallel definition form) on the same frame."""
    import numpy as np
    from oracle import model as om
    t0 = time.perf_counter()
    om.forward(cfg, Wt, y, z)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": y.size / dt, "unit": "symbols/s", "cores": threads, "kind": "oracle",
            "sample": f"one full {y.shape[0]}x{y.shape[1]}x{y.shape[2]} I-frame, float64 "
                      f"parallel form, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the wavefront path "
              "is a single-device method", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2605_20977_amd import pswa

    cfg = synth.FULL
    H, W = 68, 120
    dseed, wseed = synth.CONFIG_SEEDS["1080p_I"]
    Wt = synth.model_weights(cfg, wseed)
    y, z, _ = synth.frame_inputs(cfg, synth.FrameCfg(H, W), dseed)
    model = pswa.Model(cfg, Wt, "fp32")
    yd = torch.from_numpy(y).cuda()
    zd = torch.from_numpy(z).cuda()
    mem = torch.empty(pswa.pswa_state_bytes(model, H, W), dtype=torch.uint8, device="cuda")

    def one_frame():
        st = pswa.pswa_decode_begin(model, H, W, zd, source="device", src=yd, mem=mem)
        for t in range(st.T):
            pswa.pswa_decode_step(st, t)
        pswa.pswa_decode_end(st, H, W, cfg.C, total_bits=False)
        st.close()

    for i in range(args.warmup):
        one_frame()
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} frames)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_frame()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sym = H * W * cfg.C * args.steps
    rec = {
        "metric": "decoded latent symbols/sec (1080p-shaped) vs plain FP32, at stated bits overhead",
        "value": sym / dt, "unit": "symbols/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1080p-shaped I-frame wavefront decode, latent 68x120x192, "
                               "6 layers d=384, 8 heads, causal 9x9 window (s=5, 455 steps)",
                   "path": "plain FP32, one launch per phase", "symbol_source": "device"},
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(cfg, Wt, y, z),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
