"""Throughput of wavefront decoding of 1080p-shaped latents on one MI355X.

Workload: 1080p-shaped I-frames, latent 68x120x192 with hyperprior 17x30x128,
decoded by the 6-layer d=384 context model (8 heads of 48, causal 9x9 window,
wavefront slope 5, 455 diagonals per frame); inputs resident in HBM, symbols
read from device memory. Paths measured:
  plain      -- FP32, one kernel launch per phase per diagonal, one frame;
  persistent -- FP32, one persistent launch per batch of B frames.
The headline `value` is the fastest path; one step = one pass of that path
over its batch (1 frame for plain, B frames for persistent). `paths` gives
every path's rate and its ratio to the plain FP32 path. The roofline is that
of the headline path's dominant kernel, timed live with HIP events on its
launch stream in an instrumented repeat of the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "decoded latent symbols/sec (1080p-shaped) vs plain FP32, at stated bits overhead"
ROLE_KERNEL = {
    "persistent_decode": "k_persistent (all phases of all diagonals, one launch)",
    "down_gemm": "k_gemm<0, false, 1, 8> (residual epilogue, K=1536)",
    "gateup_swiglu_gemm": "k_gemm<0, true, 4, 2> (RMSNorm prologue, SwiGLU epilogue)",
    "qkv_gemm": "k_gemm<0, true, 2, 2> (RMSNorm prologue, QKV epilogue)",
    "o_gemm": "k_gemm<0, false, 1, 2> (residual epilogue, K=384)",
    "layer_attention": "k_attn<48>",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--paths", default="plain:fp32,batch1:bf16,batch8:bf16,batch8:fp8",
                    help="comma list of plain:<prec> and batch<N>:<prec>, prec in "
                         "fp32/bf16/fp8")
    ap.add_argument("--grid", type=int, default=0, help="persistent grid (0: default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    return ap.parse_args()


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_20977_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(role):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_1080p_decode.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    r = rec.get("roles", {}).get(role)
    return None if r is None else r["hbm_bytes_per_launch"]


def cpu_baseline(cfg, Wt, y, z):
    """The FP64 oracle (parallel definition form) on the same frame."""
    from oracle import model as om
    t0 = time.perf_counter()
    om.forward(cfg, Wt, y, z)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": y.size / dt, "unit": "symbols/s", "cores": threads, "kind": "oracle",
            "sample": f"one full {y.shape[0]}x{y.shape[1]}x{y.shape[2]} I-frame, float64 "
                      f"parallel form, {dt:.1f} s"}


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def roofline(pswa, fn, steps):
    import torch
    pswa.pswa_profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = pswa.pswa_profile_read()
    pswa.pswa_profile_enable(False)
    dom = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    avg_s = p["ms"] / 1e3 / p["launches"]
    per_launch = p["bytes"] / p["launches"]
    achieved = per_launch / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
            "kernel": ROLE_KERNEL.get(dom, dom), "role": dom,
            "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": per_launch,
            "launches_per_step": p["launches"] / steps}
    tot = sum(v["ms"] for v in prof.values())
    kernels = {k: {"share": round(v["ms"] / tot, 4),
                   "avg_us": round(1e3 * v["ms"] / v["launches"], 3),
                   "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    return roof, kernels


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the wavefront path is "
              "measured on a single device; see DESIGN.md for how it would shard",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2605_20977_amd import pswa

    cfg = synth.FULL
    H, W = 68, 120
    dseed, wseed = synth.CONFIG_SEEDS["1080p_I"]
    Wt = synth.model_weights(cfg, wseed)
    y, z, _ = synth.frame_inputs(cfg, synth.FrameCfg(H, W), dseed)
    yd = torch.from_numpy(y).cuda()
    zd = torch.from_numpy(z).cuda()
    sym_frame = H * W * cfg.C
    models = {}

    def model_for(prec):
        if prec not in models:
            models[prec] = pswa.Model(cfg, Wt, prec)
        return models[prec]

    paths = {}
    runners = {}
    keep = []
    for spec in args.paths.split(","):
        kind, prec = spec.split(":")
        model = model_for(prec)
        if kind == "plain":
            mem = torch.empty(pswa.pswa_state_bytes(model, H, W), dtype=torch.uint8,
                              device="cuda")

            def plain(model=model, mem=mem):
                st = pswa.pswa_decode_begin(model, H, W, zd, source="device", src=yd, mem=mem)
                for t in range(st.T):
                    pswa.pswa_decode_step(st, t)
                pswa.pswa_decode_end(st, H, W, cfg.C, total_bits=False)
                st.close()
            dt = timed(plain, args.steps, args.warmup)
            paths[spec] = {"frames_per_step": 1, "ms_per_step": 1e3 * dt / args.steps,
                           "value": sym_frame * args.steps / dt}
            runners[spec] = plain
        else:
            nframes = int(kind[len("batch"):])
            frames = []
            for k in range(nframes):
                yk, zk, _ = synth.frame_inputs(cfg, synth.FrameCfg(H, W), dseed + 1000 * k)
                frames.append({"latents": yk, "hyper": zk, "prev": None})
            b = pswa.Batch(model, frames, grid=args.grid)
            keep.append(b)

            def run(b=b):
                b.run()
            dt = timed(run, args.steps, args.warmup)
            b.check()
            paths[spec] = {"frames_per_step": nframes, "grid": b.grid,
                           "ms_per_step": 1e3 * dt / args.steps,
                           "value": sym_frame * nframes * args.steps / dt}
            runners[spec] = run
        print(f"{spec}: {paths[spec]['ms_per_step']:.2f} ms per step "
              f"({paths[spec]['frames_per_step']} frame(s)) -> "
              f"{paths[spec]['value'] / 1e6:.2f} M symbols/s", file=sys.stderr, flush=True)

    base = paths.get("plain:fp32", {}).get("value")
    for p in paths.values():
        p["vs_plain_fp32"] = (p["value"] / base) if base else None
    best = max(paths, key=lambda k: paths[k]["value"])
    hp = paths[best]
    roof = kernels = None
    if not args.no_roofline:
        roof, kernels = roofline(pswa, runners[best], args.steps)

    kind, prec = best.split(":")
    if kind == "plain":
        path_descr = f"{prec.upper()} projections, one kernel launch per phase per diagonal"
    else:
        path_descr = (f"{prec.upper()} projections (FP32 softmax, norms, accumulator and CDF), "
                      f"one persistent launch per batch of {kind[5:]} frames")
    rec = {
        "metric": METRIC, "value": hp["value"], "unit": "symbols/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hp["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[prec],
        "data": "synthetic",
        "config": {"workload": "1080p-shaped I-frame wavefront decode: latent 68x120x192, "
                               "hyperprior 17x30x128, 6 layers d=384, 8 heads of 48, causal "
                               "9x9 window (slope 5, 455 diagonals per frame)",
                   "path": path_descr, "frames_per_step": hp["frames_per_step"],
                   "symbol_source": "device", "bits_overhead_vs_fp64": "FP32 path, max "
                   "relative error <= 1e-4 on mean/scale against the FP64 oracle"},
        "vs_plain_fp32": hp["vs_plain_fp32"],
        "paths": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in paths.items()},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(cfg, Wt, y, z),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
