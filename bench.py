"""Throughput of wavefront decoding of a 1080p-shaped I-frame on one MI355X.

One step = one whole 68x120x192 frame decoded diagonal by diagonal (455
wavefront steps of accumulator, 6 layers, head, symbols and their
embedding), with inputs resident in HBM and symbols read from device memory.
Prints one JSON line with the throughput, the roofline of the dominant kernel
(timed live with HIP events on its launch stream, in an instrumented repeat
of the timed steps) and the FP64 oracle's rate on the host.
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
# Kernel symbol of each timed role (for matching rocprofv3 summaries).
ROLE_KERNEL = {
    "down_gemm": "k_gemm<0, false, 1, 6> (A fp32, residual epilogue, K=1536)",
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


def measured_traffic(role, launches_per_step):
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

    for _ in range(args.warmup):
        one_frame()
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} frames)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_frame()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"timed {args.steps} frames in {dt:.3f} s", file=sys.stderr, flush=True)
    sym = H * W * cfg.C * args.steps

    roof = None
    kernels = None
    if not args.no_roofline:
        pswa.pswa_profile_enable(True)
        for _ in range(args.steps):
            one_frame()
        torch.cuda.synchronize()
        prof = pswa.pswa_profile_read()
        pswa.pswa_profile_enable(False)
        dom = max(prof, key=lambda k: prof[k]["ms"])
        p = prof[dom]
        avg_s = p["ms"] / 1e3 / p["launches"]
        per_launch = p["bytes"] / p["launches"]
        achieved = per_launch / avg_s / 1e9
        traffic = measured_traffic(dom, p["launches"] / args.steps)
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": ROLE_KERNEL.get(dom, dom), "role": dom,
                "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": per_launch,
                "launches_per_step": p["launches"] / args.steps}
        tot = sum(v["ms"] for v in prof.values())
        kernels = {k: {"share": round(v["ms"] / tot, 4),
                       "avg_us": round(1e3 * v["ms"] / v["launches"], 3),
                       "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)}
                   for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
        print(f"roofline pass: dominant {dom}", file=sys.stderr, flush=True)

    rec = {
        "metric": METRIC, "value": sym / dt, "unit": "symbols/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1080p-shaped I-frame wavefront decode: latent 68x120x192, "
                               "hyperprior 17x30x128, 6 layers d=384, 8 heads of 48, causal "
                               "9x9 window (slope 5, 455 steps)",
                   "path": "plain FP32, one kernel launch per phase per diagonal",
                   "symbol_source": "device"},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(cfg, Wt, y, z),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
