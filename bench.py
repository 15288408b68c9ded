"""Throughput of wavefront decoding of 1080p-shaped latents on one MI355X.

Workload (the headline): a batch of 32 1080p-shaped I-frames, each latent
68x120x192 with hyperprior 17x30x128, decoded by the 6-layer d=384 context
model (8 heads of 48, causal 9x9 window, wavefront slope 5, 455 diagonals per
frame); inputs resident in HBM, symbols read from device memory. Paths
(`--paths`, comma separated):
  plain:<prec>     -- one frame, one kernel launch per phase per diagonal;
  batch<N>:<prec>  -- N 1080p I-frames in one persistent launch;
  mixed<N>:<prec>  -- N frames of the mixed batch (15x20, 34x60, 45x80 and
                      68x120 in equal numbers, I- and P-frames alternating)
                      in one persistent launch;
  cyclic<N>:<prec>  -- N 1080p I-frames decoded with the paper's cyclic
                      schedule (step = (i + j) mod 4, full 7x7 window: 4
                      steps per frame) by a model of the same widths;
  student4k:<prec> -- one 4K-shaped I-frame and one P-frame (135x240x192)
                      decoded by the 2-layer d=128 student model (weights
                      at initialization: the rate does not depend on them);
with <prec> one of fp32, bf16, fp8. Persistent paths split their frames into
groups that run behind their own barriers; the library's autotuner picks the
grouping and row tile, and runs replay a captured HIP graph, unless told not
to. One step = one pass of a path over its batch. The headline `value` is the
fastest path; `paths` gives every path's rate and its ratio to plain FP32.
The roofline is that of the headline path's dominant kernel, timed live with
HIP events on its launch stream over an instrumented repeat of the timed
steps (issued kernel by kernel).
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
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0}
FP32_VECTOR_TFLOPS = 157.3
METRIC = "decoded latent symbols/sec (1080p-shaped) vs plain FP32, at stated bits overhead"
ROLE_KERNEL = {
    "persistent_decode": "k_persistent (every phase of every diagonal of the batch, one launch)",
    "down_gemm": "k_gemm<0, false, 1, 8> (residual epilogue, K=1536)",
    "gateup_swiglu_gemm": "k_gemm<0, true, 4, 2> (RMSNorm prologue, SwiGLU epilogue)",
    "qkv_gemm": "k_gemm<0, true, 2, 2> (RMSNorm prologue, QKV epilogue)",
    "o_gemm": "k_gemm<0, false, 1, 2> (residual epilogue, K=384)",
    "layer_attention": "k_attn<48>",
}
DEFAULT_PATHS = ("plain:fp32,batch32:bf16,batch32:fp8,mixed32:bf16,student4k:bf16,"
                 "cyclic32:bf16")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--paths", default=DEFAULT_PATHS,
                    help="comma list of plain:<prec>, batch<N>:<prec>, mixed<N>:<prec>")
    ap.add_argument("--grid", type=int, default=0,
                    help="one group of this many blocks; 0 lets the autotuner choose")
    ap.add_argument("--rtile", type=int, default=0, help="row tile 16/32; 0: autotuner")
    ap.add_argument("--groups", default="", metavar="FxB",
                    help="F frames per group, B blocks per group (default: autotuner)")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON-lines cache file")
    ap.add_argument("--no-graph", action="store_true", help="issue runs without a HIP graph")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES bytes (a known-size "
                         "kernel for scaling memory counters)")
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


def measured_traffic(role, prec, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources, this arithmetic and this workload
    (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{role}|{prec}|{workload}")
    if not rec or rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(cfg, Wt, y, z, budget_s=12.0):
    """The FP64 oracle (parallel definition form) on whole 1080p I-frames of
    the workload, repeated until about budget_s seconds have passed."""
    from oracle import model as om
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    n = 0
    while True:
        om.forward(cfg, Wt, y, z)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    return {"value": n * y.size / dt, "unit": "symbols/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} whole {y.shape[0]}x{y.shape[1]}x{y.shape[2]} I-frame(s) of the "
                      f"workload, float64 parallel form, {dt:.1f} s, BLAS threads {threads}"}


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


def roofline(pswa, fn, steps, prec, workload):
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
    bytes_l = p["bytes"] / p["launches"]
    flops_l = p["flops"] / p["launches"]
    # the roofline's own rule: arithmetic intensity (algorithmic flops per
    # algorithmic byte) against the ridge of the compute peak in use
    peak_tf = MFMA_PEAK_TFLOPS.get(prec, FP32_VECTOR_TFLOPS) if dom == "persistent_decode" \
        else FP32_VECTOR_TFLOPS
    intensity = flops_l / bytes_l if bytes_l else float("inf")
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    tf = flops_l / avg_s / 1e12
    gbs = bytes_l / avg_s / 1e9
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma" if prec in MFMA_PEAK_TFLOPS else "alu", "achieved": tf,
                "peak": peak_tf, "unit": "TFLOP/s", "frac": tf / peak_tf}
    roof.update({"intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "compute_frac": tf / peak_tf, "compute_peak_tflops": peak_tf})
    roof.update({"traffic": measured_traffic(dom, prec, workload),
                 "kernel": ROLE_KERNEL.get(dom, dom), "role": dom,
                 "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": bytes_l,
                 "alg_flops_per_launch": flops_l, "launches_per_step": p["launches"] / steps,
                 "hbm_GBps_alg": bytes_l / avg_s / 1e9})
    tot = sum(v["ms"] for v in prof.values())
    kernels = {k: {"share": round(v["ms"] / tot, 4),
                   "avg_us": round(1e3 * v["ms"] / v["launches"], 3),
                   "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                   "TFLOPs": round(v["flops"] / (v["ms"] / 1e3) / 1e12, 3)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    return roof, kernels


def batch_frames(synth, cfg, kind, n, dseed):
    """Inputs of a batch path: n 1080p I-frames, n frames of the mixed batch
    (sizes in equal numbers, I- and P-frames alternating per size), or the
    4K-shaped I- and P-frame of the student workload."""
    frames = []
    if kind == "student4k":
        s0 = synth.CONFIG_SEEDS["4k_student"][0]
        for k, n_prev in enumerate((0, 2)):
            y, z, pv = synth.frame_inputs(synth.STUDENT, synth.FrameCfg(135, 240, n_prev), s0 + k)
            frames.append({"latents": y, "hyper": z, "prev": pv})
        return frames
    for k in range(n):
        if kind in ("batch", "cyclic"):
            fc, seed = synth.FrameCfg(68, 120), dseed + 1000 * k
        else:
            H, W = synth.BATCH_MIX[(k * len(synth.BATCH_MIX)) // n]
            fc, seed = synth.FrameCfg(H, W, 2 if k % 2 else 0), synth.CONFIG_SEEDS["batch"][0] + k
        y, z, pv = synth.frame_inputs(cfg, fc, seed)
        frames.append({"latents": y, "hyper": z, "prev": pv})
    return frames


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): every path here is "
              "measured on a single device", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2605_20977_amd import pswa

    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {args.calibrate_copy} bytes", file=sys.stderr, flush=True)
        del src, dst

    cfg = synth.FULL
    H, W = 68, 120
    dseed, wseed = synth.CONFIG_SEEDS["1080p_I"]
    Wt = synth.model_weights(cfg, wseed)
    y, z, _ = synth.frame_inputs(cfg, synth.FrameCfg(H, W), dseed)
    yd = torch.from_numpy(y).cuda()
    zd = torch.from_numpy(z).cuda()
    sym_frame = H * W * cfg.C
    models = {}

    def model_for(prec, kind="full"):
        key = (prec, kind)
        if key not in models:
            if kind == "student":
                models[key] = pswa.Model(synth.STUDENT, synth.model_weights(synth.STUDENT, 51),
                                         prec)
            elif kind == "cyclic":
                models[key] = pswa.Model(
                    synth.CYCLIC,
                    synth.model_weights(synth.CYCLIC, synth.CONFIG_SEEDS["1080p_cyclic"][1]), prec)
            else:
                models[key] = pswa.Model(cfg, Wt, prec)
        return models[key]

    paths, runners, keep = {}, {}, []
    for spec in args.paths.split(","):
        kind, prec = spec.split(":")
        model = model_for(prec, "student" if kind == "student4k"
                          else "cyclic" if kind.startswith("cyclic") else "full")
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
            paths[spec] = {"frames": 1, "symbols_per_step": sym_frame,
                           "ms_per_step": 1e3 * dt / args.steps,
                           "value": sym_frame * args.steps / dt}
            runners[spec] = plain
        else:
            if kind == "student4k":
                base, n = "student4k", 2
            else:
                base = next(b_ for b_ in ("batch", "mixed", "cyclic") if kind.startswith(b_))
                n = int(kind[len(base):])
            frames = batch_frames(synth, cfg, base, n, dseed)
            nsym = sum(f["latents"].size for f in frames)
            b = pswa.Batch(model, frames)
            keep.append(b)
            tuned = None
            if args.grid:
                b.set_grid(args.grid)
            if args.rtile:
                b.set_rtile(args.rtile)
            if args.groups:
                f, g = (int(v) for v in args.groups.split("x"))
                b.set_groups(f, g)
            if not args.grid and not args.rtile and not args.groups:
                print(f"{spec}: autotuning", file=sys.stderr, flush=True)
                f, g, r, est = b.autotune(args.tune_cache, reps=2)
                tuned = {"frames_per_group": f, "blocks_per_group": g, "rtile": r,
                         "est_ms": round(est, 2)}
            if not args.no_graph:
                b.capture()

            def run(b=b):
                b.run()
            dt = timed(run, args.steps, args.warmup)
            b.check()
            fpg, bpg, ngr = b.groups
            paths[spec] = {"frames": n, "symbols_per_step": nsym, "grid": b.grid,
                           "groups": f"{ngr} x ({fpg} frames, {bpg} blocks)", "rtile": b.rtile,
                           "graph": not args.no_graph, "autotuned": tuned,
                           "ms_per_step": 1e3 * dt / args.steps,
                           "value": nsym * args.steps / dt}
            runners[spec] = run
        print(f"{spec}: {paths[spec]['ms_per_step']:.2f} ms per step "
              f"({paths[spec]['frames']} frame(s)) -> "
              f"{paths[spec]['value'] / 1e6:.2f} M symbols/s", file=sys.stderr, flush=True)

    base = paths.get("plain:fp32", {}).get("value")
    for p in paths.values():
        p["vs_plain_fp32"] = (p["value"] / base) if base else None
    # the headline is a 1080p-shaped path (the mixed batch and the student's
    # 4K frames are reported beside it)
    # (BF16 when it ran: the tighter bits-overhead bound; FP8 is reported
    # beside it in "paths")
    cand = ([k for k in paths if k.startswith("batch") and k.endswith(":bf16")]
            or [k for k in paths if k.split(":")[0].startswith(("plain", "batch"))]
            or list(paths))
    best = max(cand, key=lambda k: paths[k]["value"])
    hp = paths[best]
    kind, prec = best.split(":")
    if kind == "plain":
        workload = "1080p-shaped I-frame, per-diagonal launches"
        path_descr = f"{prec.upper()} projections, one kernel launch per phase per diagonal"
    else:
        workload = f"{hp['frames']} 1080p-shaped I-frames, one persistent launch"
        path_descr = (f"{prec.upper()} projections on MFMA (FP32 accumulate; FP32 softmax, "
                      f"norms, accumulator and CDF), one persistent launch per batch of "
                      f"{hp['frames']} frames, {hp['groups']} groups with their own barriers, "
                      f"row tile {hp['rtile']}"
                      + (", HIP graph replay" if hp["graph"] else ""))
    roof = kernels = None
    if not args.no_roofline:
        roof, kernels = roofline(pswa, runners[best], args.steps, prec, workload)
    overhead = {"fp32": "FP32: max relative error <= 1e-4 on mean/scale against the FP64 "
                        "oracle (parity tests)",
                "bf16": "BF16 projections: bits overhead vs FP64 oracle <= 0.5 % (measured "
                        "-0.0001 % on the 1080p-shaped P-frame)",
                "fp8": "FP8 e4m3 projections: bits overhead vs FP64 oracle <= 1 % (measured "
                       "-0.0071 % on the 1080p-shaped P-frame)"}[prec]
    rec = {
        "metric": METRIC, "value": hp["value"], "unit": "symbols/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hp["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[prec],
        "data": "synthetic",
        "config": {"workload": workload + ": latent 68x120x192, hyperprior 17x30x128, "
                               "6 layers d=384, 8 heads of 48, causal 9x9 window (slope 5, "
                               "455 diagonals per frame), symbols read from device memory",
                   "path": path_descr, "frames_per_step": hp["frames"],
                   "bits_overhead": overhead},
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
