"""GPU parity of every persistent-kernel instance the benchmark and its
autotuner time, through the C ABI.

The persistent decode kernel is built once per (projection arithmetic, head
size, row tile). The 1080p-shaped model (8 heads of 48) runs in
  <BF16, 48, 32>  I-frames in groups of one frame x 8 workgroups and of four
                  frames x 4 workgroups,
  <BF16, 48, 16>  the mixed batch (grid sizes 15x20 .. 68x120, I and P) in
                  groups of two frames x 16 workgroups,
  <FP8, 48, 32>, <FP8, 48, 16>  the same with FP8 projections,
and the 4K student (4 heads of 32) in <BF16, 32, 16> / <BF16, 32, 32>.
Every batch must be bit-identical, frame by frame, to the parallel encode
form of the same model (which shares every per-row device function), and one
frame per case is compared with the FP64 oracle at sampled positions (cone
crops, tests/sampled_ref.py) within the precision's stated error bound.
"""
import numpy as np
import pytest

import synth
from sampled_ref import oracle_at, sample_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "bits", "center", "index", "latents")

# Error bounds of the low-precision forms against the FP64 oracle, per
# symbol: mean error |d mu| / max(|mu|, 1) and relative scale error; twice
# the largest errors measured on the 1080p-shaped I- and P-frames (BF16:
# 0.0152 / 0.0040; FP8 per-tensor: 0.244 / 0.068).
BOUND = {"bf16": (0.03, 0.008), "fp8": (0.5, 0.14)}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_20977_amd import pswa
    return pswa


def _frames(cfg, sizes, seed0):
    out = []
    for k, (H, W, npv) in enumerate(sizes):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), seed0 + 7 * k)
        out.append({"latents": y, "hyper": z, "prev": prev})
    return out


def _encode(P, model, f):
    o = P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"])
    o["latents"] = torch.as_tensor(f["latents"], device=o["mean"].device)
    return o


def _assert_same(a, b, label):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), f"{label}: {k} differs"
    assert a["total_bits"] == b["total_bits"], label


def _against_oracle(cfg, Wt, f, out, prec, n, seed, label):
    y = f["latents"]
    H, W = y.shape[:2]
    mu = out["mean"].cpu().numpy().astype(np.float64)
    sg = out["scale"].cpu().numpy().astype(np.float64)
    ref = oracle_at(cfg, Wt, y, f["hyper"], f["prev"], sample_positions(H, W, n, seed))
    emu = max(float(np.max(np.abs(mu[i, j] - r["mu"]) / np.maximum(np.abs(r["mu"]), 1)))
              for (i, j), r in ref.items())
    esg = max(float(np.max(np.abs(sg[i, j] - r["sigma"]) / r["sigma"])) for (i, j), r in ref.items())
    print(f"[{label}] vs FP64 oracle at {n} positions: mean err max {emu:.3e}, "
          f"scale err max {esg:.3e}", flush=True)
    bm, bs = BOUND[prec]
    assert emu <= bm and esg <= bs, (label, emu, esg)


@pytest.fixture(scope="module")
def full():
    cfg = synth.FULL
    return cfg, synth.model_weights(cfg, synth.CONFIG_SEEDS["batch"][1])


MIX = [(H, W, npv) for (H, W) in synth.BATCH_MIX for npv in (0, 2)]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_mixed_1080p_batch_every_timed_instance(P, full, prec):
    """One frame of every grid size of the mixed batch, I and P, through the
    row tiles 16 and 32 and both groupings the benchmark times, and both
    attention forms (global key loads, LDS-staged window tiles)."""
    cfg, Wt = full
    model = P.make_model(cfg, Wt, prec, synth.calibration_frames(cfg))
    fr = _frames(cfg, MIX, synth.CONFIG_SEEDS["batch"][0])
    ref = [_encode(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    assert b.T == 455
    for fpg, bpg in ((2, 16), (1, 8)):
        for rt in (16, 32):
            print(f"case mixed 1080p {prec} groups {fpg}x{bpg} rtile {rt}", flush=True)
            b.set_groups(fpg, bpg)
            b.set_rtile(rt)
            b.run()
            b.check()
            for k in range(len(fr)):
                _assert_same(b.outputs(k), ref[k], f"{prec} {fpg}x{bpg} rtile {rt} frame {k}")
    b.set_rtile(16)
    b.set_attention(True)
    for fpg, bpg in ((2, 16), (1, 8)):
        print(f"case mixed 1080p {prec} groups {fpg}x{bpg} rtile 16 staged", flush=True)
        b.set_groups(fpg, bpg)
        b.run()
        b.check()
        for k in range(len(fr)):
            _assert_same(b.outputs(k), ref[k], f"{prec} {fpg}x{bpg} staged frame {k}")
    # the 34 x 60 P-frame against the oracle
    _against_oracle(cfg, Wt, fr[3], ref[3], prec, 6, 31, f"mixed {prec} 34x60 P")


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_headline_1080p_i_batch(P, full, prec):
    """1080p-shaped I-frames, replayed from a HIP graph, in the groupings the
    headline batches use: one frame x 8 workgroups (row tile 32, global key
    loads), and four frames sharing 4 workgroups (row tile 16, LDS-staged
    attention)."""
    cfg, Wt = full
    model = P.make_model(cfg, Wt, prec, synth.calibration_frames(cfg))
    fr = _frames(cfg, [(68, 120, 0)] * 4, synth.CONFIG_SEEDS["1080p_I"][0])
    ref = [_encode(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    for fpg, bpg in ((1, 8), (4, 4)):
        b.set_groups(fpg, bpg)
        b.set_rtile(32 if fpg == 1 else 16)
        b.set_attention(fpg == 4)
        b.capture()
        for rep in range(2):
            print(f"case headline 1080p {prec} groups {fpg}x{bpg} replay {rep}", flush=True)
            b.run()
            b.check()
            for k in range(len(fr)):
                _assert_same(b.outputs(k), ref[k],
                             f"{prec} {fpg}x{bpg} replay {rep} frame {k}")
    _against_oracle(cfg, Wt, fr[0], ref[0], prec, 5, 41, f"headline {prec} 68x120 I")


@pytest.mark.parametrize("rt", [16, 32])
def test_student_4k_bf16_batch_row_tiles(P, rt):
    """The 4K student (4 heads of 32) in BF16, one frame per group of 32
    workgroups, at both row tiles (row tile 16 with LDS-staged attention)."""
    cfg = synth.STUDENT
    Wt = synth.model_weights(cfg, 51)
    model = P.make_model(cfg, Wt, "bf16")
    seed = synth.CONFIG_SEEDS["4k_student"][0]
    fr = _frames(cfg, [(135, 240, 0), (135, 240, 2)], seed + 20)
    ref = [_encode(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    b.set_groups(1, 32)
    b.set_rtile(rt)
    b.set_attention(rt == 16)
    print(f"case student 4K bf16 rtile {rt}", flush=True)
    b.run()
    b.check()
    for k in range(len(fr)):
        _assert_same(b.outputs(k), ref[k], f"student rtile {rt} frame {k}")
    _against_oracle(cfg, Wt, fr[1], ref[1], "bf16", 5, 51 + rt, f"student 4K bf16 P rtile {rt}")
