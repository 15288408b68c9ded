"""GPU tests of the Channel Transformer and grouped heads, through the C ABI.

* tiny model with 4 channel groups (I- and P-frames, frames narrower than a
  window): the encode form matches the FP64 oracle (mean and scale to 1e-4
  relative, total bits to 1e-3) and the step decode, which predicts the
  groups of each diagonal one after the other and reads each group's
  symbols before the next, is bit-identical to it;
* the 1080p-shaped model with 4 channel groups: encode against the oracle at
  sampled positions (cone crops) and a full step decode bit-identical to
  encode;
* a BF16 model with channel groups (spatial projections on MFMA, the channel
  transformer in FP32): step decode bit-identical to encode, error bounded;
* the persistent batched decode of FP32 models with channel groups (the
  channel groups as extra phases of each step): every frame bit-identical to
  its step decode, across groupings, I- and P-frames and frames narrower
  than a window, and at 1080p to the encode form;
* what is not built is refused: the batched decode of BF16/FP8 models with
  channel groups, bitstream decoding and training.
"""
import numpy as np
import pytest

import synth
from oracle import entropy as oe
from oracle import model as om
from sampled_ref import oracle_at, sample_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "bits", "center", "index")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_20977_amd import pswa
    return pswa


def _same(a, b, label):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), f"{label}: {k}"


def _err(out, ref):
    mu = out["mean"].cpu().numpy().astype(np.float64)
    sg = out["scale"].cpu().numpy().astype(np.float64)
    emu = np.max(np.abs(mu - ref["mu"]) / np.maximum(np.abs(ref["mu"]), 1))
    esg = np.max(np.abs(sg - ref["sigma"]) / ref["sigma"])
    return emu, esg


@pytest.mark.parametrize("H,W,npv", [(16, 16, 0), (13, 21, 2), (5, 3, 0), (1, 7, 2)])
def test_tiny_ct_encode_matches_oracle_and_decode(P, H, W, npv):
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 21)
    model = P.Model(cfg, Wt)
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), 80 + H)
    print(f"case tiny CT {H}x{W} P={npv}", flush=True)
    enc = P.pswa_encode_params(model, y, z, prev)
    ref = om.forward(cfg, Wt, y, z, prev)
    emu, esg = _err(enc, ref)
    b_ref = float(oe.bits(y, ref["mu"], ref["sigma"]).sum())
    print(f"[tiny CT {H}x{W}] mean err {emu:.3e} scale err {esg:.3e} bits "
          f"{enc['total_bits']:.1f} vs {b_ref:.1f}", flush=True)
    assert emu <= 1e-4 and esg <= 1e-4
    assert abs(enc["total_bits"] - b_ref) <= 1e-3 * b_ref
    dec = P.decode_frame(model, H, W, z, prev=prev, source="device", src=y)
    _same(dec, enc, f"tiny CT {H}x{W}")
    assert np.array_equal(dec["latents"].cpu().numpy(), y)


def test_1080p_ct_encode_sampled_oracle_and_decode(P):
    cfg = synth.FULL_CT
    Wt = synth.model_weights(cfg, 22)
    model = P.Model(cfg, Wt)
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(68, 120, 2), 90)
    print("case 1080p CT P-frame", flush=True)
    enc = P.pswa_encode_params(model, y, z, prev)
    mu = enc["mean"].cpu().numpy().astype(np.float64)
    sg = enc["scale"].cpu().numpy().astype(np.float64)
    ref = oracle_at(cfg, Wt, y, z, prev, sample_positions(68, 120, 6, 91))
    for (i, j), r in ref.items():
        emu = np.max(np.abs(mu[i, j] - r["mu"]) / np.maximum(np.abs(r["mu"]), 1))
        esg = np.max(np.abs(sg[i, j] - r["sigma"]) / r["sigma"])
        assert emu <= 1e-4 and esg <= 1e-4, (i, j, emu, esg)
    dec = P.decode_frame(model, 68, 120, z, prev=prev, source="device", src=y)
    _same(dec, enc, "1080p CT")


def test_bf16_ct_decode_equals_encode(P):
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 23)
    model = P.Model(cfg, Wt, "bf16")
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(12, 15, 2), 95)
    enc = P.pswa_encode_params(model, y, z, prev)
    dec = P.decode_frame(model, 12, 15, z, prev=prev, source="device", src=y)
    _same(dec, enc, "bf16 CT")
    emu, esg = _err(enc, om.forward(cfg, Wt, y, z, prev))
    print(f"[tiny CT bf16] mean err {emu:.3e} scale err {esg:.3e}", flush=True)
    assert emu <= 0.05 and esg <= 0.02


def _frames(cfg, sizes, seed):
    out = []
    for k, (H, W, npv) in enumerate(sizes):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), seed + k)
        out.append({"latents": y, "hyper": z, "prev": prev})
    return out


def test_ct_batch_equals_step_decode(P):
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 25)
    model = P.Model(cfg, Wt)
    sizes = [(16, 16, 0), (13, 21, 2), (5, 3, 0), (1, 7, 2), (9, 2, 0), (12, 4, 2)]
    fr = _frames(cfg, sizes, 300)
    ref = [P.decode_frame(model, f["latents"].shape[0], f["latents"].shape[1], f["hyper"],
                          prev=f["prev"], source="device", src=f["latents"]) for f in fr]
    b = P.Batch(model, fr)
    for fpg, bpg in ((1, 1), (2, 4), (6, 16), (1, 8)):
        for staged in (False, True):  # FP32 caches: both attention forms
            print(f"case CT batch groups {fpg}x{bpg} staged {staged}", flush=True)
            b.set_groups(fpg, bpg)
            b.set_attention(staged)
            b.run()
            b.check()
            for k in range(len(fr)):
                _same(b.outputs(k), ref[k], f"CT batch {fpg}x{bpg} staged {staged} frame {k}")
    b.capture()
    for rep in range(2):
        b.run()
        b.check()
        for k in range(len(fr)):
            _same(b.outputs(k), ref[k], f"CT batch graph replay {rep} frame {k}")


def test_ct_batch_1080p_equals_encode(P):
    cfg = synth.FULL_CT
    Wt = synth.model_weights(cfg, 26)
    model = P.Model(cfg, Wt)
    fr = _frames(cfg, [(68, 120, 0), (68, 120, 2)], 310)
    ref = [P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"]) for f in fr]
    b = P.Batch(model, fr)
    # the groupings of the benchmark's 32-frame batch (two frames per group of
    # 16 blocks, LDS-staged attention) and of one frame per 8 blocks
    for fpg, bpg, staged in ((2, 16, True), (1, 8, False)):
        print(f"case CT batch 1080p I + P groups {fpg}x{bpg} staged {staged}", flush=True)
        b.set_groups(fpg, bpg)
        b.set_attention(staged)
        b.run()
        b.check()
        for k in range(len(fr)):
            _same(b.outputs(k), ref[k], f"CT batch 1080p {fpg}x{bpg} frame {k}")


def test_unbuilt_ct_paths_are_refused(P):
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 24)
    model = P.Model(cfg, Wt)
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(8, 8, 0), 96)
    with pytest.raises(P.PswaError) as e:
        P.Batch(P.Model(cfg, Wt, "bf16"), [{"latents": y, "hyper": z, "prev": None}])
    assert "FP32 models only" in str(e.value)
    with pytest.raises(P.PswaError) as e:
        P.pswa_decode_begin(model, 8, 8, z, source="bitstream", src=b"\x00" * 16)
    assert e.value.name == "E_UNSUPPORTED"
    with pytest.raises(P.PswaError):
        P.Trainer(cfg, Wt, max_crops=1, H=8, W=8)
