"""GPU tests of the student context model on 4K-shaped latents
(135 x 240 x 192, one I-frame and one P-frame; 2 layers, d = 128, 4 heads of
32, causal 9 x 9 window), through the C ABI.

* FP32 encode against the FP64 oracle at sampled positions (cone crops, see
  tests/sampled_ref.py): mean and scale to 1e-4 relative;
* BF16 and FP8 forms: persistent batch decode of both frames is
  bit-identical to their encode, with bits within 0.5 % / 1 % of FP32;
* per-frame fallback: the student is kept exactly when its bits stay within
  1 % of the full model's on the same frame.
"""
import numpy as np
import pytest

import synth

from sampled_ref import oracle_at, sample_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H, W = 135, 240
KEYS = ("mean", "scale", "bits", "center", "index")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_20977_amd import pswa
    return pswa


@pytest.fixture(scope="module")
def frames():
    seed = synth.CONFIG_SEEDS["4k_student"][0]
    out = []
    for k, n_prev in enumerate((0, 2)):
        y, z, prev = synth.frame_inputs(synth.STUDENT, synth.FrameCfg(H, W, n_prev), seed + k)
        out.append({"latents": y, "hyper": z, "prev": prev})
    return out


@pytest.fixture(scope="module")
def weights():
    return synth.model_weights(synth.STUDENT, 51)


def test_student_fp32_matches_oracle_at_samples(P, frames, weights):
    cfg = synth.STUDENT
    model = P.Model(cfg, weights)
    for k, f in enumerate(frames):
        print(f"case student 4K fp32 frame {k}", flush=True)
        o = P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"])
        mu = o["mean"].cpu().numpy().astype(np.float64)
        sg = o["scale"].cpu().numpy().astype(np.float64)
        pos = sample_positions(H, W, 12, 70 + k)
        ref = oracle_at(cfg, weights, f["latents"], f["hyper"], f["prev"], pos)
        for (i, j), r in ref.items():
            emu = np.abs(mu[i, j] - r["mu"]) / np.maximum(np.abs(r["mu"]), 1)
            esg = np.abs(sg[i, j] - r["sigma"]) / r["sigma"]
            assert emu.max() < 1e-4 and esg.max() < 1e-4, (k, i, j, emu.max(), esg.max())


@pytest.mark.parametrize("prec,bound", [("bf16", 0.005), ("fp8", 0.01)])
def test_student_low_precision_batch_decode(P, frames, weights, prec, bound):
    cfg = synth.STUDENT
    m32 = P.Model(cfg, weights)
    model = P.make_model(cfg, weights, prec, synth.calibration_frames(cfg))
    enc = [P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"]) for f in frames]
    b = P.Batch(model, frames)
    print(f"case student 4K {prec} batch groups {b.groups}", flush=True)
    b.run()
    b.check()
    for k, f in enumerate(frames):
        out = b.outputs(k)
        for key in KEYS:
            assert torch.equal(out[key], enc[k][key]), (prec, k, key)
        ref = P.pswa_encode_params(m32, f["latents"], f["hyper"], f["prev"])["total_bits"]
        ov = enc[k]["total_bits"] / ref - 1.0
        print(f"student 4K frame {k} {prec}: bits {enc[k]['total_bits']:.0f} vs fp32 {ref:.0f} "
              f"({100 * ov:+.4f} %)", flush=True)
        assert ov <= bound


def test_student_fallback_takes_the_full_model(P, frames, weights):
    """A student whose scale offset is moved far from the data's spread
    codes the frames with many more bits than the full model: the rule must
    send those frames to the full model (the branch random-init weights
    never reach)."""
    full = P.Model(synth.FULL, synth.model_weights(synth.FULL, synth.CONFIG_SEEDS["4k_student"][1]))
    bad_w = {k: v.copy() for k, v in weights.items()}
    bad_w["head.bsig"][:] = np.float32(np.log(0.2))   # sigma ~ 0.2 against a spread of ~3
    bad = P.Model(synth.STUDENT, bad_w)
    for k, f in enumerate(frames):
        bs = P.pswa_encode_params(bad, f["latents"], f["hyper"], f["prev"])["total_bits"]
        bf = P.pswa_encode_params(full, f["latents"], f["hyper"], f["prev"])["total_bits"]
        print(f"frame {k}: perturbed student {bs:.0f} bits, full {bf:.0f} bits", flush=True)
        assert bs > 1.01 * bf
        assert not P.pswa_student_accept(bs, bf, 0.01)


def test_student_fallback_rule(P, frames, weights):
    full = P.Model(synth.FULL, synth.model_weights(synth.FULL, synth.CONFIG_SEEDS["4k_student"][1]))
    stud = P.Model(synth.STUDENT, weights)
    for k, f in enumerate(frames):
        bs = P.pswa_encode_params(stud, f["latents"], f["hyper"], f["prev"])["total_bits"]
        bf = P.pswa_encode_params(full, f["latents"], f["hyper"], f["prev"])["total_bits"]
        keep = P.pswa_student_accept(bs, bf, 0.01)
        print(f"frame {k}: student {bs:.0f} bits, full {bf:.0f} bits -> "
              f"{'student' if keep else 'full model'}", flush=True)
        assert keep == (bs <= 1.01 * bf)
