"""GPU tests of the paper's cyclic schedule (step = (i + j) mod s over the
full window; Sec. 3.2, Fig. 2), through the C ABI.

* tiny I- and P-frames: FP32 encode against the FP64 oracle; the s-step
  decode (device symbols and bitstream) and the persistent batch are
  bit-identical to the encode;
* 1080p-shaped frames (6 layers, d = 384, 7 x 7 window, s = 4): FP32 encode
  against the oracle at sampled positions (cone crops), and the BF16 batch
  decode of both an I- and a P-frame bit-identical to its encode with bits
  within 0.5 % of FP32.
"""
import numpy as np
import pytest

import synth
from oracle import model as om

from sampled_ref import oracle_at, sample_positions
from test_gpu_parity import assert_matches_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "bits", "center", "index")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_20977_amd import pswa
    return pswa


def _np(t):
    return t.detach().cpu().numpy()


def _same(a, b, label):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), f"{label}: {k}"


@pytest.mark.parametrize("H,W,n_prev", [(16, 16, 0), (13, 21, 2), (5, 3, 0)])
def test_tiny_cyclic_encode_decode(P, H, W, n_prev):
    cfg = synth.TINY_CYCLIC
    Wt = synth.model_weights(cfg, 2)
    model = P.Model(cfg, Wt)
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, n_prev), 90 + H)
    print(f"case cyclic tiny {H}x{W} P={n_prev}", flush=True)
    enc = P.pswa_encode_params(model, y, z, prev)
    assert_matches_oracle(enc, om.forward(cfg, Wt, y, z, prev), y, f"cyclic {H}x{W}")
    st = P.pswa_decode_begin(model, H, W, z, prev=prev, source="device", src=y)
    assert st.T == cfg.cycle
    st.close()
    dec = P.decode_frame(model, H, W, z, prev=prev, source="device", src=y)
    _same(enc, dec, "device decode")
    assert np.array_equal(_np(dec["latents"]), y)
    data = P.pswa_range_encode(H, W, cfg.C, cfg.window, y, _np(enc["center"]),
                               _np(enc["index"]), cycle=cfg.cycle)
    dec2 = P.decode_frame(model, H, W, z, prev=prev, source="bitstream", src=data)
    _same(enc, dec2, "bitstream decode")
    assert np.array_equal(_np(dec2["latents"]), y)
    b = P.Batch(model, [{"latents": y, "hyper": z, "prev": prev}])
    assert b.T == cfg.cycle
    b.run()
    b.check()
    _same(b.outputs(0), enc, "batch")


@pytest.fixture(scope="module")
def cyc1080():
    cfg = synth.CYCLIC
    dseed, wseed = synth.CONFIG_SEEDS["1080p_cyclic"]
    Wt = synth.model_weights(cfg, wseed)
    frames = []
    for k, n_prev in enumerate((0, 2)):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(68, 120, n_prev), dseed + k)
        frames.append({"latents": y, "hyper": z, "prev": prev})
    return cfg, Wt, frames


def test_1080p_cyclic_fp32_matches_oracle_at_samples(P, cyc1080):
    cfg, Wt, frames = cyc1080
    model = P.Model(cfg, Wt)
    for k, f in enumerate(frames):
        print(f"case cyclic 1080p fp32 frame {k}", flush=True)
        o = P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"])
        mu = _np(o["mean"]).astype(np.float64)
        sg = _np(o["scale"]).astype(np.float64)
        ref = oracle_at(cfg, Wt, f["latents"], f["hyper"], f["prev"],
                        sample_positions(68, 120, 8, 200 + k))
        for (i, j), r in ref.items():
            emu = np.abs(mu[i, j] - r["mu"]) / np.maximum(np.abs(r["mu"]), 1)
            esg = np.abs(sg[i, j] - r["sigma"]) / r["sigma"]
            assert emu.max() < 1e-4 and esg.max() < 1e-4, (k, i, j, emu.max(), esg.max())


def test_1080p_cyclic_bf16_batch(P, cyc1080):
    cfg, Wt, frames = cyc1080
    m32 = P.Model(cfg, Wt)
    model = P.Model(cfg, Wt, "bf16")
    enc = [P.pswa_encode_params(model, f["latents"], f["hyper"], f["prev"]) for f in frames]
    b = P.Batch(model, frames)
    print(f"case cyclic 1080p bf16 batch T={b.T} groups {b.groups}", flush=True)
    assert b.T == cfg.cycle
    b.run()
    b.check()
    for k, f in enumerate(frames):
        _same(b.outputs(k), enc[k], f"batch frame {k}")
        ref = P.pswa_encode_params(m32, f["latents"], f["hyper"], f["prev"])["total_bits"]
        ov = enc[k]["total_bits"] / ref - 1.0
        print(f"cyclic 1080p frame {k} bf16 bits {enc[k]['total_bits']:.0f} vs fp32 {ref:.0f} "
              f"({100 * ov:+.4f} %)", flush=True)
        assert ov <= 0.005
