"""GPU tests of the BF16 and FP8 (e4m3fn) projection forms.

Within a precision, encode, per-diagonal decode and persistent batch decode
run the same row-invariant MFMA tiles, so they must be bit-identical. Against
the FP64 oracle the forms are held to their bits-overhead targets on the
1080p-shaped P-frame (0.5 % for BF16, 1 % for FP8) and their mean/scale
errors are reported.
"""
import numpy as np
import pytest

import synth
from oracle import entropy as oe
from oracle import model as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "bits", "center", "index")
BITS_TARGET = {"bf16": 0.005, "fp8": 0.01}


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


def _report(out, ref, y, label):
    mu = _np(out["mean"]).astype(np.float64)
    sg = _np(out["scale"]).astype(np.float64)
    emu = np.abs(mu - ref["mu"]) / np.maximum(np.abs(ref["mu"]), 1)
    esg = np.abs(sg - ref["sigma"]) / ref["sigma"]
    b_ref = oe.bits(y, ref["mu"], ref["sigma"]).sum()
    b = oe.bits(y, mu, sg).sum()
    ov = (b - b_ref) / b_ref
    print(f"[{label}] mean err max {emu.max():.3e} mean {emu.mean():.3e}; scale err max "
          f"{esg.max():.3e} mean {esg.mean():.3e}; bits {b:.0f} vs fp64 {b_ref:.0f} "
          f"overhead {100 * ov:+.4f} %", flush=True)
    return ov, emu, esg


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_tiny_precision_forms_agree(P, prec):
    cfg = synth.TINY
    Wt = synth.model_weights(cfg, 1)
    model = P.Model(cfg, Wt, prec)
    fr = []
    for k, (H, W, npv) in enumerate([(16, 16, 0), (13, 21, 2), (5, 3, 0)]):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), 40 + k)
        fr.append({"latents": y, "hyper": z, "prev": prev})
        print(f"case tiny {prec} {H}x{W} P={npv}", flush=True)
        enc = P.pswa_encode_params(model, y, z, prev)
        dec = P.decode_frame(model, H, W, z, prev=prev, source="device", src=y)
        _same(enc, dec, f"{prec} {H}x{W}")
        ref = om.forward(cfg, Wt, y, z, prev)
        ov, emu, esg = _report(enc, ref, y, f"tiny {prec} {H}x{W}")
        assert emu.max() < (0.05 if prec == "bf16" else 0.2)
        fr[-1]["dec"] = dec
    b = P.Batch(model, fr)
    b.run()
    b.check()
    for k, f in enumerate(fr):
        _same(b.outputs(k), f["dec"], f"batch {prec} frame {k}")


@pytest.fixture(scope="module")
def pframe():
    cfg = synth.FULL
    Wt = synth.model_weights(cfg, synth.CONFIG_SEEDS["1080p_P"][1])
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(68, 120, 2), synth.CONFIG_SEEDS["1080p_P"][0])
    ref = om.forward(cfg, Wt, y, z, prev)
    return cfg, Wt, y, z, prev, ref


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_1080p_pframe_precision_bits_overhead(P, pframe, prec):
    cfg, Wt, y, z, prev, ref = pframe
    print(f"case 1080p P {prec}", flush=True)
    model = P.Model(cfg, Wt, prec)
    enc = P.pswa_encode_params(model, y, z, prev)
    ov, emu, esg = _report(enc, ref, y, f"1080p-P {prec}")
    assert ov <= BITS_TARGET[prec]
    dec = P.decode_frame(model, 68, 120, z, prev=prev, source="device", src=y)
    _same(enc, dec, f"1080p {prec}")
