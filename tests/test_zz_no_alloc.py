"""GPU test of the encode entry point that allocates nothing
(pswa_encode_params_noalloc, the library's static scratch as workspace),
through the C ABI: its outputs equal pswa_encode_params' bit for bit, on two
calls in a row with the second on a smaller frame (the scratch keeps the
first call's contents), and a frame whose workspace exceeds the scratch is
refused before any device work."""
import pytest

import synth

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
    assert a["total_bits"] == b["total_bits"], label


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_encode_equals_encode(P, prec):
    cfg = synth.FULL
    model = P.make_model(cfg, synth.model_weights(cfg, 11), prec)
    for k, (H, W, npv) in enumerate([(34, 60, 2), (15, 20, 0)]):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), 600 + k)
        print(f"case noalloc {prec} call {k}: {H}x{W} P={npv}", flush=True)
        ref = P.pswa_encode_params(model, y, z, prev)
        got = P.pswa_encode_params_noalloc(model, y, z, prev)
        _same(got, ref, f"{prec} call {k} {H}x{W}")


def test_noalloc_rejects_frames_beyond_the_scratch(P):
    cfg = synth.FULL
    model = P.Model(cfg, synth.model_weights(cfg, 11))
    import ctypes as C
    fd = P.frame_desc(68, 120, 2)
    need = P.lib().pswa_encode_workspace_bytes(model.handle, C.byref(fd))
    assert need > P.lib().pswa_noalloc_scratch_bytes()
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(68, 120, 2), 610)
    with pytest.raises(P.PswaError) as e:
        P.pswa_encode_params_noalloc(model, y, z, prev)
    assert e.value.name == "E_UNSUPPORTED"
