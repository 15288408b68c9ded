"""GPU tests of the persistent multi-frame decode, through the C ABI.

The batch path shares every per-row device function with the per-diagonal
decode, so its outputs must be bit-identical to it (which the parity tests
tie to the FP64 oracle); one case is also checked against the oracle
directly.
"""
import numpy as np
import pytest

import synth
from oracle import model as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "bits", "center", "index", "latents")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_20977_amd import pswa
    return pswa


@pytest.fixture(scope="module")
def tiny(P):
    cfg = synth.TINY
    Wt = synth.model_weights(cfg, 1)
    return cfg, Wt, P.Model(cfg, Wt)


def _frames(cfg, sizes, seed0):
    out = []
    for k, (H, W, npv) in enumerate(sizes):
        y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, npv), seed0 + 7 * k)
        out.append({"latents": y, "hyper": z, "prev": prev})
    return out


def _per_frame(P, model, f):
    y = f["latents"]
    return P.decode_frame(model, y.shape[0], y.shape[1], f["hyper"], prev=f["prev"],
                          source="device", src=y)


def _assert_same(a, b, label):
    for k in KEYS:
        assert torch.equal(a[k], b[k]), f"{label}: {k} differs"
    assert a["total_bits"] == b["total_bits"], label


def test_batch_one_frame_equals_step_decode(P, tiny):
    cfg, Wt, model = tiny
    fr = _frames(cfg, [(16, 16, 0)], 0)
    print("case batch tiny 1 frame", flush=True)
    b = P.Batch(model, fr)
    assert b.T == 61
    b.run()
    b.check()
    _assert_same(b.outputs(0), _per_frame(P, model, fr[0]), "1 frame")


def test_batch_mixed_frames_and_grids(P, tiny):
    cfg, Wt, model = tiny
    sizes = [(7, 9, 0), (16, 16, 2), (5, 13, 0), (12, 4, 2), (1, 1, 0), (3, 30, 2)]
    fr = _frames(cfg, sizes, 100)
    ref = [_per_frame(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    for g in (1, 3, 64, b.max_grid):
        print(f"case batch tiny mixed grid {g}", flush=True)
        b.set_grid(g)
        b.run()
        b.check()
        for k in range(len(fr)):
            _assert_same(b.outputs(k), ref[k], f"grid {g} frame {k}")
    # against the oracle, one P-frame of the batch
    o = b.outputs(1)
    r = om.forward(cfg, Wt, fr[1]["latents"], fr[1]["hyper"], fr[1]["prev"])
    mu = o["mean"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(mu - r["mu"]) / np.maximum(np.abs(r["mu"]), 1)) < 1e-4


def test_batch_repeat_runs_identical(P, tiny):
    cfg, Wt, model = tiny
    fr = _frames(cfg, [(9, 11, 0), (16, 16, 2)], 300)
    b = P.Batch(model, fr)
    b.run()
    first = [b.outputs(k) for k in range(2)]
    for _ in range(3):
        b.run()
        for k in range(2):
            _assert_same(b.outputs(k), first[k], "repeat")


def test_batch_barrier_timeout_reports_abort(P, tiny):
    """Forced from the host: a zero spin bound makes the first barrier wait
    give up; every block must drain and the host must see the abort."""
    cfg, Wt, model = tiny
    fr = _frames(cfg, [(8, 8, 0)], 500)
    b = P.Batch(model, fr, grid=8)
    b.set_spin_limit(0)
    b.run()
    with pytest.raises(P.PswaError) as e:
        b.check()
    assert e.value.name == "E_HIP"
    # the batch recovers with a sane bound
    b.set_spin_limit(1 << 21)
    b.run()
    b.check()
    _assert_same(b.outputs(0), _per_frame(P, model, fr[0]), "after abort")


def test_batch_1080p_mix_equals_step_decode(P):
    cfg = synth.FULL
    Wt = synth.model_weights(cfg, synth.CONFIG_SEEDS["batch"][1])
    model = P.Model(cfg, Wt)
    sizes = [(68, 120, 0), (34, 60, 2), (15, 20, 2), (45, 80, 0)]
    fr = _frames(cfg, sizes, synth.CONFIG_SEEDS["batch"][0])
    print("case batch 1080p mix", flush=True)
    b = P.Batch(model, fr)
    assert b.T == 455
    b.run()
    b.check()
    for k in range(len(fr)):
        _assert_same(b.outputs(k), _per_frame(P, model, fr[k]), f"frame {k}")
