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
    b = P.Batch(model, fr)
    assert b.T == 455
    ref = [_per_frame(P, model, f) for f in fr]
    for staged in (False, True):  # FP32 caches: both attention forms
        print(f"case batch 1080p mix staged={staged}", flush=True)
        b.set_attention(staged)
        b.run()
        b.check()
        for k in range(len(fr)):
            _assert_same(b.outputs(k), ref[k], f"staged={staged} frame {k}")


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_batch_row_tile_and_autotune_keep_outputs(P, prec, tmp_path):
    """The row tile and grid only move rows between tiles and blocks: every
    (grid, row tile) choice, the autotuner's included, gives the same bits."""
    cfg = synth.TINY
    model = P.make_model(cfg, synth.model_weights(cfg, 1), prec,
                         synth.calibration_frames(cfg, 16, 16))
    fr = _frames(cfg, [(16, 16, 0), (13, 21, 2), (4, 37, 0)], 700)
    b = P.Batch(model, fr)
    b.run()
    ref = [b.outputs(k) for k in range(len(fr))]
    for k in range(len(fr)):
        _assert_same(ref[k], _per_frame(P, model, fr[k]), f"{prec} frame {k}")
    for r in (16, 32):
        for g in (5, 64):
            print(f"case {prec} rtile {r} grid {g}", flush=True)
            b.set_rtile(r)
            b.set_grid(g)
            b.run()
            b.check()
            for k in range(len(fr)):
                _assert_same(b.outputs(k), ref[k], f"{prec} rtile {r} grid {g} frame {k}")
    cache = str(tmp_path / "tune.jsonl")
    f1, g1, r1, ms1 = b.autotune(cache, reps=2)
    assert 1 <= f1 <= len(fr) and r1 in (16, 32) and ms1 > 0
    ng = -(-len(fr) // f1)
    assert 1 <= ng * g1 <= b.max_grid
    assert b.groups == (f1, g1, ng) and b.rtile == r1
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and f'"blocks_per_group": {g1}' in lines[0]
    b.set_grid(1)
    f2, g2, r2, ms2 = b.autotune(cache, reps=2)          # answered from the cache
    assert (f2, g2, r2) == (f1, g1, r1) and len(open(cache).read().splitlines()) == 1
    b.run()
    b.check()
    for k in range(len(fr)):
        _assert_same(b.outputs(k), ref[k], f"{prec} autotuned frame {k}")


def test_batch_groupings_keep_outputs(P, tiny):
    """Frames split over groups with their own blocks and barriers decode
    exactly as one group does."""
    cfg, Wt, model = tiny
    sizes = [(7, 9, 0), (16, 16, 2), (5, 13, 0), (12, 4, 2), (1, 1, 0), (3, 30, 2), (9, 9, 0)]
    fr = _frames(cfg, sizes, 1200)
    ref = [_per_frame(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    for fpg, bpg in ((1, 1), (1, 4), (2, 8), (3, 2), (4, 16), (7, 5)):
        print(f"case grouping {fpg} frames x {bpg} blocks", flush=True)
        b.set_groups(fpg, bpg)
        ng = -(-len(fr) // fpg)
        assert b.groups == (fpg, bpg, ng) and b.grid == ng * bpg
        b.run()
        b.check()
        for k in range(len(fr)):
            _assert_same(b.outputs(k), ref[k], f"groups {fpg}x{bpg} frame {k}")
    with pytest.raises(P.PswaError):
        b.set_groups(1, b.max_grid)          # 7 groups of max_grid blocks cannot fit


def test_batch_fp32_rejects_short_row_tile(P, tiny):
    cfg, Wt, model = tiny
    b = P.Batch(model, _frames(cfg, [(4, 4, 0)], 800))
    with pytest.raises(P.PswaError):
        b.set_rtile(16)
    with pytest.raises(P.PswaError):
        b.set_rtile(8)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_graph_replays_match_eager(P, prec):
    """A captured run replays bit-identically, several times, with eager work
    in between, and reads the frames' inputs as they are at replay time."""
    cfg = synth.TINY
    model = P.Model(cfg, synth.model_weights(cfg, 1), prec)
    fa = _frames(cfg, [(9, 11, 2), (16, 16, 0)], 900)
    fb = _frames(cfg, [(9, 11, 2)], 950)[0]
    ref_a = [_per_frame(P, model, f) for f in fa]
    ref_b = _per_frame(P, model, fb)
    b = P.Batch(model, fa, grid=24)
    b.run()
    for k in range(2):
        _assert_same(b.outputs(k), ref_a[k], f"{prec} eager frame {k}")
    print(f"case graph capture {prec}", flush=True)
    b.capture()
    for rep in range(3):
        b.run()
        b.check()
        for k in range(2):
            _assert_same(b.outputs(k), ref_a[k], f"{prec} replay {rep} frame {k}")
        # eager work on the same stream between replays
        _assert_same(_per_frame(P, model, fa[1]), ref_a[1], f"{prec} eager between {rep}")
    y, z, pv = b.inputs(0)
    y.copy_(torch.as_tensor(fb["latents"], device=y.device))
    z.copy_(torch.as_tensor(fb["hyper"], device=z.device))
    pv.copy_(torch.as_tensor(fb["prev"], device=pv.device))
    b.run()
    b.check()
    _assert_same(b.outputs(0), ref_b, f"{prec} replay on new inputs")
    _assert_same(b.outputs(1), ref_a[1], f"{prec} replay on new inputs, frame 1")
    b.set_grid(7)                                     # drops the graph: eager again
    b.run()
    b.check()
    _assert_same(b.outputs(0), ref_b, f"{prec} eager after drop")


def test_batch_barrier_forms_agree(P, tiny):
    """Groups on one XCD (one-XCD barrier) and the device-scope barrier
    give the same bits; groups that span XCDs fall back by themselves."""
    cfg, Wt, model = tiny
    fr = _frames(cfg, [(16, 16, 2), (9, 13, 0), (12, 7, 2), (5, 5, 0)], 1500)
    ref = [_per_frame(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    for fpg, bpg in ((1, 4), (1, 8), (2, 16), (4, 64)):
        for on in (True, False):
            print(f"case barrier one_xcd={on} groups {fpg}x{bpg}", flush=True)
            b.set_groups(fpg, bpg)
            b.set_xcd_barrier(on)
            b.run()
            b.check()
            for k in range(len(fr)):
                _assert_same(b.outputs(k), ref[k], f"one_xcd={on} {fpg}x{bpg} frame {k}")


def test_batch_attention_forms_agree(P, tiny):
    """LDS-staged window tiles and per-lane global key loads give the same
    bits, across groupings (tiles cut at frame borders and block runs),
    I- and P-frames, frames narrower than a window, FP32 caches and the BF16
    caches of BF16 and FP8 models; the cyclic schedule refuses the staged
    form."""
    cfg, Wt, model = tiny
    sizes = [(7, 9, 0), (16, 16, 2), (5, 13, 0), (12, 4, 2), (1, 1, 0), (3, 30, 2), (9, 2, 0)]
    fr = _frames(cfg, sizes, 1700)
    ref = [_per_frame(P, model, f) for f in fr]
    b = P.Batch(model, fr)
    for fpg, bpg in ((1, 1), (1, 3), (2, 8), (7, 5), (7, 64)):
        for staged in (True, False):
            print(f"case attention staged={staged} groups {fpg}x{bpg}", flush=True)
            b.set_groups(fpg, bpg)
            b.set_attention(staged)
            assert b.attention_staged == staged
            b.run()
            b.check()
            for k in range(len(fr)):
                _assert_same(b.outputs(k), ref[k], f"staged={staged} {fpg}x{bpg} frame {k}")
    for prec in ("bf16", "fp8"):
        mq = P.make_model(cfg, Wt, prec, fr[:2])
        refq = [_per_frame(P, mq, f) for f in fr]
        bq = P.Batch(mq, fr)
        for fpg, bpg in ((1, 3), (7, 5)):
            for staged in (True, False):
                print(f"case attention {prec} staged={staged} groups {fpg}x{bpg}", flush=True)
                bq.set_groups(fpg, bpg)
                bq.set_attention(staged)
                assert bq.attention_staged == staged
                bq.run()
                bq.check()
                for k in range(len(fr)):
                    _assert_same(bq.outputs(k), refq[k],
                                 f"{prec} staged={staged} {fpg}x{bpg} frame {k}")
    cm = P.Model(synth.TINY_CYCLIC, synth.model_weights(synth.TINY_CYCLIC, 1))
    bc = P.Batch(cm, _frames(synth.TINY_CYCLIC, [(8, 8, 0)], 1800))
    with pytest.raises(P.PswaError):
        bc.set_attention(True)
    assert not bc.attention_staged
