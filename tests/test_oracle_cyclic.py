"""Pins of the oracle's cyclic schedule (the paper's repeating s x s mask,
Sec. 3.2 / Fig. 2): step = (i + j) mod s, full window, the accumulator sees
strictly earlier steps and the layers steps up to the query's own.

* parallel form == dense fully masked model (tests/dense_ref.py) for I and P;
* parallel form == step-by-step decoding (every step decoded at once);
* an order that splits a step is rejected (same-step positions must be
  predicted together), and so is raster order;
* perturbing the latent at p leaves every prediction of steps <= step(p)
  bit-identical (the accumulator reads decoded latents only);
* Fig. 2b: 5 x 5 window, s = 4, a step-3 target sees 12 past, 6 same-step
  and 6 future cells; the frame is decoded in exactly s steps.
"""
import numpy as np
import pytest

import synth
from oracle import model as om

from dense_ref import dense_forward

CFG = synth.ModelCfg(L=2, d=32, heads=2, window=5, mlp_ratio=2, C=8, Ch=4, cycle=4)


@pytest.mark.parametrize("n_prev", [0, 2])
def test_cyclic_parallel_equals_dense(n_prev):
    Wt = synth.model_weights(CFG, 21)
    y, z, prev = synth.frame_inputs(CFG, synth.FrameCfg(7, 9, n_prev), 60 + n_prev)
    o = om.forward(CFG, Wt, y, z, prev)
    ref = dense_forward(CFG, Wt, y, z, prev)
    assert np.allclose(o["mu"], ref["mu"], rtol=0, atol=1e-11)
    assert np.allclose(o["sigma"], ref["sigma"], rtol=1e-11, atol=0)


@pytest.mark.parametrize("n_prev", [0, 2])
def test_cyclic_parallel_equals_step_decoding(n_prev):
    Wt = synth.model_weights(CFG, 22)
    H, W = 8, 11
    y, z, prev = synth.frame_inputs(CFG, synth.FrameCfg(H, W, n_prev), 70 + n_prev)
    groups = om.schedule_groups(CFG, H, W)
    assert len(groups) == CFG.cycle
    assert sum(len(g) for g in groups) == H * W
    par = om.forward(CFG, Wt, y, z, prev)
    seq = om.forward_sequential(CFG, Wt, y, z, groups, prev)
    for k in ("mu", "sigma"):
        assert np.allclose(par[k], seq[k], rtol=0, atol=1e-12)


def test_cyclic_rejects_split_steps_and_raster():
    Wt = synth.model_weights(CFG, 23)
    y, z, _ = synth.frame_inputs(CFG, synth.FrameCfg(6, 6), 80)
    groups = om.schedule_groups(CFG, 6, 6)
    split = [groups[0][:3], groups[0][3:]] + groups[1:]
    with pytest.raises(AssertionError):
        om.forward_sequential(CFG, Wt, y, z, split)
    with pytest.raises(AssertionError):
        om.forward_sequential(CFG, Wt, y, z, om.raster_order(6, 6))


def test_cyclic_causality():
    Wt = synth.model_weights(CFG, 24)
    H, W = 9, 10
    y, z, _ = synth.frame_inputs(CFG, synth.FrameCfg(H, W), 81)
    base = om.forward(CFG, Wt, y, z)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    st = om.cyclic_step(ii, jj, CFG.cycle)
    for (pi, pj) in [(4, 4), (0, 0), (8, 9), (3, 7)]:
        y2 = y.copy()
        y2[pi, pj] += 5
        o = om.forward(CFG, Wt, y2, z)
        same = st <= st[pi, pj]
        assert np.array_equal(o["mu"][same], base["mu"][same])
        assert np.array_equal(o["sigma"][same], base["sigma"][same])
    # step-0 positions never see a latent: any change keeps them
    o = om.forward(CFG, Wt, y + 3, z)
    assert np.array_equal(o["mu"][st == 0], base["mu"][st == 0])


def test_fig2b_counts_with_cyclic_predicate():
    cfg = synth.ModelCfg(L=1, d=32, heads=2, window=5, mlp_ratio=2, C=4, Ch=4, cycle=4)
    r, s = cfg.r, cfg.cycle
    i, j = 10, 12          # (i + j) mod 4 = 2: the figure's step 3
    sp = om.schedule_step(cfg, i, j)
    assert sp == 2
    past = same = future = 0
    for a, b in om.full_window(r):
        if (a, b) == (0, 0):
            continue
        sq = om.schedule_step(cfg, i + a, j + b)
        past += sq < sp
        same += sq == sp
        future += sq > sp
    assert (past, same, future) == (12, 6, 6)
    assert om.acc_slots(cfg) == om.full_window(r) and len(om.layer_slots(cfg)) == (2 * r + 1) ** 2
    assert synth.bias_sizes(cfg) == (25, 25, 50)
