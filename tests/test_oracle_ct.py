"""Pins of the oracle's Channel Transformer and grouped heads (CPU only).

* Decoding the channel groups one after the other, each from the symbols
  of the earlier groups only (the later ones hidden), equals the definition
  form that sees every symbol: the mask and the shift make group g read
  groups 0 .. g-1 alone.
* Causality by perturbation: changing the symbols of group g at a position
  leaves that position's groups 0 .. g unchanged and changes a later one;
  group 0 depends on no symbol of its own position.
* The masked blocks are dead: random weights in the masked blocks of every
  mixing map and of the latent input projection change nothing; the
  diagonal blocks are live (group g reads groups 0 .. g, itself included).
* With one group, an identity input projection and blocks that add nothing,
  the model reduces to the plain head on the spatial output (to within the
  RMSNorm epsilon of the extra normalization).
* With every Channel Transformer weight zero the heads output the offsets:
  mean = b_mu, scale = exp(clamp(b_sigma)).
"""
import dataclasses
import math

import numpy as np
import pytest

import synth
from oracle import model as om


def _frame(cfg, H, W, n_prev, seed):
    return synth.frame_inputs(cfg, synth.FrameCfg(H, W, n_prev), seed)


@pytest.mark.parametrize("n_prev", [0, 2])
def test_group_by_group_decoding_equals_definition(n_prev):
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 2)
    y, z, prev = _frame(cfg, 9, 11, n_prev, 30 + n_prev)
    a = om.forward(cfg, Wt, y, z, prev)
    b = om.forward_sequential(cfg, Wt, y, z, om.schedule_groups(cfg, 9, 11), prev)
    for k in ("mu", "sigma", "lsig"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=1e-12)


def test_groups_read_only_earlier_groups_of_their_position():
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 3)
    y, z, _ = _frame(cfg, 8, 10, 0, 40)
    N, Cg = cfg.ch_groups, cfg.C // cfg.ch_groups
    base = om.forward(cfg, Wt, y, z)
    i, j = 5, 6
    for g in range(N):
        y2 = y.copy()
        y2[i, j, g * Cg:(g + 1) * Cg] += 3
        o = om.forward(cfg, Wt, y2, z)
        # groups 0 .. g of the position do not move
        assert np.array_equal(o["mu"][i, j, :(g + 1) * Cg], base["mu"][i, j, :(g + 1) * Cg])
        assert np.array_equal(o["lsig"][i, j, :(g + 1) * Cg], base["lsig"][i, j, :(g + 1) * Cg])
        if g < N - 1:  # a later group does
            assert not np.allclose(o["mu"][i, j, (g + 1) * Cg:], base["mu"][i, j, (g + 1) * Cg:])
    # group 0 reads none of its position's symbols
    y3 = y.copy()
    y3[i, j] = -y3[i, j] + 7
    o = om.forward(cfg, Wt, y3, z)
    assert np.array_equal(o["mu"][i, j, :Cg], base["mu"][i, j, :Cg])


def test_masked_blocks_are_dead():
    cfg = synth.TINY_CT
    N, dc, C = cfg.ch_groups, cfg.ch_d, cfg.C
    Wt = synth.model_weights(cfg, 4)
    y, z, _ = _frame(cfg, 7, 9, 0, 50)
    rng = np.random.default_rng(5)
    Wm = {k: v.copy() for k, v in Wt.items()}
    dead_m = 1 - om.group_mask(dc, dc, N)
    dead_y = 1 - om.group_mask(dc, C, N)
    for b in range(cfg.ch_L):
        k = f"ct{b}.M"
        Wm[k] = (Wt[k] + dead_m * rng.standard_normal((dc, dc))).astype(np.float32)
    Wm["ct.Wy"] = (Wt["ct.Wy"] + dead_y * rng.standard_normal((dc, C))).astype(np.float32)
    a = om.forward(cfg, Wt, y, z)
    b = om.forward(cfg, Wm, y, z)
    for k in ("mu", "lsig"):
        assert np.array_equal(a[k], b[k])
    # the diagonal blocks are live: group g mixes its own slice too
    Wd = {k: v.copy() for k, v in Wt.items()}
    eye_blocks = om.group_mask(dc, dc, N) * om.group_mask(dc, dc, N).T
    Wd["ct0.M"] = (Wt["ct0.M"] * (1 - eye_blocks)).astype(np.float32)
    c = om.forward(cfg, Wd, y, z)
    assert not np.allclose(c["mu"], a["mu"])


def test_one_group_reduces_to_the_plain_head():
    base = synth.TINY
    cfg1 = dataclasses.replace(base, ch_groups=1, ch_d=base.d, ch_L=1, ch_ratio=1)
    Wp = synth.model_weights(base, 6)
    W1 = {k: v for k, v in Wp.items() if not k.startswith("head.") or k in
          ("head.gmu", "head.bmu", "head.gsig", "head.bsig")}
    d, C = base.d, base.C
    W1.update({
        "ct.gx": np.ones(d, np.float32), "ct.Wx": np.eye(d, dtype=np.float32),
        "ct.gy": np.full(C, 1 / 3, np.float32),
        "ct.Wy": np.random.default_rng(7).standard_normal((d, C)).astype(np.float32),
        "ct0.g1": np.ones(d, np.float32), "ct0.M": np.zeros((d, d), np.float32),
        "ct0.g2": np.ones(d, np.float32),
        "ct0.Wgate": np.ones((1, d, d), np.float32), "ct0.Wup": np.ones((1, d, d), np.float32),
        "ct0.Wdown": np.zeros((1, d, d), np.float32),
        "ctH.g": Wp["head.g"], "ctH.W1": Wp["head.W1"][None], "ctH.W2": Wp["head.W2"][None],
    })
    y, z, _ = _frame(base, 8, 8, 0, 60)
    a = om.forward(base, Wp, y, z)
    b = om.forward(cfg1, W1, y, z)
    np.testing.assert_allclose(b["mu"], a["mu"], rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(b["lsig"], a["lsig"], rtol=1e-4, atol=1e-4)


def test_zero_channel_transformer_outputs_the_offsets():
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 8)
    for k in list(Wt):
        if k.startswith("ct"):
            Wt[k] = np.zeros_like(Wt[k])
    Wt["head.bmu"] = np.linspace(-2, 2, cfg.C).astype(np.float32)
    y, z, _ = _frame(cfg, 5, 6, 0, 70)
    o = om.forward(cfg, Wt, y, z)
    assert np.array_equal(o["mu"], np.broadcast_to(Wt["head.bmu"].astype(np.float64), o["mu"].shape))
    ls = float(np.clip(np.float64(Wt["head.bsig"][0]), om.LN_SIGMA_MIN, om.LN_SIGMA_MAX))
    assert np.allclose(o["sigma"], math.exp(ls), rtol=0, atol=0)


def test_sampled_latents_with_channel_groups_reproduce_the_draw():
    cfg = synth.TINY_CT
    Wt = synth.model_weights(cfg, 9)
    Wt["head.bsig"][:] = np.float32(math.log(0.5))
    z = synth.hyper_frame(3, 3, cfg.Ch, 11)
    noise = np.random.default_rng(12).standard_normal((10, 12, cfg.C))
    y = om.sample_latents(cfg, Wt, z, noise)
    ref = om.forward(cfg, Wt, y, z)
    assert np.abs(y - (ref["mu"] + ref["sigma"] * noise)).max() <= 0.5 + 1e-9
