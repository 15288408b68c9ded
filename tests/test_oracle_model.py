"""Pins of the FP64 oracle's context model (CPU only).

Each test fixes the oracle against something other than itself: closed
forms of the schedule, brute-force levelisation of the dependency graph,
the paper's printed mask (Fig. 2), a dense fully-masked re-statement built
on torch's own attention/linear/RMSNorm routines, order invariance, and
special cases that reduce to a textbook result.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import model as om
from tests.dense_ref import dense_forward

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = synth.ModelCfg(L=2, d=32, heads=4, window=5, mlp_ratio=4, C=8, Ch=6)
SMALL9 = synth.ModelCfg(L=1, d=16, heads=2, window=9, mlp_ratio=2, C=4, Ch=3)


def small_inputs(cfg, H, W, seed, p_frame=False):
    f = synth.FrameCfg(H, W, 2 if p_frame else 0)
    return synth.frame_inputs(cfg, f, seed)


# ----------------------------------------------------------------- schedule

@pytest.mark.parametrize("H,W,k", [(16, 16, 5), (68, 120, 9), (135, 240, 9),
                                   (15, 20, 9), (34, 60, 9), (45, 80, 9),
                                   (1, 1, 5), (1, 7, 9), (7, 1, 9), (3, 2, 5)])
def test_schedule_partitions_and_is_causal(H, W, k):
    r = (k - 1) // 2
    s = om.wavefront_slope(r)
    diags = om.diagonals(H, W, s)
    assert len(diags) == om.num_steps(H, W, s) == (W - 1) + s * (H - 1) + 1
    step = np.full((H, W), -1)
    for t, dg in enumerate(diags):
        for i, j in dg:
            assert step[i, j] == -1
            step[i, j] = t
            assert t == j + s * i
    assert (step >= 0).all()
    # every causal neighbour is on an earlier diagonal; every other cell of
    # W(p) on the same diagonal is p itself.
    for i in range(H):
        for j in range(W):
            for a, b in om.causal_window(r):
                if 0 <= i + a < H and 0 <= j + b < W:
                    assert step[i + a, j + b] < step[i, j]


@pytest.mark.parametrize("H,W,k", [(6, 9, 5), (5, 14, 9), (9, 9, 3)])
def test_schedule_is_asap_levelisation(H, W, k):
    """Brute force: the earliest step at which each position can be decoded
    (longest dependency path through W-(p)) equals t = j + s*i."""
    r = (k - 1) // 2
    level = np.zeros((H, W), dtype=int)
    # positions in raster order are a topological order of W-(p)
    for i in range(H):
        for j in range(W):
            deps = [level[i + a, j + b] + 1 for a, b in om.causal_window(r)
                    if 0 <= i + a < H and 0 <= j + b < W]
            level[i, j] = max(deps, default=0)
    s = om.wavefront_slope(r)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    assert (level == om.step_index(ii, jj, s)).all()


def test_slope_is_minimal():
    for r in (1, 2, 4):
        s = om.wavefront_slope(r) - 1
        bad = [(a, b) for a, b in om.causal_window(r)
               if om.step_index(a, b, s) >= 0]
        assert bad, "a slope below r + 1 must break causality"


def test_window_sizes():
    for r in (1, 2, 4):
        assert len(om.causal_window(r)) == 2 * r * (r + 1)
        assert len(set(om.causal_window(r))) == 2 * r * (r + 1)
        assert om.layer_window(r)[-1] == (0, 0)
        assert len(om.temporal_window(r)) == 2 * (2 * r + 1) ** 2


def test_cyclic_mask_matches_fig2a():
    """Fig. 2a prints the 4x4 repeating mask (values = step + 1)."""
    gold = np.loadtxt(os.path.join(GOLDEN, "fig2a_cyclic_mask.txt"), dtype=int)
    ii, jj = np.meshgrid(np.arange(-2, 6), np.arange(-2, 6), indexing="ij")
    assert (om.cyclic_step(ii, jj, 4) + 1 == gold).all()


def test_cyclic_mask_fig2b_counts():
    """Fig. 2b: 5x5 window around target (1, 1) (printed value 3): the
    accumulator sees the earlier-step cells, same-step cells are visible to
    spatial self-attention only, later-step cells are masked."""
    t0 = om.cyclic_step(1, 1)
    past = same = future = 0
    for i in range(-1, 4):
        for j in range(-1, 4):
            if (i, j) == (1, 1):
                continue
            t = om.cyclic_step(i, j)
            past += t < t0
            same += t == t0
            future += t > t0
    assert (past, same, future) == (12, 6, 6)
    # every s-th diagonal shares a step: s steps at any resolution (Sec. 2)
    ii, jj = np.meshgrid(np.arange(40), np.arange(57), indexing="ij")
    assert len(np.unique(om.cyclic_step(ii, jj))) == 4


# ---------------------------------------------------------- dense brute force

@pytest.mark.parametrize("cfg,H,W,seed", [(SMALL, 5, 6, 3), (SMALL, 4, 4, 4),
                                          (SMALL9, 6, 11, 5),
                                          (synth.TINY, 6, 7, 6)])
def test_windowed_equals_dense_masked(cfg, H, W, seed):
    y, z, _ = small_inputs(cfg, H, W, seed)
    Wt = synth.model_weights(cfg, seed + 100)
    o = om.forward(cfg, Wt, y, z)
    ref = dense_forward(cfg, Wt, y, z)
    np.testing.assert_allclose(o["mu"], ref["mu"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(o["sigma"], ref["sigma"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("cfg,H,W,seed", [(SMALL, 5, 6, 7), (SMALL9, 5, 10, 8)])
def test_windowed_equals_dense_masked_pframe(cfg, H, W, seed):
    y, z, prev = small_inputs(cfg, H, W, seed, p_frame=True)
    Wt = synth.model_weights(cfg, seed + 100)
    o = om.forward(cfg, Wt, y, z, prev)
    ref = dense_forward(cfg, Wt, y, z, prev)
    np.testing.assert_allclose(o["mu"], ref["mu"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(o["sigma"], ref["sigma"], rtol=1e-12, atol=0)


# ---------------------------------------------------------- order invariance

def _close(a, b):
    for k in ("mu", "sigma"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("p_frame", [False, True])
def test_order_invariance_tiny(p_frame):
    cfg = synth.TINY
    y, z, prev = small_inputs(cfg, 16, 16, 0, p_frame)
    Wt = synth.model_weights(cfg, 1)
    par = om.forward(cfg, Wt, y, z, prev)
    s = om.wavefront_slope(cfg.r)
    _close(par, om.forward_sequential(cfg, Wt, y, z, om.wavefront_order(16, 16, s), prev))
    _close(par, om.forward_sequential(cfg, Wt, y, z, om.raster_order(16, 16), prev))


def test_order_invariance_random_topological():
    cfg = SMALL
    y, z, _ = small_inputs(cfg, 7, 9, 11)
    Wt = synth.model_weights(cfg, 12)
    par = om.forward(cfg, Wt, y, z)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(20):
        order = om.random_topological_order(7, 9, cfg.r, rng)
        _close(par, om.forward_sequential(cfg, Wt, y, z, order))


def test_sequential_rejects_non_causal_order():
    cfg = SMALL
    y, z, _ = small_inputs(cfg, 4, 4, 2)
    Wt = synth.model_weights(cfg, 3)
    order = list(reversed(om.raster_order(4, 4)))
    with pytest.raises(AssertionError):
        om.forward_sequential(cfg, Wt, y, z, order)


def test_causality_perturbation():
    """Changing y at p leaves every prediction on diagonals <= t(p) intact
    and changes some later one."""
    cfg = SMALL9
    H, W = 7, 12
    y, z, _ = small_inputs(cfg, H, W, 21)
    Wt = synth.model_weights(cfg, 22)
    base = om.forward(cfg, Wt, y, z)
    s = om.wavefront_slope(cfg.r)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for (pi, pj) in [(3, 5), (0, 0), (6, 11), (2, 11)]:
        y2 = y.copy()
        y2[pi, pj] += 7
        o = om.forward(cfg, Wt, y2, z)
        same = om.step_index(ii, jj, s) <= om.step_index(pi, pj, s)
        assert np.array_equal(o["mu"][same], base["mu"][same])
        assert np.array_equal(o["sigma"][same], base["sigma"][same])
        if (pi, pj) != (6, 11):
            assert not np.allclose(o["mu"][~same], base["mu"][~same])


# ------------------------------------------------------------ special cases

def test_rmsnorm_closed_form():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 37)) * 3
    u = om.rmsnorm(x, np.ones(37))
    ms = np.mean(x * x, axis=-1)
    np.testing.assert_allclose(np.sqrt(np.mean(u * u, -1)),
                               (1 + om.EPS / ms) ** -0.5, rtol=1e-14)


def test_hyper_token_reduces_to_nearest_upsampling():
    cfg = synth.ModelCfg(L=1, d=6, heads=2, window=3, mlp_ratio=1, C=2, Ch=6)
    Wt = synth.model_weights(cfg, 0)
    Wt["hyper.W"] = np.eye(6, dtype=np.float32)
    Wt["hyper.P4"] = np.zeros((16, 6), np.float32)
    z = synth.hyper_frame(3, 4, 6, 1)
    h = om.hyper_tokens(Wt, z, 10, 13)
    up = np.kron(z, np.ones((4, 4, 1)))[:10, :13]
    np.testing.assert_array_equal(h, up)
    # one-hot sub-position embedding: token (i, j) picks row 4(i%4)+(j%4)
    Wt["hyper.W"] = np.zeros((6, 6), np.float32)
    Wt["hyper.P4"] = np.arange(96, dtype=np.float32).reshape(16, 6)
    h = om.hyper_tokens(Wt, z, 10, 13)
    assert h[5, 7, 0] == 6 * (4 * 1 + 3)


def test_zero_blocks_pass_residual_and_head_offsets():
    cfg = SMALL
    y, z, _ = small_inputs(cfg, 5, 5, 31)
    Wt = synth.model_weights(cfg, 32)
    for l in range(cfg.L):
        for n in ("Wqkv", "Wo", "Wgate", "Wup", "Wdown"):
            Wt[f"layer{l}.{n}"] = np.zeros_like(Wt[f"layer{l}.{n}"])
    o = om.forward(cfg, Wt, y, z, keep=True)
    np.testing.assert_array_equal(o[f"x{cfg.L}"], o["x0"])
    Wt["head.W2"] = np.zeros_like(Wt["head.W2"])
    Wt["head.bmu"] = np.linspace(-2, 2, cfg.C).astype(np.float32)
    Wt["head.bsig"] = np.linspace(-5, 6, cfg.C).astype(np.float32)
    o = om.forward(cfg, Wt, y, z)
    np.testing.assert_array_equal(o["mu"], np.broadcast_to(
        Wt["head.bmu"].astype(np.float64), o["mu"].shape))
    lsig = np.clip(Wt["head.bsig"].astype(np.float64), math.log(0.11), math.log(64))
    np.testing.assert_array_equal(o["sigma"], np.broadcast_to(np.exp(lsig), o["sigma"].shape))


def test_accumulator_first_position_is_null_value():
    """(0, 0) has no decoded neighbour: it attends to the null slot only and
    gets h + W_o^a v_null."""
    cfg = SMALL
    y, z, _ = small_inputs(cfg, 4, 5, 41)
    Wt = synth.model_weights(cfg, 42)
    o = om.forward(cfg, Wt, y, z, keep=True)
    vnull = Wt["acc.vnull"].astype(np.float64)
    exp = o["h"][0, 0] + Wt["acc.Wo"].astype(np.float64) @ vnull
    np.testing.assert_allclose(o["x0"][0, 0], exp, rtol=1e-13, atol=1e-13)


def test_attention_single_key_and_equal_logits():
    rng = np.random.default_rng(3)
    H, W, d, heads = 2, 3, 8, 2
    q = rng.standard_normal((H, W, d))
    V1 = rng.standard_normal((H, W, d))
    K1 = rng.standard_normal((H, W, d))
    ok = np.ones((H, W), bool)
    out = om._windowed_attention(q, [(K1, V1, ok, np.zeros(heads))], heads)
    np.testing.assert_allclose(out, V1, rtol=1e-14)
    # zero keys and zero bias: equal logits -> mean of values
    Vs = [rng.standard_normal((H, W, d)) for _ in range(3)]
    slots = [(np.zeros((H, W, d)), V, ok, np.zeros(heads)) for V in Vs]
    out = om._windowed_attention(q, slots, heads)
    np.testing.assert_allclose(out, sum(Vs) / 3, rtol=1e-13, atol=1e-14)
    # a masked slot contributes nothing, whatever its logit
    bad = (q * 100, np.full((H, W, d), 1e9), ~ok, np.zeros(heads))
    out2 = om._windowed_attention(q, slots + [bad], heads)
    np.testing.assert_allclose(out2, out, rtol=1e-14)
