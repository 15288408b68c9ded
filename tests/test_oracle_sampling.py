"""Pins of the oracle's model-sampled latents and of the bits-overhead
metric on them (CPU only).

oracle.model.sample_latents draws y from the model itself in decode order.
Pinned by: the parallel form on the drawn latents reproduces the draw
(y = rint(mu + sigma * noise) at every symbol); causality (noise changed on
later diagonals leaves earlier symbols alone); and the ideal bits match the
entropy of the predicted distributions (the model is the source). The
metric the precision tests use, (bits - bits_FP64) / bits_FP64, is then
shown to reject mean errors of the size FP8 can make and to accept those of
BF16's size.
"""
import math

import numpy as np
import pytest

import synth
from oracle import entropy as oe
from oracle import model as om


@pytest.fixture(scope="module")
def sampled():
    cfg = synth.TINY
    Wt = synth.model_weights(cfg, 3)
    Wt["head.bsig"][:] = np.float32(math.log(0.5))
    H, W = 16, 16
    z = synth.hyper_frame(4, 4, cfg.Ch, 5)
    noise = np.random.default_rng(6).standard_normal((H, W, cfg.C))
    y = om.sample_latents(cfg, Wt, z, noise)
    return cfg, Wt, z, noise, y, om.forward(cfg, Wt, y, z)


def test_draw_is_reproduced_by_the_parallel_form(sampled):
    cfg, Wt, z, noise, y, ref = sampled
    resid = np.abs(y - (ref["mu"] + ref["sigma"] * noise))
    assert resid.max() <= 0.5 + 1e-9


def test_draw_is_causal(sampled):
    cfg, Wt, z, noise, y, _ = sampled
    s = om.wavefront_slope(cfg.r)
    t0 = 20
    ii, jj = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    later = (jj + s * ii) >= t0
    n2 = noise.copy()
    n2[later] = np.random.default_rng(7).standard_normal(n2[later].shape)
    y2 = om.sample_latents(cfg, Wt, z, n2)
    assert np.array_equal(y2[~later], y[~later])
    assert not np.array_equal(y2[later], y[later])


def _entropy_bits(mu, sg):
    """Entropy in bits of the discretized Gaussian of every symbol."""
    ks = np.arange(-12, 13)[None, :] + np.floor(mu).reshape(-1, 1)
    mu1, sg1 = mu.reshape(-1, 1), sg.reshape(-1, 1)
    p = oe.likelihood(ks, mu1, sg1)
    p = np.where(p > 0, p, 1e-300)
    return float(-(p * np.log2(p)).sum())


def test_bits_match_the_entropy_of_the_source(sampled):
    cfg, Wt, z, noise, y, ref = sampled
    bits = oe.bits(y, ref["mu"], ref["sigma"])
    ent = _entropy_bits(ref["mu"], ref["sigma"])
    n = y.size
    # per-symbol bits have a spread of about 1 bit: the mean agrees with the
    # mean entropy to a few standard errors
    assert abs(bits.sum() - ent) / n < 4 * bits.std() / math.sqrt(n)
    assert 0.8 < bits.mean() < 2.0


def test_overhead_metric_rejects_fp8_sized_mean_errors(sampled):
    cfg, Wt, z, noise, y, ref = sampled
    b0 = oe.bits(y, ref["mu"], ref["sigma"]).sum()

    def overhead(delta):
        mu = ref["mu"] + delta * np.random.default_rng(11).standard_normal(ref["mu"].shape)
        return (oe.bits(y, mu, ref["sigma"]).sum() - b0) / b0
    assert overhead(0.0) == 0.0
    assert overhead(0.016) < 0.005   # BF16-sized mean errors pass the 0.5 % bound
    assert overhead(0.1) > 0.01      # FP8-sized (up to 0.2) ones fail the 1 % bound
    assert overhead(0.2) > 0.05
