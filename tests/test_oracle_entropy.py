"""Pins of the oracle's likelihood, bits and integer CDF tables (CPU only)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import entropy as oe


def test_likelihood_closed_form_at_mean():
    """P(y = mu | sigma = 1) = erf(1 / (2 sqrt 2)) = 0.3829249225...,
    i.e. 1.384867 bits."""
    p = oe.likelihood(np.array([5]), 5.0, 1.0)[0]
    assert abs(p - math.erf(1 / (2 * math.sqrt(2)))) < 1e-15
    assert abs(p - 0.3829249225) < 1e-10
    assert abs(oe.bits(np.array([5]), 5.0, 1.0)[0] - 1.384867) < 5e-7


def test_likelihood_matches_textbook_cdf_difference():
    """Against scipy's normal CDF where the direct difference is accurate."""
    rng = np.random.default_rng(0)
    mu = rng.uniform(-5, 5, 2000)
    sig = np.exp(rng.uniform(math.log(0.11), math.log(64), 2000))
    y = np.rint(mu + rng.standard_normal(2000) * sig * 0.8)
    ref = norm.cdf((y + 0.5 - mu) / sig) - norm.cdf((y - 0.5 - mu) / sig)
    got = oe.likelihood(y, mu, sig)
    ok = ref > 1e-6
    np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-9)


def test_likelihood_symmetry():
    for mu in (-3, 0, 4):
        for dlt in range(0, 6):
            for sig in (0.2, 1.0, 7.5):
                a = oe.likelihood(np.array([mu + dlt]), float(mu), sig)
                b = oe.likelihood(np.array([mu - dlt]), float(mu), sig)
                assert a[0] == b[0]


@pytest.mark.parametrize("mu,sig", [(0.3, 0.11), (-2.7, 1.3), (10.49, 64.0),
                                    (0.5, 3.0), (-100.2, 0.5)])
def test_mass_sums_to_one(mu, sig):
    """Telescoping: sum over a covering range plus both tails, the tails
    computed separately, is 1."""
    lo, hi = int(math.floor(mu - 40 * sig)) - 3, int(math.ceil(mu + 40 * sig)) + 3
    k = np.arange(lo, hi + 1)
    below, above = oe.tail_masses(lo, hi, mu, sig)
    total = oe.likelihood(k, mu, sig).sum() + below + above
    assert abs(total - 1.0) < 1e-12
    lo, hi = int(round(mu)) - 2, int(round(mu)) + 2
    k = np.arange(lo, hi + 1)
    below, above = oe.tail_masses(lo, hi, mu, sig)
    assert abs(oe.likelihood(k, mu, sig).sum() + below + above - 1) < 1e-12


def test_bits_floor():
    assert oe.bits(np.array([1000]), 0.0, 0.11)[0] == pytest.approx(-math.log2(1e-9))


def test_cdf_tables_are_valid():
    tabs = oe.cdf_tables()
    assert len(tabs) == 64 * 16
    for idx, (R, freq) in enumerate(tabs):
        assert len(freq) == 2 * R + 2
        assert 4 <= R <= 255
        assert freq.sum() == 1 << 16
        assert freq.min() >= 1
        cdf = np.concatenate([[0], np.cumsum(freq)])
        assert (np.diff(cdf) > 0).all()
    # radius follows the scale: clamp(ceil(8 sigma), 4, 255)
    assert tabs[0][0] == 4 and tabs[63 * 16][0] == 255


def test_cdf_table_tracks_pmf():
    """Each quantized frequency is within the rounding of its FP64 mass."""
    for s in (0, 17, 40, 63):
        for m in (0, 7, 15):
            pmf = oe.table_pmf(s, m)
            assert abs(pmf.sum() - 1) < 1e-12
            freq = oe.quantize_pmf(pmf)
            K = (1 << 16) - len(pmf)
            big = int(np.argmax(freq))
            others = np.delete(np.arange(len(pmf)), big)
            assert (freq[others] >= np.floor(pmf[others] * K)).all()
            assert (freq[others] <= np.maximum(1, pmf[others] * K)).all()


def test_table_grid_endpoints():
    assert oe.table_scale(0) == pytest.approx(0.11, rel=1e-15)
    assert oe.table_scale(63) == pytest.approx(64.0, rel=1e-13)
    assert oe.table_phase(0) == -0.5 + 1 / 32 and oe.table_phase(15) == 0.5 - 1 / 32


def test_selection_f32_agrees_with_f64_away_from_ties():
    rng = np.random.default_rng(1)
    mu = rng.uniform(-50, 50, 200000)
    lsig = rng.uniform(math.log(0.11), math.log(64), 200000)
    c64, i64 = oe.cdf_select_f64(mu, lsig)
    c32, i32 = oe.cdf_select_f32(mu.astype(np.float32), lsig.astype(np.float32))
    far = oe.decision_margin(mu, lsig) > 1e-4
    assert far.mean() > 0.99
    assert (c64[far] == c32[far]).all() and (i64[far] == i32[far]).all()


def test_selection_hand_cases():
    # mu = 2.26 -> centre 2, phase 0.26 -> m = floor(0.76*16) = 12;
    # sigma = 0.11 -> scale 0; sigma = 64 -> scale 63
    c, i = oe.cdf_select_f64(np.array([2.26, -0.5, 0.49999]),
                             np.array([math.log(0.11), math.log(64.0), 0.0]))
    assert list(c) == [2, 0, 0]
    assert i[0] == 0 * 16 + 12
    assert i[1] == 63 * 16 + 0
    s_mid = math.floor((0 - math.log(0.11)) / oe.DELTA + 0.5)
    assert i[2] == s_mid * 16 + 15
    c, i = oe.cdf_select_f32(np.float32([2.26, -0.5]),
                             np.float32([math.log(0.11), math.log(64.0)]))
    assert list(c) == [2, 0] and list(i) == [12, 63 * 16]
