"""FP64 oracle of the entropy-coding side: likelihoods, bits and integer CDFs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each latent symbol y is coded with a Gaussian of mean mu and scale sigma
(Sec. 3.1 and Fig. 1: the prediction heads output mu and sigma, which drive
the arithmetic coder). Its probability is the Gaussian mass of the unit bin
around y:

    P(y) = Phi((y + 1/2 - mu) / sigma) - Phi((y - 1/2 - mu) / sigma).

It depends on |y - mu| only, so it is evaluated as
    P = (erfc((v - 1/2) / (sigma sqrt 2)) - erfc((v + 1/2) / (sigma sqrt 2))) / 2,
v = |y - mu|, which never subtracts two numbers close to 1. Bits are
-log2(max(P, 1e-9)).

Integer CDF tables (reading: the paper fixes no table format; the tables are
integer and built deterministically in float64 so that encoder and decoder
agree bit for bit):
  * S = 64 scales sigma_s = 0.11 * exp(s * Delta), Delta = ln(64/0.11) / 63;
  * M = 16 mean phases f_m = (m + 1/2) / 16 - 1/2;
  * table (s, m) covers offsets k = -R..R around the centre (R = clamp(
    ceil(8 sigma_s), 4, 255)) plus one escape bin holding both tails;
  * frequencies at 16-bit precision: freq = max(1, floor(pmf * (2^16 -
    n_bins))), and what is left of 2^16 goes to the largest bin (lowest
    index on ties).
A symbol selects its table by centre c = floor(mu + 1/2), phase index
m = min(15, floor((mu - c + 1/2) * 16)) and scale index
s = clamp(floor((ln sigma - ln 0.11) / Delta + 1/2), 0, 63).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .model import LN_SIGMA_MAX, LN_SIGMA_MIN, SIGMA_MIN

P_FLOOR = 1e-9
N_SCALES = 64
N_PHASES = 16
PREC_BITS = 16
DELTA = (LN_SIGMA_MAX - LN_SIGMA_MIN) / (N_SCALES - 1)
SQRT2 = math.sqrt(2.0)


def likelihood(y, mu, sigma):
    """Discretized-Gaussian probability of integer y (float64)."""
    v = np.abs(np.asarray(y, dtype=np.float64) - mu)
    s2 = np.asarray(sigma, dtype=np.float64) * SQRT2
    return 0.5 * (erfc((v - 0.5) / s2) - erfc((v + 0.5) / s2))


def bits(y, mu, sigma):
    return -np.log2(np.maximum(likelihood(y, mu, sigma), P_FLOOR))


def tail_masses(lo, hi, mu, sigma):
    """P(Y < lo - 1/2) and P(Y > hi + 1/2), each from its own erfc."""
    s2 = np.asarray(sigma, dtype=np.float64) * SQRT2
    below = 0.5 * erfc((mu - (lo - 0.5)) / s2)
    above = 0.5 * erfc(((hi + 0.5) - mu) / s2)
    return below, above


# --------------------------------------------------------------------------
# Integer CDF tables
# --------------------------------------------------------------------------

def table_scale(s):
    return SIGMA_MIN * math.exp(s * DELTA)


def table_phase(m):
    return (m + 0.5) / N_PHASES - 0.5


def table_radius(sig):
    return int(min(255, max(4, math.ceil(8.0 * sig))))


def table_pmf(s, m):
    """FP64 pmf of table (s, m): bins k = -R..R then the escape bin."""
    sig, f = table_scale(s), table_phase(m)
    R = table_radius(sig)
    k = np.arange(-R, R + 1, dtype=np.float64)
    pmf = likelihood(k, f, sig)
    below, above = tail_masses(-R, R, f, sig)
    return np.concatenate([pmf, [below + above]])


def quantize_pmf(pmf):
    """16-bit integer frequencies, every bin >= 1, summing to 2^16."""
    n = len(pmf)
    total = 1 << PREC_BITS
    freq = np.maximum(1, np.floor(pmf * (total - n))).astype(np.int64)
    freq[int(np.argmax(freq))] += total - int(freq.sum())
    return freq


def cdf_tables():
    """List over table index s*16 + m of (R, freq int64 [2R+2])."""
    out = []
    for s in range(N_SCALES):
        for m in range(N_PHASES):
            pmf = table_pmf(s, m)
            out.append(((len(pmf) - 2) // 2, quantize_pmf(pmf)))
    return out


def cdf_select_f64(mu, lsig):
    """(centre int32, table index uint16) decided in float64."""
    mu = np.asarray(mu, dtype=np.float64)
    lsig = np.asarray(lsig, dtype=np.float64)
    c = np.floor(mu + 0.5)
    m = np.minimum(N_PHASES - 1, np.floor((mu - c + 0.5) * N_PHASES))
    s = np.clip(np.floor((lsig - LN_SIGMA_MIN) / DELTA + 0.5), 0, N_SCALES - 1)
    return c.astype(np.int32), (s * N_PHASES + m).astype(np.uint16)


# float32 constants of the single-precision decision.
LN_SIGMA_MIN_F32 = np.float32(LN_SIGMA_MIN)
INV_DELTA_F32 = np.float32(1.0 / DELTA)


def cdf_select_f32(mu, lsig):
    """The same decision taken in float32, one rounding per operation:
    c = floor(mu + 0.5); m = min(15, floor((mu - c + 0.5) * 16));
    s = clamp(floor((lsig - ln 0.11) * (1 / Delta) + 0.5), 0, 63)."""
    f32 = np.float32
    mu = np.asarray(mu, dtype=f32)
    lsig = np.asarray(lsig, dtype=f32)
    c = np.floor(mu + f32(0.5))
    ph = (mu - c) + f32(0.5)
    m = np.minimum(f32(N_PHASES - 1), np.floor(ph * f32(N_PHASES)))
    t = (lsig - LN_SIGMA_MIN_F32) * INV_DELTA_F32
    s = np.clip(np.floor(t + f32(0.5)), f32(0), f32(N_SCALES - 1))
    return c.astype(np.int32), (s.astype(np.int32) * N_PHASES
                                + m.astype(np.int32)).astype(np.uint16)


def decision_margin(mu, lsig):
    """Distance (in the decision's own units) of each symbol from the
    nearest centre/phase/scale boundary; small values are ties that either
    precision may break either way."""
    mu = np.asarray(mu, dtype=np.float64)
    lsig = np.asarray(lsig, dtype=np.float64)
    ph = (mu + 0.5) * N_PHASES
    dm = np.abs(ph - np.rint(ph)) / N_PHASES
    ts = (lsig - LN_SIGMA_MIN) / DELTA + 0.5
    ds = np.abs(ts - np.rint(ts)) * DELTA
    return np.minimum(dm, ds)
