"""Host quantizer of the projection weights against brute-force encoders."""
import numpy as np
import pytest

P = pytest.importorskip("paper_2605_20977_amd.pswa")


def e4m3fn_values():
    """All 256 OCP e4m3fn codes decoded from the format's definition
    (bias 7, 3 mantissa bits, exponent 0 subnormal, code 0x7f/0xff NaN)."""
    v = np.empty(256)
    for c in range(256):
        s, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            v[c] = np.nan
            continue
        mag = (1 + m / 8) * 2.0 ** (e - 7) if e else (m / 8) * 2.0 ** -6
        v[c] = -mag if s else mag
    return v


def nearest_even(x, table, codes):
    """Nearest finite table value; ties to the code with an even mantissa."""
    out = np.empty(len(x), np.int64)
    for i, xv in enumerate(x):
        d = np.abs(table - xv)
        best = np.nanmin(d)
        cand = codes[np.where(d == best)[0]]
        even = [c for c in cand if (c & 1) == 0]
        out[i] = even[0] if even else cand[0]
    return out


def test_fp8_matches_brute_force():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(3000) * 0.05, rng.uniform(-1, 1, 2000) * 3e-3,
                        [0.0, -0.0, 1.0, -1.0, 5e-4, 1e-9]]).astype(np.float32)
    got, inv = P.pswa_quantize("fp8", x)
    s = 448.0 / float(np.max(np.abs(x.astype(np.float64))))
    assert abs(inv - 1 / s) <= 1e-7 / s
    table = e4m3fn_values()
    fin = ~np.isnan(table)
    codes = np.arange(256)[fin]
    ref = nearest_even((x.astype(np.float64) * s).astype(np.float32).astype(np.float64),
                       table[fin], codes)
    vals_got, vals_ref = table[got], table[ref]
    # +0 and -0 are the same value
    assert np.array_equal(vals_got, vals_ref)
    assert got.max() <= 0xfe and (got & 0x7f).max() <= 0x7e


def test_fp8_saturates_and_keeps_max():
    x = np.array([1.0, -2.0, 0.5], np.float32)
    got, inv = P.pswa_quantize("fp8", x)
    assert got[1] == 0xfe and got[0] == 0x76  # -448 and 224
    assert abs(inv - 2.0 / 448) < 1e-9


def test_bf16_matches_brute_force():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-6, 6, 4000),
                        [0.0, 1.0, -1.5, 3.0e38]]).astype(np.float32)
    got, inv = P.pswa_quantize("bf16", x)
    assert inv == 1.0
    bits = x.view(np.uint32)
    lo = (bits >> 16).astype(np.uint32)
    hi = lo + 1
    vlo = (lo << 16).view(np.float32).astype(np.float64)
    vhi = (hi << 16).view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo, dhi = np.abs(xd - vlo), np.abs(vhi - xd)
    ref = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    assert np.array_equal(got.astype(np.uint32), ref)
