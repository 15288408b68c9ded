"""Host-side checks of the C ABI library (no GPU needed): symbol exports,
argument validation, integer CDF tables against the oracle, and the range
coder's round trip."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import entropy as oe

pswa_mod = pytest.importorskip("paper_2605_20977_amd.pswa")
P = pswa_mod
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pswa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pswa_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 15
    lib = C.CDLL(P.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTED)


@pytest.mark.parametrize("cfg", [synth.TINY, synth.FULL, synth.STUDENT, synth.TINY_CT,
                                 synth.FULL_CT])
def test_blob_size_matches_weight_shapes(cfg):
    d = P.model_desc(cfg)
    n = P.lib().pswa_model_blob_floats(C.byref(d))
    assert n == sum(int(np.prod(s)) for _, s in synth.weight_shapes(cfg))
    assert P.blob_order(cfg) == [nm for nm, _ in synth.weight_shapes(cfg)]


def test_invalid_descs_rejected():
    lib = P.lib()
    bad = [dict(window=4), dict(window=11), dict(heads=5), dict(d=96), dict(C=0),
           dict(prec=7), dict(L=0)]
    for b in bad:
        kw = dict(L=2, d=64, heads=4, window=5, mlp_ratio=4, C=32, Ch=16, prec=0)
        kw.update(b)
        d = P.ModelDesc(*[kw[k] for k in ("L", "d", "heads", "window", "mlp_ratio", "C", "Ch", "prec")])
        assert lib.pswa_model_blob_floats(C.byref(d)) == 0
        h = C.c_void_p()
        st = lib.pswa_model_create(C.byref(d), 256, 1, 256, 1 << 30, None, C.byref(h))
        assert st == -1 and not h.value


def test_create_checks_blob_and_alignment_before_any_device_call():
    lib = P.lib()
    d = P.model_desc(synth.TINY)
    n = lib.pswa_model_blob_floats(C.byref(d))
    h = C.c_void_p()
    assert lib.pswa_model_create(C.byref(d), 256, n - 1, 256, 1 << 30, None, C.byref(h)) == -2
    assert b"blob" in lib.pswa_last_error()
    assert lib.pswa_model_create(C.byref(d), 256, n, 257, 1 << 30, None, C.byref(h)) == -1
    assert lib.pswa_model_create(C.byref(d), None, n, 256, 1 << 30, None, C.byref(h)) == -1
    assert lib.pswa_model_create(C.byref(d), 256, n, 256, 16, None, C.byref(h)) == -1


def test_null_handles_rejected():
    lib = P.lib()
    fd = P.frame_desc(16, 16)
    assert lib.pswa_encode_workspace_bytes(None, C.byref(fd)) == 0
    assert lib.pswa_state_bytes(None, C.byref(fd)) == 0
    assert lib.pswa_decode_step(None, 0, None) == -1
    assert lib.pswa_num_steps(None) == -1
    assert lib.pswa_decode_end(None, None, None, None, None, None, None, None, None) == -1
    h = C.c_void_p()
    assert lib.pswa_decode_begin(None, C.byref(fd), 256, None, 0, 256, 0, 256, 1, None,
                                 C.byref(h)) == -1


def test_cdf_tables_equal_oracle_byte_for_byte():
    rad, off, freq = P.pswa_cdf_tables()
    ref = oe.cdf_tables()
    assert len(ref) == 1024
    for x, (R, fq) in enumerate(ref):
        assert rad[x] == R
        got = freq[off[x]:off[x + 1]].astype(np.int64)
        assert np.array_equal(got, fq), f"table {x}"


def _random_symbols(rng, n, esc_frac=0.02):
    mu = rng.uniform(-30, 30, n)
    lsig = rng.uniform(np.log(0.11), np.log(64), n)
    c, idx = oe.cdf_select_f64(mu, lsig)
    sig = np.exp(lsig)
    y = np.rint(mu + sig * rng.standard_normal(n)).astype(np.int64)
    esc = rng.random(n) < esc_frac
    y[esc] = c[esc] + rng.choice([-1, 1], esc.sum()) * rng.integers(256, 100000, esc.sum())
    y[:3] = [c[0] + 2 ** 30, c[1] - 2 ** 30, c[2]]
    return y.astype(np.int32), c, idx


def test_range_coder_round_trip():
    rng = np.random.default_rng(7)
    y, c, idx = _random_symbols(rng, 50000)
    data = P.pswa_range_encode_seq(y, c, idx)
    back = P.pswa_range_decode_seq(data, c, idx)
    assert np.array_equal(back, y)
    # close to the ideal code length (escapes aside)
    assert len(data) > 0


def test_range_coder_rate_matches_table_entropy():
    """Coded size equals the table's ideal length within a few bytes."""
    rng = np.random.default_rng(8)
    n = 20000
    mu = rng.uniform(-5, 5, n)
    lsig = rng.uniform(np.log(0.5), np.log(8), n)
    c, idx = oe.cdf_select_f64(mu, lsig)
    y = np.rint(mu + np.exp(lsig) * rng.standard_normal(n)).astype(np.int32)
    tabs = oe.cdf_tables()
    ideal = 0.0
    for k in range(n):
        R, fq = tabs[idx[k]]
        off = int(y[k]) - int(c[k])
        assert abs(off) <= R
        ideal += -np.log2(fq[off + R] / 65536.0)
    data = P.pswa_range_encode_seq(y, c, idx)
    assert abs(len(data) * 8 - ideal) < 64 + 1e-4 * ideal


def test_range_coder_detects_truncation_and_bad_index():
    rng = np.random.default_rng(9)
    y, c, idx = _random_symbols(rng, 5000)
    data = P.pswa_range_encode_seq(y, c, idx)
    with pytest.raises(P.PswaError) as e:
        P.pswa_range_decode_seq(data[: len(data) // 2], c, idx)
    assert e.value.name == "E_CORRUPT"
    bad = idx.copy()
    bad[10] = 5000
    with pytest.raises(P.PswaError):
        P.pswa_range_encode_seq(y, c, bad)
    with pytest.raises(P.PswaError):
        P.pswa_range_decode_seq(data, c, bad)


def test_frame_encode_uses_wavefront_order():
    rng = np.random.default_rng(10)
    H, W, Cc, k = 5, 9, 3, 5
    s = (k - 1) // 2 + 1
    y, c, idx = _random_symbols(rng, H * W * Cc, 0.0)
    y, c, idx = (a.reshape(H, W, Cc) for a in (y, c, idx))
    data = P.pswa_range_encode(H, W, Cc, k, y, c, idx)
    order = sorted(((j + s * i, i, j) for i in range(H) for j in range(W)))
    seq = [(i, j) for _, i, j in order]
    ys = np.concatenate([y[i, j] for i, j in seq])
    cs = np.concatenate([c[i, j] for i, j in seq])
    xs = np.concatenate([idx[i, j] for i, j in seq])
    assert data == P.pswa_range_encode_seq(ys, cs, xs)


def test_blob_shapes_round_trip():
    """The binding's blob layout matches the generator's weight list, and
    unpack_blob inverts pack_blob (the trainer reads weights back this way)."""
    import numpy as np
    import synth
    from paper_2605_20977_amd import pswa
    for cfg in (synth.TINY, synth.FULL, synth.STUDENT):
        assert pswa.blob_shapes(cfg) == synth.weight_shapes(cfg)
        W = synth.model_weights(cfg, 3)
        u = pswa.unpack_blob(cfg, pswa.pack_blob(cfg, W))
        assert all(np.array_equal(u[k], W[k]) for k in W)


def test_student_accept_rule():
    from paper_2605_20977_amd import pswa
    assert pswa.pswa_student_accept(101.0, 100.0, 0.01)
    assert not pswa.pswa_student_accept(101.01, 100.0, 0.01)
    assert pswa.pswa_student_accept(90.0, 100.0, 0.0)
    assert not pswa.pswa_student_accept(float("nan"), 100.0, 0.01)
    assert not pswa.pswa_student_accept(-1.0, 100.0, 0.01)


def test_frame_encode_uses_cyclic_order():
    """Cyclic schedule: steps t = 0..c-1, each in raster order."""
    rng = np.random.default_rng(11)
    H, W, Cc, k, cyc = 6, 7, 2, 7, 4
    y, c, idx = _random_symbols(rng, H * W * Cc, 0.0)
    y, c, idx = (a.reshape(H, W, Cc) for a in (y, c, idx))
    data = P.pswa_range_encode(H, W, Cc, k, y, c, idx, cycle=cyc)
    seq = [(i, j) for t in range(cyc) for i in range(H) for j in range(W) if (i + j) % cyc == t]
    ys = np.concatenate([y[i, j] for i, j in seq])
    cs = np.concatenate([c[i, j] for i, j in seq])
    xs = np.concatenate([idx[i, j] for i, j in seq])
    assert data == P.pswa_range_encode_seq(ys, cs, xs)
    with pytest.raises(P.PswaError):
        P.pswa_range_encode(H, W, Cc, k, y, c, idx, cycle=1)


def test_fp8_activation_scaling_descs():
    """FP8 per-tensor models carry one calibrated maximum per projection
    input after the weights (6 + 4 L of them); the per-row form and the
    other precisions carry none; a negative or NaN maximum is refused before
    any device call; per-row scaling is only for FP8."""
    lib = P.lib()
    cfg = synth.TINY
    nw = lib.pswa_model_blob_floats(C.byref(P.model_desc(cfg, "fp32")))
    assert lib.pswa_act_points(C.byref(P.model_desc(cfg))) == 6 + 4 * cfg.L
    assert lib.pswa_model_blob_floats(C.byref(P.model_desc(cfg, "bf16"))) == nw
    assert lib.pswa_model_blob_floats(C.byref(P.model_desc(cfg, "fp8", "row"))) == nw
    assert lib.pswa_model_blob_floats(C.byref(P.model_desc(cfg, "fp8"))) == nw + 6 + 4 * cfg.L
    for prec in ("fp32", "bf16"):
        assert lib.pswa_model_blob_floats(C.byref(P.model_desc(cfg, prec, "row"))) == 0
    d = P.model_desc(cfg, "fp8")
    n = nw + 6 + 4 * cfg.L
    for bad in (-1.0, float("nan"), float("inf")):
        blob = np.zeros(n, np.float32)
        blob[nw + 3] = bad
        h = C.c_void_p()
        st = lib.pswa_model_create(C.byref(d), blob.ctypes.data, n, 256, 1 << 30, None,
                                   C.byref(h))
        assert st == -1 and not h.value
        assert b"activation maximum 3" in lib.pswa_last_error()
    with pytest.raises(P.PswaError):
        P.Model(cfg, synth.model_weights(cfg, 1), "fp8", device="cpu")  # no maxima given


def test_channel_group_descs_validated():
    lib = P.lib()
    good = P.model_desc(synth.TINY_CT)
    assert lib.pswa_model_blob_floats(C.byref(good)) > 0
    base = dict(L=2, d=64, heads=4, window=5, mlp_ratio=4, C=32, Ch=16, prec=0, cycle=0,
                act_scaling=0, ch_groups=4, ch_d=64, ch_L=2, ch_ratio=2)
    bad = [dict(ch_groups=9), dict(ch_groups=3), dict(ch_d=60), dict(ch_d=4 * 528),
           dict(ch_L=0), dict(ch_L=5), dict(ch_ratio=0), dict(ch_ratio=5),
           dict(ch_groups=0)]   # ch_d / ch_L must then be 0
    names = ("L", "d", "heads", "window", "mlp_ratio", "C", "Ch", "prec", "cycle", "act_scaling",
             "ch_groups", "ch_d", "ch_L", "ch_ratio")
    for b in bad:
        kw = dict(base)
        kw.update(b)
        d = P.ModelDesc(*[kw[k] for k in names])
        assert lib.pswa_model_blob_floats(C.byref(d)) == 0, b
