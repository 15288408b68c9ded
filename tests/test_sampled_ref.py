"""The cone-crop oracle (tests/sampled_ref.py) equals whole-frame oracle
runs, for I- and P-frames, at corners, borders and inside positions."""
import numpy as np
import pytest

import synth
from oracle import model as om

from sampled_ref import oracle_at, sample_positions


@pytest.mark.parametrize("n_prev,cycle", [(0, 0), (2, 0), (0, 4), (2, 4)])
def test_crop_oracle_equals_full_frame(n_prev, cycle):
    cfg = synth.ModelCfg(L=2, d=32, heads=2, window=5, mlp_ratio=2, C=8, Ch=4, cycle=cycle)
    Wt = synth.model_weights(cfg, 12)
    H, W = (23, 29) if not cycle else (30, 31)
    y, z, prev = synth.frame_inputs(cfg, synth.FrameCfg(H, W, n_prev), 40 + n_prev)
    full = om.forward(cfg, Wt, y, z, prev)
    pos = sample_positions(H, W, 12, 3)
    got = oracle_at(cfg, Wt, y, z, prev, pos)
    for (i, j), o in got.items():
        for k in ("mu", "sigma"):
            assert np.allclose(o[k], full[k][i, j], rtol=0, atol=1e-12), (i, j, k)
