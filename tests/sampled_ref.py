"""Oracle values at sampled positions of large frames (test helper).

The prediction at p = (i, j) depends only on a cone of positions: the last
layer reads W(p), each layer below one window further, and the accumulator
one window beyond that, so nothing farther than R = (L + 1) r rows above or
columns aside matters; previous frames add rows down to i + r, and the
cyclic schedule (full windows) rows down to i + R. The oracle run on the crop
rows [i0, i + 1 (+ r for P-frames, + R cyclic)), columns [j0, j + R + 1),
with i0, j0 the multiples of 4 at or below i - R and j - R (so the
hyperprior cells and sub-positions line up; for the cyclic schedule also
i0 + j0 = 0 mod cycle, so every step index is kept), therefore gives exactly
the full-frame value at p. tests/test_sampled_ref.py checks this against
whole-frame oracle runs.
"""
import numpy as np

from oracle import model as om


def oracle_at(cfg, Wt, y, z, prev, positions):
    """{(i, j): dict(mu, sigma, lsig) [C]} from per-position crops."""
    H, W, _ = y.shape
    R = (cfg.L + 1) * cfg.r
    cyc = getattr(cfg, "cycle", 0)
    out = {}
    for i, j in positions:
        i0 = max(0, i - R) // 4 * 4
        j0 = max(0, j - R) // 4 * 4
        if cyc:
            while (i0 + j0) % cyc:
                j0 -= 4
            assert j0 >= 0, "crop origin cannot keep the step index"
        below = R if cyc else (cfg.r if prev is not None else 0)
        i1 = min(H, i + 1 + below)
        j1 = min(W, j + R + 1)
        yc = y[i0:i1, j0:j1]
        zc = z[i0 // 4:-(-i1 // 4), j0 // 4:-(-j1 // 4)]
        pc = None if prev is None else prev[:, i0:i1, j0:j1]
        o = om.forward(cfg, Wt, yc, zc, pc)
        out[(i, j)] = {k: o[k][i - i0, j - j0] for k in ("mu", "sigma", "lsig")}
    return out


def sample_positions(H, W, n, seed):
    """n positions spread over the frame, corners and borders included."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2)]
    rnd = [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(max(0, n - len(fixed)))]
    return fixed[:n] + rnd
