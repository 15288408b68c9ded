"""Seeded synthetic inputs for the P-SWA wavefront context model.

This module is shared by the FP64 oracle, the tests and the benchmark. It
holds shapes, seeds and random draws only: none of the context model's
arithmetic lives here, so the oracle and the HIP path stay independent.

Everything is drawn with NumPy's PCG64 generator in float64 and rounded once
(to int32 for symbols, to float32 for weights); each kind of draw (weights,
latent, hyperprior, previous frames) has its own stream, seeded by
SeedSequence([seed, kind]).

Data recipe (a stand-in for the 1080p test sequences the paper evaluates on,
which are not available):
  * latent y[i, j, c] = rint(mu[i, j, c] + b[c] * Laplace(0, 1)), with mu a
    per-channel smooth Gaussian random field (white N(0, 1) noise filtered
    by a periodic Gaussian kernel of std 2 latent pixels, scaled to std 3)
    and b[c] log-uniform in [0.2, 4];
  * hyperprior z[u, v, c] = rint(N(0, 2)), std 2;
  * previous frames (P-frames): y_tau = y + rint(N(0, 1)), independent for
    tau = 1 (most recent) and tau = 2.

Weight recipe ("random-init weights from the seed"): linear weights
N(0, 1/fan_in); norm gains 1; input scale 1/3; sub-position embedding and
null key/value N(0, 1); relative-position biases N(0, 0.1^2); mean gain 1,
mean offset 0, scale gain 0.25, scale offset ln 3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "ModelCfg", "FrameCfg", "TINY", "FULL", "STUDENT",
    "bias_sizes", "weight_shapes", "model_weights",
    "latent_frame", "hyper_frame", "prev_frames", "frame_inputs",
    "BATCH_MIX", "CONFIG_SEEDS", "CYCLIC", "TINY_CYCLIC", "CALIB_SEED", "calibration_frames",
    "TINY_CT", "FULL_CT",
]


@dataclasses.dataclass(frozen=True)
class ModelCfg:
    """Shape of a context model: L layers of width d with `heads` heads,
    window k x k, SwiGLU hidden width mlp_ratio * d, C latent channels and
    Ch hyperprior channels. cycle = 0: wavefront schedule t = j + s i with
    the causal half-window; cycle = s >= 2: the cyclic schedule
    step = (i + j) mod s with the full window masked by step. ch_groups =
    N >= 2 replaces the head by a Channel Transformer over N channel groups
    (width ch_d, ch_L blocks, grouped SwiGLU of ch_ratio * ch_d / N per
    group) with grouped prediction heads; 0 keeps the plain head."""
    L: int
    d: int
    heads: int
    window: int
    mlp_ratio: int
    C: int
    Ch: int
    cycle: int = 0
    ch_groups: int = 0
    ch_d: int = 0
    ch_L: int = 0
    ch_ratio: int = 4

    @property
    def dh(self) -> int:
        return self.d // self.heads

    @property
    def F(self) -> int:
        return self.mlp_ratio * self.d

    @property
    def r(self) -> int:
        return (self.window - 1) // 2


@dataclasses.dataclass(frozen=True)
class FrameCfg:
    """Latent grid H x W (C channels come from the model) and hyperprior grid
    Hh x Wh; n_prev = 0 for an I-frame, 2 for a P-frame."""
    H: int
    W: int
    n_prev: int = 0

    @property
    def Hh(self) -> int:
        return -(-self.H // 4)

    @property
    def Wh(self) -> int:
        return -(-self.W // 4)


# Tiny intra model: 2 layers, d = 64, 4 heads, causal 5x5 window.
TINY = ModelCfg(L=2, d=64, heads=4, window=5, mlp_ratio=4, C=32, Ch=16)
# 1080p model: 6 layers, d = 384, 8 heads of 48, causal 9x9 window.
FULL = ModelCfg(L=6, d=384, heads=8, window=9, mlp_ratio=4, C=192, Ch=128)
# Distilled student: 2 layers, d = 128, 4 heads, causal 9x9 window.
STUDENT = ModelCfg(L=2, d=128, heads=4, window=9, mlp_ratio=4, C=192, Ch=128)

# The cyclic schedule of the paper (full 7x7 window, s = 4 steps per frame)
# on the 1080p model's widths, and its tiny counterpart.
CYCLIC = ModelCfg(L=6, d=384, heads=8, window=7, mlp_ratio=4, C=192, Ch=128, cycle=4)
TINY_CYCLIC = ModelCfg(L=2, d=64, heads=4, window=5, mlp_ratio=4, C=32, Ch=16, cycle=4)

# The Channel Transformer (N = 4 channel groups, 2 blocks) on the tiny and
# the 1080p-shaped models.
TINY_CT = ModelCfg(L=2, d=64, heads=4, window=5, mlp_ratio=4, C=32, Ch=16,
                   ch_groups=4, ch_d=64, ch_L=2, ch_ratio=2)
FULL_CT = ModelCfg(L=6, d=384, heads=8, window=9, mlp_ratio=4, C=192, Ch=128,
                   ch_groups=4, ch_d=512, ch_L=2, ch_ratio=4)

# Batched decode mix: 8 frames of each grid size, I and P alternating.
BATCH_MIX = [(15, 20), (34, 60), (45, 80), (68, 120)]

# (data seed, weight seed) of each workload.
CONFIG_SEEDS = {
    "tiny": (0, 1),
    "1080p_I": (10, 11),
    "1080p_P": (20, 11),
    "batch": (30, 11),
    "4k_student": (40, 11),
    "1080p_cyclic": (50, 12),
}

# Data seeds of the frames that calibrate FP8 per-tensor activation scales:
# disjoint from every seed a test or the benchmark decodes.
CALIB_SEED = 9000


def calibration_frames(mcfg: ModelCfg, H: int = 68, W: int = 120) -> list[dict]:
    """One I-frame and one P-frame of H x W for calibrating activation
    scales, as dicts of latents, hyper and prev."""
    out = []
    for k, n_prev in enumerate((0, 2)):
        y, z, prev = frame_inputs(mcfg, FrameCfg(H, W, n_prev), CALIB_SEED + 10 * k)
        out.append({"latents": y, "hyper": z, "prev": prev})
    return out


# Every kind of draw has its own stream, keyed by (seed, kind), so that equal
# seed numbers of different kinds never share random numbers (a hyperprior
# drawn from the weights' own stream would be correlated with the hyperprior
# projection).
_WEIGHTS, _LATENT, _HYPER, _PREV = 1, 2, 3, 4


def _rng(seed: int, kind: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, kind])))


def bias_sizes(cfg: ModelCfg) -> tuple[int, int, int]:
    """Number of relative-bias slots: (accumulator, spatial layer, temporal
    layer). Wavefront schedule: the causal window holds r rows of 2r+1 above
    and r to the left (2r(r+1) cells) and the layer window adds the query
    itself. Cyclic schedule: both use the full (2r+1)^2 window. The temporal
    window is (2r+1)^2 cells in each of two previous frames."""
    r = cfg.r
    k2 = (2 * r + 1) ** 2
    if cfg.cycle:
        return k2, k2, 2 * k2
    n_acc = 2 * r * (r + 1)
    return n_acc, n_acc + 1, 2 * k2


def weight_shapes(cfg: ModelCfg) -> list[tuple[str, tuple[int, ...]]]:
    """Ordered (name, shape) list of every parameter. Linear weights are
    stored [out_features, in_features]."""
    d, C, Ch, F, h = cfg.d, cfg.C, cfg.Ch, cfg.F, cfg.heads
    n_acc, n_sp, n_tm = bias_sizes(cfg)
    out = [
        ("hyper.W", (d, Ch)), ("hyper.P4", (16, d)),
        ("in.g", (C,)), ("in.W", (d, C)),
        ("acc.gq", (d,)), ("acc.Wq", (d, d)),
        ("acc.gkv", (d,)), ("acc.Wkv", (2 * d, d)),
        ("acc.knull", (d,)), ("acc.vnull", (d,)),
        ("acc.bias", (h, n_acc)), ("acc.Wo", (d, d)),
    ]
    for l in range(cfg.L):
        p = f"layer{l}."
        out += [
            (p + "g1", (d,)), (p + "Wqkv", (3 * d, d)),
            (p + "bias", (h, n_sp + n_tm)), (p + "Wo", (d, d)),
            (p + "g2", (d,)), (p + "Wgate", (F, d)), (p + "Wup", (F, d)),
            (p + "Wdown", (d, F)),
        ]
    if cfg.ch_groups:
        N, dc = cfg.ch_groups, cfg.ch_d
        dg, Cg = dc // N, C // N
        Fg = cfg.ch_ratio * dg
        out += [("ct.gx", (d,)), ("ct.Wx", (dc, d)), ("ct.gy", (C,)), ("ct.Wy", (dc, C))]
        for b in range(cfg.ch_L):
            p = f"ct{b}."
            out += [(p + "g1", (dc,)), (p + "M", (dc, dc)), (p + "g2", (dc,)),
                    (p + "Wgate", (N, Fg, dg)), (p + "Wup", (N, Fg, dg)),
                    (p + "Wdown", (N, dg, Fg))]
        out += [("ctH.g", (dc,)), ("ctH.W1", (N, dg, dg)), ("ctH.W2", (N, 2 * Cg, dg))]
    else:
        out += [("head.g", (d,)), ("head.W1", (d, d)), ("head.W2", (2 * C, d))]
    out += [
        ("head.gmu", (C,)), ("head.bmu", (C,)),
        ("head.gsig", (C,)), ("head.bsig", (C,)),
    ]
    return out


def model_weights(cfg: ModelCfg, seed: int) -> dict[str, np.ndarray]:
    """Random-init float32 weights, drawn in float64 and rounded once."""
    rng = _rng(seed, _WEIGHTS)
    w: dict[str, np.ndarray] = {}
    for name, shape in weight_shapes(cfg):
        leaf = name.split(".")[-1]
        if leaf.startswith("W") or leaf == "M":
            a = rng.standard_normal(shape) / math.sqrt(shape[-1])
        elif leaf in ("g", "gq", "gkv", "g1", "g2", "gmu", "gx"):
            a = np.ones(shape)
        elif leaf == "bias":
            a = 0.1 * rng.standard_normal(shape)
        elif leaf in ("P4", "knull", "vnull"):
            a = rng.standard_normal(shape)
        elif leaf == "bmu":
            a = np.zeros(shape)
        elif leaf == "gsig":
            a = np.full(shape, 0.25)
        elif leaf == "gy":  # set below (input scale)
            a = np.zeros(shape)
        elif leaf == "bsig":
            a = np.full(shape, math.log(3.0))
        else:
            raise KeyError(name)
        if name in ("in.g", "ct.gy"):
            a = np.full(shape, 1.0 / 3.0)
        w[name] = np.ascontiguousarray(a, dtype=np.float32)
    return w


def _smooth_field(rng, H, W, C, std_px=2.0, target_std=3.0):
    white = rng.standard_normal((C, H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    # Fourier transform of a periodic Gaussian kernel of std `std_px`.
    kern = np.exp(-2.0 * (math.pi * std_px) ** 2 * (fy ** 2 + fx ** 2))
    f = np.fft.ifft2(np.fft.fft2(white, axes=(1, 2)) * kern, axes=(1, 2)).real
    sd = f.reshape(C, -1).std(axis=1)
    # a one-pixel grid has no spread: its field is the constant 0
    gain = np.where(sd > 1e-9, target_std / np.maximum(sd, 1e-9), 0.0)
    f = (f - f.reshape(C, -1).mean(axis=1)[:, None, None] * (sd <= 1e-9)[:, None, None]) \
        * gain[:, None, None]
    return np.transpose(f, (1, 2, 0))


def latent_frame(H: int, W: int, C: int, seed: int) -> np.ndarray:
    """int32 [H, W, C] latent symbols (see the module recipe)."""
    rng = _rng(seed, _LATENT)
    mu = _smooth_field(rng, H, W, C)
    b = np.exp(rng.uniform(math.log(0.2), math.log(4.0), size=C))
    lap = rng.laplace(0.0, 1.0, size=(H, W, C))
    return np.rint(mu + b[None, None, :] * lap).astype(np.int32)


def hyper_frame(Hh: int, Wh: int, Ch: int, seed: int) -> np.ndarray:
    """int32 [Hh, Wh, Ch] hyperprior symbols, rint(N(0, 2))."""
    rng = _rng(seed, _HYPER)
    return np.rint(2.0 * rng.standard_normal((Hh, Wh, Ch))).astype(np.int32)


def prev_frames(y: np.ndarray, seed: int) -> np.ndarray:
    """int32 [2, H, W, C]: y plus independent rint(N(0, 1)) drift per frame."""
    rng = _rng(seed, _PREV)
    drift = np.rint(rng.standard_normal((2,) + y.shape)).astype(np.int32)
    return (y[None] + drift).astype(np.int32)


def frame_inputs(mcfg: ModelCfg, fcfg: FrameCfg, seed: int):
    """(y, z, prev-or-None) for one frame, all from one data seed: the latent
    uses `seed`, the hyperprior `seed + 1`, the previous frames `seed + 2`."""
    y = latent_frame(fcfg.H, fcfg.W, mcfg.C, seed)
    z = hyper_frame(fcfg.Hh, fcfg.Wh, mcfg.Ch, seed + 1)
    prev = prev_frames(y, seed + 2) if fcfg.n_prev else None
    return y, z, prev
