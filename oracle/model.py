"""FP64 oracle of the P-SWA context model run as a diagonal wavefront.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Kopte and Kaup, "Parallel Context Modeling for Sliding Window
Attention in Neural Video Coding" (arXiv 2605.20977).

What is computed, with the passage each part follows:

* Window and schedule -- Sec. 2 (WPP: one active diagonal wavefront) and
  Sec. 3.2 / Fig. 2 (a repeating local dependency pattern lets every position
  of a diagonal be predicted in one step). The causal k x k window W-(p) of a
  position p = (i, j) holds all 2r+1 columns of the r rows above and the r
  cells to its left (r = (k-1)/2). With step t(i, j) = j + s*i and slope
  s = r + 1 every cell of W-(p) lies on an earlier diagonal. The paper's own
  cyclic schedule, step = (i + j) mod s (Fig. 2a), is given as well.
* Hyperprior token -- Sec. 3.1 (the decoded hyperprior is the accumulator's
  query and its residual) and Fig. 1 (hyperprior at 1/4 resolution). Reading:
  nearest x4 upsampling of a linear embedding of z plus a learned 16-entry
  sub-position embedding.
* Decoded-latent embedding -- Sec. 3.1: learnable channel-wise input scale
  (rate re-injection), then a linear embedding.
* Accumulator -- Sec. 3.1 and Fig. 2b: cross-attention, query and residual
  from the hyperprior token, keys/values from already decoded neighbours
  only (strictly past), plus a learned null key/value so that a position with
  no decoded neighbour still attends somewhere.
* Layers -- Sec. 3.1 (Llama-2 style blocks: RMSNorm pre-norm, SwiGLU MLP)
  with causal sliding-window self-attention over W(p) = W-(p) + {p}; for
  P-frames one softmax also runs over the (2r+1)^2 window of each of the two
  previous frames (time-causal SWA, Sec. 3.1).
* Head -- Sec. 3.1: two-layer MLP to the mean and scale of a Gaussian, with
  learnable channel-wise output scales.
* Channel Transformer (models with ch_groups = N >= 2) -- Sec. 3.1 and
  Sec. 3.2 (s spatial steps decoupled from N channel groups): the channels
  are split into N groups and decoded group after group at every position.
  Its input joins the spatial output with the channel-shifted latent (the
  shift by one group means group 0 sees the spatio-temporal context only);
  each block mixes the groups with a dense linear map whose
  block-lower-triangular mask lets group g read groups 0..g only (a masked
  1x1 convolution), then runs a SwiGLU MLP per group; grouped two-layer
  heads give the mean and scale of each group's channels. Readings: every
  norm and MLP acts on one group's slice (a norm over all groups would let
  later groups leak into earlier ones), pre-norm residual blocks as in the
  spatial layers, the input projection of the shifted latent is masked
  like the mixing map.

Readings where the paper is silent: per-head learned relative-position bias
as the only positional signal; RMSNorm eps 1e-5; no biases in linears;
SwiGLU hidden width = mlp_ratio * d; scale = exp of an affine output clamped
to [0.11, 64]; out-of-frame keys are masked, never zero-padded.

Weights are stored [out_features, in_features]; the oracle promotes the
float32 values every path loads to float64.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 1e-5
SIGMA_MIN = 0.11
SIGMA_MAX = 64.0
LN_SIGMA_MIN = math.log(SIGMA_MIN)
LN_SIGMA_MAX = math.log(SIGMA_MAX)


# --------------------------------------------------------------------------
# Window geometry and schedules (Sec. 2 WPP; Sec. 3.2, Fig. 2)
# --------------------------------------------------------------------------

def causal_window(r: int) -> list[tuple[int, int]]:
    """Offsets (da, db) of W-(p), in bias-slot order: the r rows above, each
    from column -r to +r, then the r cells left of p on its own row."""
    offs = [(a, b) for a in range(-r, 0) for b in range(-r, r + 1)]
    offs += [(0, b) for b in range(-r, 0)]
    return offs


def layer_window(r: int) -> list[tuple[int, int]]:
    """W(p) = W-(p) plus p itself (self is the last bias slot)."""
    return causal_window(r) + [(0, 0)]


def temporal_window(r: int) -> list[tuple[int, int, int]]:
    """(tau, da, db) of the temporal window: a full (2r+1)^2 window centred
    on p in each previous frame tau = 1 (most recent), 2."""
    return [(tau, a, b) for tau in (1, 2)
            for a in range(-r, r + 1) for b in range(-r, r + 1)]


def wavefront_slope(r: int) -> int:
    """Smallest slope s of t = j + s*i that puts the above-right neighbour
    (i-1, j+r) on an earlier diagonal: s = r + 1."""
    return r + 1


def step_index(i, j, s):
    """Wavefront step of position (i, j)."""
    return j + s * i


def num_steps(H: int, W: int, s: int) -> int:
    return (W - 1) + s * (H - 1) + 1


def diagonals(H: int, W: int, s: int) -> list[np.ndarray]:
    """D_t for t = 0..T-1: int arrays [n_t, 2] of (i, j), i ascending."""
    out = []
    for t in range(num_steps(H, W, s)):
        rows = [(i, t - s * i) for i in range(H) if 0 <= t - s * i < W]
        out.append(np.array(rows, dtype=np.int64).reshape(-1, 2))
    return out


def cyclic_step(i, j, s: int = 4):
    """The paper's repeating s x s mask (Fig. 2a): each mask row is a cyclic
    shift of the one above, step = (i + j) mod s (the figure prints step+1)."""
    return (np.asarray(i) % s + np.asarray(j) % s) % s


def full_window(r: int) -> list[tuple[int, int]]:
    """Offsets of the full (2r+1) x (2r+1) window in raster order (the query
    itself at index r(2r+1) + r): the cyclic schedule's spatial slots."""
    return [(a, b) for a in range(-r, r + 1) for b in range(-r, r + 1)]


def schedule_step(cfg, i, j):
    """Decoding step of position (i, j): j + s i (wavefront, s = r + 1), or
    (i + j) mod cycle (the paper's cyclic pattern, Fig. 2a)."""
    if cfg.cycle:
        return cyclic_step(i, j, cfg.cycle)
    return step_index(np.asarray(i), np.asarray(j), wavefront_slope(cfg.r))


def acc_slots(cfg) -> list[tuple[int, int]]:
    """Spatial key slots of the accumulator: the causal window (wavefront),
    or the full window masked to strictly earlier steps (cyclic)."""
    return full_window(cfg.r) if cfg.cycle else causal_window(cfg.r)


def layer_slots(cfg) -> list[tuple[int, int]]:
    """Spatial key slots of a layer: the causal window plus the query
    (wavefront), or the full window masked to steps up to the query's own
    (cyclic: same-step positions see each other in the layers, Fig. 2b)."""
    return full_window(cfg.r) if cfg.cycle else layer_window(cfg.r)


def schedule_groups(cfg, H: int, W: int) -> list[np.ndarray]:
    """Positions decoded together, step by step: the diagonals of the
    wavefront, or for the cyclic schedule every position of one step (in
    raster order)."""
    if not cfg.cycle:
        return diagonals(H, W, wavefront_slope(cfg.r))
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    st = cyclic_step(ii, jj, cfg.cycle)
    return [np.argwhere(st == t).reshape(-1, 2) for t in range(cfg.cycle)]


def _step_mask(cfg, H, W, a, b, strict):
    """Whether the key at offset (a, b) is decoded early enough for each
    query: always, in the wavefront's causal windows; step(key) < step(p)
    (strict, accumulator) or <= (layers) for the cyclic schedule. Out-of-
    frame keys are masked separately."""
    if not cfg.cycle:
        return np.ones((H, W), dtype=bool)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    sp = cyclic_step(ii, jj, cfg.cycle)
    sq = cyclic_step(ii + a, jj + b, cfg.cycle)
    return sq < sp if strict else sq <= sp


# --------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------

def rmsnorm(x, g):
    """RMSNorm pre-norm (Sec. 3.1, Llama 2): x / sqrt(mean(x^2) + eps) * g."""
    return x / np.sqrt(np.mean(x * x, axis=-1, keepdims=True) + EPS) * g


def silu(x):
    return x / (1.0 + np.exp(-x))


def linear(x, W):
    """x @ W^T with W stored [out, in]."""
    return x @ np.asarray(W, dtype=np.float64).T


def _w(Wt, name):
    return np.asarray(Wt[name], dtype=np.float64)


def _shift(A, da, db):
    """B[i, j] = A[i+da, j+db] where that cell is in the frame; returns
    (B, valid) with B zero where invalid (masked, not used as a value)."""
    H, W = A.shape[:2]
    B = np.zeros_like(A)
    valid = np.zeros((H, W), dtype=bool)
    i0, i1 = max(0, -da), min(H, H - da)
    j0, j1 = max(0, -db), min(W, W - db)
    if i0 < i1 and j0 < j1:
        B[i0:i1, j0:j1] = A[i0 + da:i1 + da, j0 + db:j1 + db]
        valid[i0:i1, j0:j1] = True
    return B, valid


def hyper_tokens(Wt, z, H, W):
    """h_p = W_h z[i//4, j//4] + P4[4 (i mod 4) + (j mod 4)]   [H, W, d]."""
    ii = np.arange(H)[:, None]
    jj = np.arange(W)[None, :]
    zz = np.asarray(z, dtype=np.float64)[ii // 4, jj // 4]
    sub = (ii % 4) * 4 + (jj % 4)
    return linear(zz, _w(Wt, "hyper.W")) + _w(Wt, "hyper.P4")[sub]


def latent_embed(Wt, y):
    """e = W_in (g_in * y)  (input scale re-injects the rate, Sec. 3.1)."""
    return linear(np.asarray(y, dtype=np.float64) * _w(Wt, "in.g"),
                  _w(Wt, "in.W"))


def acc_keys_values(Wt, e):
    """Accumulator K/V of decoded positions: W_kv^a RMSNorm(e)  [.., 2d]."""
    return linear(rmsnorm(e, _w(Wt, "acc.gkv")), _w(Wt, "acc.Wkv"))


def temporal_keys_values(Wt, l, e_prev):
    """Layer-l K/V of a previous frame's embedded latent: the k/v rows of
    that layer's QKV projection applied to RMSNorm_{g1}(e)   [.., 2d]."""
    d = e_prev.shape[-1]
    Wkv = _w(Wt, f"layer{l}.Wqkv")[d:]
    return linear(rmsnorm(e_prev, _w(Wt, f"layer{l}.g1")), Wkv)


def _windowed_attention(q, slots, heads):
    """Softmax attention of each query over its key slots.

    q: [H, W, d]. slots: list of (K, V, valid, bias) with K, V [H, W, d]
    (already aligned to the query position), valid [H, W] and bias [heads].
    Every query must have at least one valid slot."""
    H, W, d = q.shape
    dh = d // heads
    qh = q.reshape(H, W, heads, dh)
    logits = np.empty((len(slots), H, W, heads))
    for n, (K, _, valid, bias) in enumerate(slots):
        lg = (qh * K.reshape(H, W, heads, dh)).sum(-1) / math.sqrt(dh) + bias
        logits[n] = np.where(valid[..., None], lg, -np.inf)
    mx = logits.max(axis=0)
    w = np.exp(logits - mx)
    w /= w.sum(axis=0)
    out = np.zeros((H, W, heads, dh))
    for n, (_, V, valid, _) in enumerate(slots):
        out += w[n][..., None] * V.reshape(H, W, heads, dh)
    return out.reshape(H, W, d)


# --------------------------------------------------------------------------
# Parallel (definition) form
# --------------------------------------------------------------------------

def forward(cfg, Wt, y, z, prev=None, keep=False):
    """Mean, scale and log-scale of every symbol, all positions at once.

    cfg: ModelCfg; Wt: weight dict; y int [H, W, C]; z int [Hh, Wh, Ch];
    prev int [2, H, W, C] (tau = 1, 2) for a P-frame, else None.
    Returns dict(mu, sigma, lsig) of [H, W, C] float64 (and, with keep=True,
    the hyper tokens 'h', the accumulator output 'x0' and each layer's
    output 'x1'..'xL')."""
    H, W, C = y.shape
    d, heads, r = cfg.d, cfg.heads, cfg.r
    dh = d // heads
    out = {}

    h = hyper_tokens(Wt, z, H, W)
    e = latent_embed(Wt, y)

    # Accumulator: keys strictly past (W-(p)) plus the null slot.
    kv = acc_keys_values(Wt, e)
    K, V = kv[..., :d], kv[..., d:]
    q = linear(rmsnorm(h, _w(Wt, "acc.gq")), _w(Wt, "acc.Wq"))
    bias = _w(Wt, "acc.bias")
    slots = []
    for n, (a, b) in enumerate(acc_slots(cfg)):
        Ks, valid = _shift(K, a, b)
        Vs, _ = _shift(V, a, b)
        slots.append((Ks, Vs, valid & _step_mask(cfg, H, W, a, b, True), bias[:, n]))
    knull = np.broadcast_to(_w(Wt, "acc.knull"), (H, W, d))
    vnull = np.broadcast_to(_w(Wt, "acc.vnull"), (H, W, d))
    slots.append((knull, vnull, np.ones((H, W), bool), np.zeros(heads)))
    x = h + linear(_windowed_attention(q, slots, heads), _w(Wt, "acc.Wo"))
    if keep:
        out["h"], out["x0"] = h, x

    e_prev = None
    if prev is not None:
        e_prev = [latent_embed(Wt, prev[t]) for t in range(2)]

    n_sp = len(layer_slots(cfg))
    for l in range(cfg.L):
        p = f"layer{l}."
        u = rmsnorm(x, _w(Wt, p + "g1"))
        qkv = linear(u, _w(Wt, p + "Wqkv"))
        q, k, v = qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:]
        bias = _w(Wt, p + "bias")
        slots = []
        for n, (a, b) in enumerate(layer_slots(cfg)):
            Ks, valid = _shift(k, a, b)
            Vs, _ = _shift(v, a, b)
            slots.append((Ks, Vs, valid & _step_mask(cfg, H, W, a, b, False), bias[:, n]))
        if e_prev is not None:
            tkv = [temporal_keys_values(Wt, l, e_prev[t]) for t in range(2)]
            for n, (tau, a, b) in enumerate(temporal_window(r)):
                Ks, valid = _shift(tkv[tau - 1][..., :d], a, b)
                Vs, _ = _shift(tkv[tau - 1][..., d:], a, b)
                slots.append((Ks, Vs, valid, bias[:, n_sp + n]))
        att = _windowed_attention(q, slots, heads)
        yres = x + linear(att, _w(Wt, p + "Wo"))
        vn = rmsnorm(yres, _w(Wt, p + "g2"))
        mlp = silu(linear(vn, _w(Wt, p + "Wgate"))) * linear(vn, _w(Wt, p + "Wup"))
        x = yres + linear(mlp, _w(Wt, p + "Wdown"))
        if keep:
            out[f"x{l + 1}"] = x

    out.update(ct_head(cfg, Wt, x, y) if cfg.ch_groups else head(cfg, Wt, x))
    return out


def group_rmsnorm(x, g, N):
    """RMSNorm of each of the N equal channel groups of x on its own."""
    sh = x.shape
    xg = x.reshape(sh[:-1] + (N, sh[-1] // N))
    out = xg / np.sqrt((xg * xg).mean(-1, keepdims=True) + EPS)
    return out.reshape(sh) * g


def group_mask(rows: int, cols: int, N: int) -> np.ndarray:
    """[rows, cols] 0/1 mask, block (g, j) of N x N blocks set for j <= g."""
    gi = np.arange(rows) // (rows // N)
    gj = np.arange(cols) // (cols // N)
    return (gj[None, :] <= gi[:, None]).astype(np.float64)


def ct_head(cfg, Wt, x, y):
    """Channel Transformer and grouped heads (definition form, every
    position and group at once): mean, scale and log-scale of every symbol.
    x: the spatial network's output [..., d]; y: the decoded latent [..., C]
    (group g's prediction reads its groups 0 .. g-1 only)."""
    N, C = cfg.ch_groups, cfg.C
    dc = cfg.ch_d
    dg, Cg = dc // N, C // N
    xs = rmsnorm(x, _w(Wt, "ct.gx"))
    ys = np.asarray(y, dtype=np.float64) * _w(Wt, "ct.gy")
    sy = np.zeros_like(ys)
    sy[..., Cg:] = ys[..., :C - Cg]  # channel shift by one group
    c = linear(xs, _w(Wt, "ct.Wx")) + linear(sy, _w(Wt, "ct.Wy") * group_mask(dc, C, N))
    mask = group_mask(dc, dc, N)
    for b in range(cfg.ch_L):
        p = f"ct{b}."
        c = c + linear(group_rmsnorm(c, _w(Wt, p + "g1"), N), _w(Wt, p + "M") * mask)
        v = group_rmsnorm(c, _w(Wt, p + "g2"), N)
        Wg, Wu, Wd = _w(Wt, p + "Wgate"), _w(Wt, p + "Wup"), _w(Wt, p + "Wdown")
        parts = []
        for g in range(N):
            vg = v[..., g * dg:(g + 1) * dg]
            parts.append(linear(silu(linear(vg, Wg[g])) * linear(vg, Wu[g]), Wd[g]))
        c = c + np.concatenate(parts, axis=-1)
    z = group_rmsnorm(c, _w(Wt, "ctH.g"), N)
    W1, W2 = _w(Wt, "ctH.W1"), _w(Wt, "ctH.W2")
    mu = np.empty(x.shape[:-1] + (C,))
    raw = np.empty(x.shape[:-1] + (C,))
    for g in range(N):
        t = linear(silu(linear(z[..., g * dg:(g + 1) * dg], W1[g])), W2[g])
        mu[..., g * Cg:(g + 1) * Cg] = t[..., :Cg]
        raw[..., g * Cg:(g + 1) * Cg] = t[..., Cg:]
    mu = _w(Wt, "head.gmu") * mu + _w(Wt, "head.bmu")
    lsig = np.clip(_w(Wt, "head.gsig") * raw + _w(Wt, "head.bsig"), LN_SIGMA_MIN, LN_SIGMA_MAX)
    return {"mu": mu, "sigma": np.exp(lsig), "lsig": lsig}


def head(cfg, Wt, x):
    """mu = g_mu * t[:C] + b_mu; lsig = clamp(g_sig * t[C:] + b_sig);
    sigma = exp(lsig), with t = W2 SiLU(W1 RMSNorm(x))."""
    C = cfg.C
    zf = rmsnorm(x, _w(Wt, "head.g"))
    t = linear(silu(linear(zf, _w(Wt, "head.W1"))), _w(Wt, "head.W2"))
    mu = _w(Wt, "head.gmu") * t[..., :C] + _w(Wt, "head.bmu")
    lsig = np.clip(_w(Wt, "head.gsig") * t[..., C:] + _w(Wt, "head.bsig"),
                   LN_SIGMA_MIN, LN_SIGMA_MAX)
    return {"mu": mu, "sigma": np.exp(lsig), "lsig": lsig}


# --------------------------------------------------------------------------
# Sequential form: positions decoded group by group from caches
# --------------------------------------------------------------------------

def forward_sequential(cfg, Wt, y, z, groups, prev=None, on_group=None):
    """Decode in the given order and return dict(mu, sigma, lsig).

    groups: list of int arrays [n, 2] of (i, j). Each group is predicted at
    once from caches filled by earlier groups only; every cell the
    accumulator may see must have been decoded in an earlier group, and
    every cell a layer may see must be decoded or in the same group
    (checked); each group's own latents are read only after its prediction.
    This is the decoder's view: it never touches y of undecoded positions.
    on_group(grp, prediction, channels), if given, runs after a group is
    predicted and before its latents are read (prediction: dict(mu, sigma,
    lsig) of the group's rows, final for the `channels` slice: all channels,
    or one channel group at a time for a Channel Transformer); it may write
    y at the group's positions and those channels."""
    H, W, C = y.shape
    d, heads, r, L = cfg.d, cfg.heads, cfg.r, cfg.L
    dh = d // heads
    decoded = np.zeros((H, W), dtype=bool)
    acc_cache = np.full((H, W, 2 * d), np.nan)
    kv_cache = np.full((L, H, W, 2 * d), np.nan)
    h_all = hyper_tokens(Wt, z, H, W)
    res = {k: np.full((H, W, C), np.nan) for k in ("mu", "sigma", "lsig")}

    tkv = None
    if prev is not None:
        e_prev = [latent_embed(Wt, prev[t]) for t in range(2)]
        tkv = [[temporal_keys_values(Wt, l, e_prev[t]) for t in range(2)]
               for l in range(L)]

    cw, lw, tw = acc_slots(cfg), layer_slots(cfg), temporal_window(r)

    def seen(i, j, a, b, strict):
        # in the frame and, for the cyclic schedule, decoded early enough
        if not (0 <= i + a < H and 0 <= j + b < W):
            return False
        if not cfg.cycle:
            return True
        sp, sq = cyclic_step(i, j, cfg.cycle), cyclic_step(i + a, j + b, cfg.cycle)
        return sq < sp if strict else sq <= sp

    def attend(qv, keys, vals, biases):
        # qv [d]; keys/vals [n, d]; biases [n, heads]
        o = np.empty(d)
        for m in range(heads):
            sl = slice(m * dh, (m + 1) * dh)
            lg = keys[:, sl] @ qv[sl] / math.sqrt(dh) + biases[:, m]
            w = np.exp(lg - lg.max())
            w /= w.sum()
            o[sl] = w @ vals[:, sl]
        return o

    for grp in groups:
        grp = np.asarray(grp).reshape(-1, 2)
        in_grp = np.zeros((H, W), dtype=bool)
        in_grp[grp[:, 0], grp[:, 1]] = True
        for i, j in grp:
            for a, b in cw:
                if seen(i, j, a, b, True):
                    assert decoded[i + a, j + b], "order violates the mask"
            for a, b in lw:
                if seen(i, j, a, b, False):
                    assert decoded[i + a, j + b] or in_grp[i + a, j + b], \
                        "order violates the layer mask"
        n = len(grp)
        gi, gj = grp[:, 0], grp[:, 1]
        h = h_all[gi, gj]
        # Accumulator over decoded neighbours + null slot.
        q = linear(rmsnorm(h, _w(Wt, "acc.gq")), _w(Wt, "acc.Wq"))
        bias = _w(Wt, "acc.bias")
        att = np.empty((n, d))
        for g, (i, j) in enumerate(grp):
            ks, vs, bs = [], [], []
            for s_, (a, b) in enumerate(cw):
                if seen(i, j, a, b, True):
                    ks.append(acc_cache[i + a, j + b, :d])
                    vs.append(acc_cache[i + a, j + b, d:])
                    bs.append(bias[:, s_])
            ks.append(_w(Wt, "acc.knull"))
            vs.append(_w(Wt, "acc.vnull"))
            bs.append(np.zeros(heads))
            att[g] = attend(q[g], np.array(ks), np.array(vs), np.array(bs))
        x = h + linear(att, _w(Wt, "acc.Wo"))
        for l in range(L):
            p = f"layer{l}."
            qkv = linear(rmsnorm(x, _w(Wt, p + "g1")), _w(Wt, p + "Wqkv"))
            kv_cache[l, gi, gj] = qkv[:, d:]
            bias = _w(Wt, p + "bias")
            att = np.empty((n, d))
            for g, (i, j) in enumerate(grp):
                ks, vs, bs = [], [], []
                for s_, (a, b) in enumerate(lw):
                    if seen(i, j, a, b, False):
                        ks.append(kv_cache[l, i + a, j + b, :d])
                        vs.append(kv_cache[l, i + a, j + b, d:])
                        bs.append(bias[:, s_])
                if tkv is not None:
                    for s_, (tau, a, b) in enumerate(tw):
                        if 0 <= i + a < H and 0 <= j + b < W:
                            ks.append(tkv[l][tau - 1][i + a, j + b, :d])
                            vs.append(tkv[l][tau - 1][i + a, j + b, d:])
                            bs.append(bias[:, len(lw) + s_])
                att[g] = attend(qkv[g, :d], np.array(ks), np.array(vs),
                                np.array(bs))
            yres = x + linear(att, _w(Wt, p + "Wo"))
            vn = rmsnorm(yres, _w(Wt, p + "g2"))
            mlp = silu(linear(vn, _w(Wt, p + "Wgate"))) * linear(vn, _w(Wt, p + "Wup"))
            x = yres + linear(mlp, _w(Wt, p + "Wdown"))
        if cfg.ch_groups:
            # channel groups one after the other: group g is predicted from
            # the symbols of groups < g of these positions only (the later
            # groups are hidden), then its symbols become known
            Cg = cfg.C // cfg.ch_groups
            for g in range(cfg.ch_groups):
                ys = np.array(y[gi, gj], dtype=np.int64)
                ys[:, g * Cg:] = 0
                hd = ct_head(cfg, Wt, x, ys)
                sl = slice(g * Cg, (g + 1) * Cg)
                for k in res:
                    res[k][gi, gj, sl] = hd[k][:, sl]
                if on_group is not None:
                    on_group(grp, hd, sl)
        else:
            hd = head(cfg, Wt, x)
            for k in res:
                res[k][gi, gj] = hd[k]
            if on_group is not None:
                on_group(grp, hd, slice(0, C))
        # The group's symbols are now decoded: fill the accumulator cache.
        e = latent_embed(Wt, y[gi, gj])
        acc_cache[gi, gj] = acc_keys_values(Wt, e)
        decoded[gi, gj] = True
    assert decoded.all()
    return res


def sample_latents(cfg, Wt, z, noise, prev=None):
    """Latents drawn from the model itself, in decode order: at each
    diagonal the model predicts mu and sigma from the symbols drawn so far,
    and y = rint(mu + sigma * noise) there (noise [H, W, C], given). On such
    data the model is the true source, so its ideal bits approach the
    entropy and errors in mu or sigma show up as rate (test data for the
    precision forms; the method itself never samples)."""
    H, W, C = noise.shape
    y = np.zeros((H, W, C), dtype=np.int32)

    def draw(grp, pred, ch):
        gi, gj = grp[:, 0], grp[:, 1]
        y[gi, gj, ch] = np.rint(pred["mu"][:, ch] + pred["sigma"][:, ch] * noise[gi, gj][:, ch])

    forward_sequential(cfg, Wt, y, z, schedule_groups(cfg, H, W), prev, on_group=draw)
    return y


def raster_order(H, W):
    return [np.array([[i, j]]) for i in range(H) for j in range(W)]


def wavefront_order(H, W, s):
    return diagonals(H, W, s)


def random_topological_order(H, W, r, rng):
    """A random order in which every W-(p) cell precedes p: repeatedly pick
    a random position whose causal neighbours are all decoded."""
    cw = causal_window(r)
    need = np.zeros((H, W), dtype=np.int64)
    dependents = [[[] for _ in range(W)] for _ in range(H)]
    for i in range(H):
        for j in range(W):
            for a, b in cw:
                if 0 <= i + a < H and 0 <= j + b < W:
                    need[i, j] += 1
                    dependents[i + a][j + b].append((i, j))
    ready = [(i, j) for i in range(H) for j in range(W) if need[i, j] == 0]
    order = []
    while ready:
        k = int(rng.integers(len(ready)))
        ready[k], ready[-1] = ready[-1], ready[k]
        i, j = ready.pop()
        order.append(np.array([[i, j]]))
        for (pi, pj) in dependents[i][j]:
            need[pi, pj] -= 1
            if need[pi, pj] == 0:
                ready.append((pi, pj))
    assert len(order) == H * W
    return order
