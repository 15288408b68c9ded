"""Dense, fully masked re-statement of the context model in torch float64.

Used only to pin the oracle: every token attends to every other token of the
frame through torch's scaled_dot_product_attention, with an additive mask
built from the visibility predicate (relative bias where visible, -inf
elsewhere). Linear layers, RMSNorm and SiLU are torch's own. Nothing here is
shared with the oracle: the window is expressed as a predicate on offsets,
not as an offset list, and the bias slot of an offset comes from a closed
form.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

EPS = 1e-5


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def acc_visible(da, db, r):
    """Key at offset (da, db) from the query is strictly past and inside the
    causal window: one of the r rows above within r columns, or one of the
    r cells to the left."""
    return ((-r <= da <= -1) and abs(db) <= r) or (da == 0 and -r <= db <= -1)


def bias_slot(da, db, r):
    """Closed-form bias slot of a spatial offset (self is slot 2r(r+1))."""
    if da < 0:
        return (da + r) * (2 * r + 1) + (db + r)
    if da == 0 and db < 0:
        return r * (2 * r + 1) + (db + r)
    assert da == 0 and db == 0
    return 2 * r * (r + 1)


def temporal_slot(tau, da, db, r, n_sp=None):
    n_sp = 2 * r * (r + 1) + 1 if n_sp is None else n_sp
    k = 2 * r + 1
    return n_sp + (tau - 1) * k * k + (da + r) * k + (db + r)


# The cyclic schedule (cycle c): key k is visible to the accumulator of query
# p when it lies in the full window and ((i_k + j_k) mod c) < ((i_p + j_p)
# mod c); to a layer when the step is <=. Bias slot: raster index in the
# (2r+1)^2 window.
def cyc_visible(ip, jp, ik, jk, r, c, strict):
    if abs(ik - ip) > r or abs(jk - jp) > r:
        return False
    sp, sk = (ip + jp) % c, (ik + jk) % c
    return sk < sp if strict else sk <= sp


def cyc_slot(da, db, r):
    return (da + r) * (2 * r + 1) + (db + r)


def _rms(x, g):
    return F.rms_norm(x, (x.shape[-1],), weight=g, eps=EPS)


def dense_forward(cfg, Wt, y, z, prev=None):
    H, W, C = y.shape
    d, nh, r = cfg.d, cfg.heads, cfg.r
    dh = d // nh
    N = H * W
    w = {k: _t(v) for k, v in Wt.items()}
    yy = _t(y).reshape(N, C)
    ii = torch.arange(H).repeat_interleave(W)
    jj = torch.arange(W).repeat(H)

    # hyper token: nearest x4 upsampling + sub-position embedding
    zt = _t(z)
    zz = zt[ii // 4, jj // 4]
    h = F.linear(zz, w["hyper.W"]) + w["hyper.P4"][(ii % 4) * 4 + (jj % 4)]

    e = F.linear(yy * w["in.g"], w["in.W"])

    def heads_(x):  # [N', d] -> [nh, N', dh]
        return x.reshape(x.shape[0], nh, dh).transpose(0, 1)

    # accumulator
    kv = F.linear(_rms(e, w["acc.gkv"]), w["acc.Wkv"])
    K = torch.cat([kv[:, :d], w["acc.knull"][None]], 0)
    V = torch.cat([kv[:, d:], w["acc.vnull"][None]], 0)
    q = F.linear(_rms(h, w["acc.gq"]), w["acc.Wq"])
    cyc = getattr(cfg, "cycle", 0)
    mask = torch.full((nh, N, N + 1), -math.inf, dtype=torch.float64)
    mask[:, :, N] = 0.0
    for p in range(N):
        for k in range(N):
            da, db = int(ii[k] - ii[p]), int(jj[k] - jj[p])
            if cyc:
                if cyc_visible(int(ii[p]), int(jj[p]), int(ii[k]), int(jj[k]), r, cyc, True):
                    mask[:, p, k] = w["acc.bias"][:, cyc_slot(da, db, r)]
            elif acc_visible(da, db, r):
                mask[:, p, k] = w["acc.bias"][:, bias_slot(da, db, r)]
    a = F.scaled_dot_product_attention(heads_(q), heads_(K), heads_(V),
                                       attn_mask=mask)
    x = h + F.linear(a.transpose(0, 1).reshape(N, d), w["acc.Wo"])

    e_prev = None
    if prev is not None:
        e_prev = [F.linear(_t(prev[t]).reshape(N, C) * w["in.g"], w["in.W"])
                  for t in range(2)]

    for l in range(cfg.L):
        p_ = f"layer{l}."
        qkv = F.linear(_rms(x, w[p_ + "g1"]), w[p_ + "Wqkv"])
        q, k_, v_ = qkv[:, :d], qkv[:, d:2 * d], qkv[:, 2 * d:]
        Ks, Vs = [k_], [v_]
        if e_prev is not None:
            for t in range(2):
                tkv = F.linear(_rms(e_prev[t], w[p_ + "g1"]), w[p_ + "Wqkv"][d:])
                Ks.append(tkv[:, :d])
                Vs.append(tkv[:, d:])
        K = torch.cat(Ks, 0)
        V = torch.cat(Vs, 0)
        mask = torch.full((nh, N, K.shape[0]), -math.inf, dtype=torch.float64)
        b = w[p_ + "bias"]
        n_sp = (2 * r + 1) ** 2 if cyc else None
        for p in range(N):
            for k in range(N):
                da, db = int(ii[k] - ii[p]), int(jj[k] - jj[p])
                if cyc:
                    if cyc_visible(int(ii[p]), int(jj[p]), int(ii[k]), int(jj[k]), r, cyc, False):
                        mask[:, p, k] = b[:, cyc_slot(da, db, r)]
                elif acc_visible(da, db, r) or (da == 0 and db == 0):
                    mask[:, p, k] = b[:, bias_slot(da, db, r)]
                if e_prev is not None and abs(da) <= r and abs(db) <= r:
                    for t in range(2):
                        mask[:, p, (t + 1) * N + k] = b[:, temporal_slot(t + 1, da, db, r, n_sp)]
        a = F.scaled_dot_product_attention(heads_(q), heads_(K), heads_(V),
                                           attn_mask=mask)
        yr = x + F.linear(a.transpose(0, 1).reshape(N, d), w[p_ + "Wo"])
        vn = _rms(yr, w[p_ + "g2"])
        x = yr + F.linear(F.silu(F.linear(vn, w[p_ + "Wgate"]))
                          * F.linear(vn, w[p_ + "Wup"]), w[p_ + "Wdown"])

    t_ = F.linear(F.silu(F.linear(_rms(x, w["head.g"]), w["head.W1"])), w["head.W2"])
    mu = w["head.gmu"] * t_[:, :C] + w["head.bmu"]
    lsig = torch.clamp(w["head.gsig"] * t_[:, C:] + w["head.bsig"],
                       math.log(0.11), math.log(64.0))
    return {"mu": mu.reshape(H, W, C).numpy(),
            "sigma": torch.exp(lsig).reshape(H, W, C).numpy()}
