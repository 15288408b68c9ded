"""FP64 oracle of the distillation step of the student context model.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The student is the same context model as `oracle.model` with a smaller
shape. It is trained to reproduce the mean and log-scale that the full model
predicts on generated latents (the distillation target of the learned part;
the paper's own models are trained for rate, Sec. 4, which needs data that
is not available here). One training step:

* forward in the parallel form (teacher forcing: every position sees the
  true latents of its causal window, which is exactly what the decoder sees)
  -- the same definition as `oracle.model.forward`, restated here with torch
  float64 tensors so that autograd can differentiate it;
* loss = mean over symbols of (mu_s - mu_t)^2 + mean over symbols of
  (lsig_s - lsig_t)^2, with lsig the clamped log-scale (its gradient is zero
  where the clamp is active);
* gradients by torch autograd (a library primitive used as one step);
* AdamW (Loshchilov and Hutter): m, v moments with bias correction and a
  decoupled weight decay applied to the linear weights only (names whose
  last part starts with "W").

The torch forward is pinned to `oracle.model.forward`, its gradients to
central finite differences of that numpy forward, and `adamw_step` to
torch.optim.AdamW (tests/test_oracle_train.py).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import model as om

EPS = om.EPS
LN_SIGMA_MIN = om.LN_SIGMA_MIN
LN_SIGMA_MAX = om.LN_SIGMA_MAX


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def _rms(x, g):
    return x / torch.sqrt((x * x).mean(-1, keepdim=True) + EPS) * g


def _silu(x):
    return x / (1.0 + torch.exp(-x))


def _lin(x, W):
    return x @ W.T


def _shift(A, da, db):
    """B[i, j] = A[i+da, j+db] inside the frame, zero elsewhere; and the
    validity mask."""
    H, W = A.shape[:2]
    B = torch.zeros_like(A)
    valid = torch.zeros((H, W), dtype=torch.bool)
    i0, i1 = max(0, -da), min(H, H - da)
    j0, j1 = max(0, -db), min(W, W - db)
    if i0 < i1 and j0 < j1:
        B[i0:i1, j0:j1] = A[i0 + da:i1 + da, j0 + db:j1 + db]
        valid[i0:i1, j0:j1] = True
    return B, valid


def _attend(q, slots, heads):
    H, W, d = q.shape
    dh = d // heads
    qh = q.reshape(H, W, heads, dh)
    logits = []
    for K, _, valid, bias in slots:
        lg = (qh * K.reshape(H, W, heads, dh)).sum(-1) / math.sqrt(dh) + bias
        logits.append(torch.where(valid[..., None], lg,
                                  torch.tensor(float("-inf"), dtype=lg.dtype)))
    w = torch.softmax(torch.stack(logits), dim=0)
    out = torch.zeros((H, W, heads, dh), dtype=q.dtype)
    for n, (_, V, _, _) in enumerate(slots):
        out = out + w[n][..., None] * V.reshape(H, W, heads, dh)
    return out.reshape(H, W, d)


def forward(cfg, P, y, z, prev=None):
    """Student (or any) model forward, parallel form, torch float64.

    P: dict name -> float64 tensor (may require grad). Returns (mu, lsig)
    [H, W, C]; the same definition as oracle.model.forward."""
    H, W, C = y.shape
    d, heads, r = cfg.d, cfg.heads, cfg.r
    yf = _t(y)
    ii = torch.arange(H)[:, None]
    jj = torch.arange(W)[None, :]
    zz = _t(z)[ii // 4, jj // 4]
    h = _lin(zz, P["hyper.W"]) + P["hyper.P4"][(ii % 4) * 4 + (jj % 4)]
    e = _lin(yf * P["in.g"], P["in.W"])

    kv = _lin(_rms(e, P["acc.gkv"]), P["acc.Wkv"])
    K, V = kv[..., :d], kv[..., d:]
    q = _lin(_rms(h, P["acc.gq"]), P["acc.Wq"])
    slots = []
    for n, (a, b) in enumerate(om.causal_window(r)):
        Ks, valid = _shift(K, a, b)
        Vs, _ = _shift(V, a, b)
        slots.append((Ks, Vs, valid, P["acc.bias"][:, n]))
    ones = torch.ones((H, W), dtype=torch.bool)
    slots.append((P["acc.knull"].expand(H, W, d), P["acc.vnull"].expand(H, W, d), ones,
                  torch.zeros(heads, dtype=torch.float64)))
    x = h + _lin(_attend(q, slots, heads), P["acc.Wo"])

    e_prev = None
    if prev is not None:
        e_prev = [_lin(_t(prev[t]) * P["in.g"], P["in.W"]) for t in range(2)]
    n_sp = len(om.layer_window(r))
    for l in range(cfg.L):
        p = f"layer{l}."
        qkv = _lin(_rms(x, P[p + "g1"]), P[p + "Wqkv"])
        q, k, v = qkv[..., :d], qkv[..., d:2 * d], qkv[..., 2 * d:]
        slots = []
        for n, (a, b) in enumerate(om.layer_window(r)):
            Ks, valid = _shift(k, a, b)
            Vs, _ = _shift(v, a, b)
            slots.append((Ks, Vs, valid, P[p + "bias"][:, n]))
        if e_prev is not None:
            Wkv = P[p + "Wqkv"][d:]
            tkv = [_lin(_rms(e_prev[t], P[p + "g1"]), Wkv) for t in range(2)]
            for n, (tau, a, b) in enumerate(om.temporal_window(r)):
                Ks, valid = _shift(tkv[tau - 1][..., :d], a, b)
                Vs, _ = _shift(tkv[tau - 1][..., d:], a, b)
                slots.append((Ks, Vs, valid, P[p + "bias"][:, n_sp + n]))
        yres = x + _lin(_attend(q, slots, heads), P[p + "Wo"])
        vn = _rms(yres, P[p + "g2"])
        x = yres + _lin(_silu(_lin(vn, P[p + "Wgate"])) * _lin(vn, P[p + "Wup"]), P[p + "Wdown"])

    zf = _rms(x, P["head.g"])
    t = _lin(_silu(_lin(zf, P["head.W1"])), P["head.W2"])
    mu = P["head.gmu"] * t[..., :C] + P["head.bmu"]
    lsig = torch.clamp(P["head.gsig"] * t[..., C:] + P["head.bsig"], LN_SIGMA_MIN, LN_SIGMA_MAX)
    return mu, lsig


def distill_loss(cfg, P, batch):
    """Mean squared error of mean and log-scale over every symbol of the
    batch: batch = list of dicts with latents, hyper, prev (or None),
    mu_t and lsig_t (the teacher's outputs on that crop)."""
    se_mu, se_ls, n = 0.0, 0.0, 0
    for c in batch:
        mu, ls = forward(cfg, P, c["latents"], c["hyper"], c.get("prev"))
        se_mu = se_mu + ((mu - _t(c["mu_t"])) ** 2).sum()
        se_ls = se_ls + ((ls - _t(c["lsig_t"])) ** 2).sum()
        n += mu.numel()
    return se_mu / n + se_ls / n


def loss_numpy(cfg, Wt, batch):
    """The same loss through the numpy oracle forward (for finite
    differences)."""
    se_mu, se_ls, n = 0.0, 0.0, 0
    for c in batch:
        o = om.forward(cfg, Wt, c["latents"], c["hyper"], c.get("prev"))
        se_mu += ((o["mu"] - c["mu_t"]) ** 2).sum()
        se_ls += ((o["lsig"] - c["lsig_t"]) ** 2).sum()
        n += o["mu"].size
    return se_mu / n + se_ls / n


def loss_and_grads(cfg, Wt, batch):
    """(loss, {name: float64 gradient}) at the weights Wt."""
    P = {k: _t(v).clone().requires_grad_(True) for k, v in Wt.items()}
    loss = distill_loss(cfg, P, batch)
    loss.backward()
    return loss.item(), {k: P[k].grad.numpy().copy() for k in P}


def decayed(name: str) -> bool:
    """Weight decay applies to the linear weights only."""
    return name.split(".")[-1].startswith("W")


def adamw_step(W, G, m, v, t, lr, wd, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW step (t = 1, 2, ...) on dicts of float64 arrays; returns the
    new (W, m, v)."""
    Wn, mn, vn = {}, {}, {}
    for k in W:
        g = np.asarray(G[k], dtype=np.float64)
        mn[k] = beta1 * m[k] + (1.0 - beta1) * g
        vn[k] = beta2 * v[k] + (1.0 - beta2) * g * g
        mhat = mn[k] / (1.0 - beta1 ** t)
        vhat = vn[k] / (1.0 - beta2 ** t)
        w = np.asarray(W[k], dtype=np.float64)
        if decayed(k):
            w = w * (1.0 - lr * wd)
        Wn[k] = w - lr * mhat / (np.sqrt(vhat) + eps)
    return Wn, mn, vn
