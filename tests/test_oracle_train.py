"""Pins of the distillation oracle (oracle/train.py), CPU only.

* the torch float64 forward equals the numpy oracle forward (I and P);
* autograd gradients equal central finite differences of the loss computed
  through the numpy oracle, along a random direction in every tensor;
* teacher == student gives zero loss and zero gradient;
* where the log-scale clamp is active its gradient vanishes;
* adamw_step equals torch.optim.AdamW (a library routine) over several steps.
"""
import numpy as np
import pytest

import synth
from oracle import model as om

torch = pytest.importorskip("torch")
from oracle import train as ot  # noqa: E402

CFG = synth.ModelCfg(L=2, d=32, heads=2, window=5, mlp_ratio=2, C=8, Ch=4)


def _crop(seed, H=6, W=7, n_prev=0):
    y, z, prev = synth.frame_inputs(CFG, synth.FrameCfg(H, W, n_prev), seed)
    return {"latents": y, "hyper": z, "prev": prev}


def _labelled(Wt_teacher, crops):
    out = []
    for c in crops:
        o = om.forward(CFG, Wt_teacher, c["latents"], c["hyper"], c["prev"])
        out.append(dict(c, mu_t=o["mu"], lsig_t=o["lsig"]))
    return out


@pytest.mark.parametrize("n_prev", [0, 2])
def test_torch_forward_equals_numpy_oracle(n_prev):
    Wt = synth.model_weights(CFG, 3)
    c = _crop(10 + n_prev, n_prev=n_prev)
    P = {k: torch.as_tensor(v, dtype=torch.float64) for k, v in Wt.items()}
    mu, ls = ot.forward(CFG, P, c["latents"], c["hyper"], c["prev"])
    o = om.forward(CFG, Wt, c["latents"], c["hyper"], c["prev"])
    assert np.allclose(mu.numpy(), o["mu"], rtol=0, atol=1e-11)
    assert np.allclose(ls.numpy(), o["lsig"], rtol=0, atol=1e-11)


def test_gradients_equal_finite_differences():
    teacher = synth.model_weights(CFG, 5)
    Wt = {k: v.astype(np.float64) for k, v in synth.model_weights(CFG, 6).items()}
    batch = _labelled(teacher, [_crop(20, 5, 6, 0), _crop(21, 4, 5, 2)])
    loss, G = ot.loss_and_grads(CFG, Wt, batch)
    assert abs(loss - ot.loss_numpy(CFG, Wt, batch)) < 1e-12 * max(1.0, loss)
    rng = np.random.default_rng(0)
    h = 1e-5
    for name, g in G.items():
        u = rng.standard_normal(g.shape)
        u /= np.linalg.norm(u)
        Wp = dict(Wt)
        Wm = dict(Wt)
        Wp[name] = Wt[name] + h * u
        Wm[name] = Wt[name] - h * u
        fd = (ot.loss_numpy(CFG, Wp, batch) - ot.loss_numpy(CFG, Wm, batch)) / (2 * h)
        an = float((g * u).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (name, fd, an)


def test_teacher_equals_student_gives_zero():
    Wt = synth.model_weights(CFG, 7)
    batch = _labelled(Wt, [_crop(30)])
    loss, G = ot.loss_and_grads(CFG, Wt, batch)
    assert loss < 1e-24
    assert max(np.abs(g).max() for g in G.values()) < 1e-12


def test_clamped_log_scale_has_no_gradient():
    Wt = synth.model_weights(CFG, 8)
    Wt["head.bsig"] = np.full_like(Wt["head.bsig"], 20.0)  # far above ln 64
    batch = _labelled(synth.model_weights(CFG, 9), [_crop(31)])
    _, G = ot.loss_and_grads(CFG, Wt, batch)
    assert np.all(G["head.gsig"] == 0) and np.all(G["head.bsig"] == 0)
    assert np.abs(G["head.gmu"]).max() > 0


def test_adamw_equals_torch():
    rng = np.random.default_rng(1)
    names = ["a.W", "a.g", "b.Wx", "b.bias"]
    W = {n: rng.standard_normal((3, 4)) for n in names}
    m = {n: np.zeros((3, 4)) for n in names}
    v = {n: np.zeros((3, 4)) for n in names}
    tp = {n: torch.tensor(W[n], requires_grad=True) for n in names}
    opt = torch.optim.AdamW([{"params": [tp[n] for n in names if ot.decayed(n)],
                              "weight_decay": 0.05},
                             {"params": [tp[n] for n in names if not ot.decayed(n)],
                              "weight_decay": 0.0}],
                            lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        G = {n: rng.standard_normal((3, 4)) for n in names}
        for n in names:
            tp[n].grad = torch.tensor(G[n])
        opt.step()
        W, m, v = ot.adamw_step(W, G, m, v, t, lr=0.01, wd=0.05)
        for n in names:
            assert np.allclose(W[n], tp[n].detach().numpy(), rtol=0, atol=1e-13), (t, n)
