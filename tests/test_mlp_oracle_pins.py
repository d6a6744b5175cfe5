"""Pins of the FP64 MLP oracle (learned demapper network), CPU only.

* gradients against central finite differences of the loss (relative error <= 1e-7);
* GELU (tanh form) against the erf form within the approximation's known bound and its
  derivative against finite differences;
* the soft-BCE loss is zero at its target and positive elsewhere (Gibbs), with a zero
  gradient there;
* Adam's first step equals -lr * g / (|g| + eps) element-wise (closed form);
* a few Adam steps on a fixed batch lower the loss.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy.special import erf

import workloads as W
from oracle import mlp


def _tiny(seed=3, D=2, H=5, m=3, B=7):
    g = np.random.default_rng(seed)
    w = {"W1": g.normal(0, 0.7, (D + 1, H)), "b1": g.normal(0, 0.1, H), "W2": g.normal(0, 0.5, (H, H)),
         "b2": g.normal(0, 0.1, H), "W3": g.normal(0, 0.5, (H, m)), "b3": g.normal(0, 0.1, m)}
    X = g.normal(0, 1, (B, D + 1))
    T = g.normal(0, 3, (B, m))
    return w, X, T


def test_gradients_match_finite_differences():
    w, X, T = _tiny()
    out, cache = mlp.forward(w, X)
    g = mlp.backward(w, cache, out, T)
    h = 1e-6
    for k in w:
        flat = w[k].reshape(-1)
        num = np.empty_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(mlp.forward(w, X)[0], T)
            flat[i] = old - h
            lm = mlp.loss(mlp.forward(w, X)[0], T)
            flat[i] = old
            num[i] = (lp - lm) / (2 * h)
        ana = g[k].reshape(-1)
        err = np.max(np.abs(num - ana)) / max(np.max(np.abs(ana)), 1e-12)
        assert err <= 1e-7, (k, err)


def test_gelu_tanh_form_and_derivative():
    x = np.linspace(-6, 6, 2001)
    exact = 0.5 * x * (1 + erf(x / math.sqrt(2)))
    assert np.max(np.abs(mlp.gelu(x) - exact)) < 1e-3  # the tanh form's known accuracy
    h = 1e-6
    num = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(num - mlp.gelu_grad(x))) < 1e-8
    assert mlp.gelu(np.array([0.0]))[0] == 0.0


def test_soft_bce_minimum_at_target():
    g = np.random.default_rng(5)
    T = g.normal(0, 5, (50, 4))
    assert abs(mlp.loss(T, T)) < 1e-12
    for _ in range(5):
        O = T + g.normal(0, 1, T.shape)
        assert mlp.loss(O, T) > 0
    d = mlp.sigmoid(T) - mlp.sigmoid(T)
    assert np.all(d == 0)


def test_adam_first_step_closed_form():
    w, X, T = _tiny()
    out, cache = mlp.forward(w, X)
    g = mlp.backward(w, cache, out, T)
    w0 = {k: v.copy() for k, v in w.items()}
    mlp.adam_step(w, g, {}, lr=1e-3, step=1)
    for k in w:
        expect = w0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(w[k], expect, rtol=0, atol=1e-15)


def test_training_lowers_the_loss():
    w, X, _ = _tiny(B=64)
    teacher, _, _ = _tiny(seed=11)
    T = 4.0 * mlp.forward(teacher, X)[0]  # learnable targets
    state = {}
    l0 = mlp.loss(mlp.forward(w, X)[0], T)
    for step in range(1, 201):
        out, cache = mlp.forward(w, X)
        mlp.adam_step(w, mlp.backward(w, cache, out, T), state, lr=1e-2, step=step)
    assert mlp.loss(mlp.forward(w, X)[0], T) < 0.5 * l0


def test_seeded_initial_weights_shapes():
    w = W.mlp_init_weights(8, 256, 11)
    assert w["W1"].shape == (9, 256) and w["W2"].shape == (256, 256) and w["W3"].shape == (256, 11)
    assert all(v.dtype == np.float32 for v in w.values())
    assert np.all(w["b1"] == 0) and abs(float(np.max(np.abs(w["W2"]))) - 0.5 * math.sqrt(6 / 256)) < 1e-3
    w2 = W.mlp_init_weights(8, 256, 11)
    assert all(np.array_equal(w[k], w2[k]) for k in w)


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -2.5, 3.0e38, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 2.9993e38, 0.0])
    got = mlp.bf16_round(vals)
    assert np.all(np.abs(got[:5] - want[:5]) == 0.0)
    assert abs(got[5] / 3.0e38 - 1.0) < 2.0 ** -8 and got[6] == 0.0
    # every output is representable: 8 significant bits
    x = np.random.default_rng(0).normal(0, 10, 1000)
    r = mlp.bf16_round(x)
    m, e = np.frexp(r)
    assert np.all(m * 256 == np.round(m * 256))
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_stored_rounding_hooks_reduce_to_the_pinned_network():
    w, X, T = _tiny()
    out, cache = mlp.forward(w, X)
    out2, cache2 = mlp.forward_stored(w, X, rnd=mlp.identity)
    assert np.array_equal(out, out2)
    g = mlp.backward(w, cache, out, T)
    g2 = mlp.backward_stored(w, cache2, out2, T, rnd=mlp.identity)
    for k in g:
        assert np.array_equal(g[k], g2[k]), k
    # with BF16 storage the result moves by about the BF16 resolution, not more
    out3, _ = mlp.forward_stored(w, X)
    assert 0 < np.max(np.abs(out3 - out)) < 0.05 * np.max(np.abs(out))


def _torch_net(w, X, T):
    """The same network and loss written with torch's own library routines (float64, CPU):
    torch.nn.functional.gelu(approximate="tanh"), matmul, binary_cross_entropy_with_logits."""
    import torch
    import torch.nn.functional as F
    tw = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    x = torch.tensor(X, dtype=torch.float64)
    t = torch.tensor(T, dtype=torch.float64)
    a1 = F.gelu(x @ tw["W1"] + tw["b1"], approximate="tanh")
    a2 = F.gelu(a1 @ tw["W2"] + tw["b2"], approximate="tanh")
    out = a2 @ tw["W3"] + tw["b3"]
    p = torch.sigmoid(t)
    # soft BCE minus its minimum (the entropy of p), averaged over samples and bits
    loss = (F.binary_cross_entropy_with_logits(out, p, reduction="none")
            - F.binary_cross_entropy_with_logits(t, p, reduction="none")).mean()
    loss.backward()
    return out.detach().numpy(), loss.item(), {k: v.grad.numpy() for k, v in tw.items()}


def test_forward_loss_and_gradients_match_torch_library_routines():
    w, X, T = _tiny(seed=8, D=3, H=6, m=4, B=9)
    out, cache = mlp.forward(w, X)
    t_out, t_loss, t_grad = _torch_net(w, X, T)
    assert np.max(np.abs(out - t_out)) <= 1e-13 * max(1.0, np.max(np.abs(t_out)))
    assert abs(mlp.loss(out, T) - t_loss) <= 1e-14 * max(1.0, abs(t_loss))
    g = mlp.backward(w, cache, out, T)
    for k in w:
        assert np.max(np.abs(g[k] - t_grad[k])) <= 1e-13 * max(1e-3, np.max(np.abs(t_grad[k]))), k


def test_gelu_tanh_form_known_value():
    # the tanh-form GELU at 1 (as torch's approximate="tanh" gives it): 0.8411919906082768
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8411919906082768) <= 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + 0.15880800939172324) <= 1e-15


def test_adam_several_steps_match_torch_optimizer():
    import torch
    w, X, T = _tiny(seed=13)
    state = {}
    tw = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    opt = torch.optim.Adam(list(tw.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    g = np.random.default_rng(21)
    for step in range(1, 6):  # bias corrections beyond the first step
        grads = {k: g.normal(0, 1e-2 * step, v.shape) for k, v in w.items()}
        mlp.adam_step(w, grads, state, lr=3e-3, step=step)
        opt.zero_grad()
        for k, v in tw.items():
            v.grad = torch.tensor(grads[k], dtype=torch.float64)
        opt.step()
        for k in w:
            assert np.max(np.abs(w[k] - tw[k].detach().numpy())) <= 1e-15, (step, k)


def test_bf16_hi_lo_pair_known_values():
    # x = 1 + 2^-8 + 2^-12: hi rounds up to 1 + 2^-7, x - hi = -15 * 2^-12 is a BF16 value, so the
    # pair represents x exactly while one BF16 word is off by 15 * 2^-12
    x = np.array([1.0 + 2.0 ** -8 + 2.0 ** -12])
    assert mlp.bf16_round(x)[0] == 1.0 + 2.0 ** -7
    assert mlp.bf16x2_round(x)[0] == x[0]
    # in general the pair keeps about 16 significant bits
    v = np.random.default_rng(1).normal(0, 3, 4000).astype(np.float32).astype(np.float64)
    r = mlp.bf16x2_round(v)
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -16)
    assert np.max(np.abs(r - v) / np.abs(v)) > 2.0 ** -20  # and not all 24
