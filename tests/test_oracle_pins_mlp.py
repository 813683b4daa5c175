"""Pins of the FP64 warm-start network oracle: finite differences, the gelu
derivative identity, and one Adam step in closed form."""
import math

import numpy as np
from scipy.stats import norm

from oracle import mlp


def small():
    m = mlp.init_mlp(6, 9, 4, seed=3)
    r = np.random.default_rng(4)
    # non-zero biases so their gradients are exercised away from 0
    for b in (m.b1, m.b2, m.b3):
        b[:] = 0.1 * r.standard_normal(b.shape)
    X = r.standard_normal((5, 6))
    C = r.standard_normal((5, 4))
    Wt = r.uniform(1.0, 3.0, (5, 4))
    return m, X, C, Wt


def test_gelu_is_x_times_normal_cdf_and_its_derivative():
    a = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(a), a * norm.cdf(a), atol=1e-14)
    assert np.allclose(mlp.gelu_grad(a), norm.cdf(a) + a * norm.pdf(a), atol=1e-14)


def test_gradients_match_central_differences():
    m, X, C, Wt = small()
    L, grads = mlp.loss_and_grads(m, X, C, Wt)
    h = 1e-6
    for P, G in zip(m.params(), grads):
        fd = np.zeros_like(P)
        it = np.nditer(P, flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = P[i]
            P[i] = old + h
            lp = mlp.loss(m, X, C, Wt)
            P[i] = old - h
            lm = mlp.loss(m, X, C, Wt)
            P[i] = old
            fd[i] = (lp - lm) / (2 * h)
        assert np.allclose(G, fd, rtol=1e-6, atol=1e-8)


def test_adam_first_step_closed_form():
    # after one step with bias correction, m_hat = g and v_hat = g^2, so the
    # update is lr * g / (|g| + eps) (Kingma & Ba, Algorithm 1)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 0.0])]
    opt = mlp.Adam(lr=0.1, eps=1e-8)
    opt.step(p, g)
    expect = np.array([1.0, -2.0, 3.0]) - 0.1 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.allclose(p[0], expect, rtol=1e-12, atol=1e-15)


def test_training_reduces_loss_on_a_linear_map():
    # the ideal warm-start map is close to linear: a small net learns one
    r = np.random.default_rng(5)
    M = r.standard_normal((6, 4)) * 0.5
    X = r.standard_normal((256, 6))
    C = X @ M
    Wt = np.ones_like(C)
    m = mlp.init_mlp(6, 32, 4, seed=6)
    opt = mlp.Adam(lr=3e-3)
    l0 = mlp.loss(m, X, C, Wt)
    for _ in range(300):
        L, g = mlp.loss_and_grads(m, X, C, Wt)
        opt.step(m.params(), g)
    assert mlp.loss(m, X, C, Wt) < 0.05 * l0
