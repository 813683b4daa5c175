"""Warm-start network, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

Not in the paper: the learned warm start proposes the PCG starting point of
the ADMM x-subproblem in the Nystrom basis, x0 = U c with
c = MLP([U^T rhs, log gamma, log rho]).  The network is
    h1 = gelu(X W1 + b1), h2 = gelu(h1 W2 + b2), out = h2 W3 + b3
with the erf form gelu(a) = a/2 (1 + erf(a / sqrt(2))), rows of X being
samples.  The loss is the energy-weighted squared error
    L = (1/B) sum_i sum_k w_ik (out_ik - c*_ik)^2,   w_ik = (lambda_k + rho_i)/rho_i,
which is, for exact eigenvectors, the error of x0 measured in the norm of
H + rho I (scaled by 1/rho).  Adam follows Kingma & Ba (2015) with bias
correction.

Pins (tests/test_oracle_pins_mlp.py): central finite differences of the loss
with respect to every parameter block, the derivative of gelu against the
textbook identity, and one Adam step against its closed form.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    """d/da of a Phi(a): Phi(a) + a phi(a)."""
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


@dataclasses.dataclass
class MLP:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]


def init_mlp(n_in, hidden, n_out, seed=0):
    """He-style initialisation (scale sqrt(2/fan_in)), zero biases."""
    r = np.random.default_rng(seed)
    return MLP(r.standard_normal((n_in, hidden)) * math.sqrt(2.0 / n_in), np.zeros(hidden),
               r.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden), np.zeros(hidden),
               r.standard_normal((hidden, n_out)) * math.sqrt(2.0 / hidden), np.zeros(n_out))


def forward(m: MLP, X):
    a1 = X @ m.W1 + m.b1
    h1 = gelu(a1)
    a2 = h1 @ m.W2 + m.b2
    h2 = gelu(a2)
    out = h2 @ m.W3 + m.b3
    return out, (X, a1, h1, a2, h2)


def loss(m: MLP, X, C, Wt):
    out, _ = forward(m, X)
    return float(np.sum(Wt * (out - C) ** 2) / X.shape[0])


def loss_and_grads(m: MLP, X, C, Wt):
    out, (X, a1, h1, a2, h2) = forward(m, X)
    B = X.shape[0]
    L = float(np.sum(Wt * (out - C) ** 2) / B)
    g_out = 2.0 * Wt * (out - C) / B
    gW3 = h2.T @ g_out
    gb3 = g_out.sum(axis=0)
    g_h2 = g_out @ m.W3.T
    g_a2 = g_h2 * gelu_grad(a2)
    gW2 = h1.T @ g_a2
    gb2 = g_a2.sum(axis=0)
    g_h1 = g_a2 @ m.W2.T
    g_a1 = g_h1 * gelu_grad(a1)
    gW1 = X.T @ g_a1
    gb1 = g_a1.sum(axis=0)
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]


@dataclasses.dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = None
    v: list = None

    def step(self, params, grads):
        if self.m is None:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        c1 = 1.0 - self.beta1 ** self.t
        c2 = 1.0 - self.beta2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.beta1
            m += (1.0 - self.beta1) * g
            v *= self.beta2
            v += (1.0 - self.beta2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def features(U, rhs, gamma, rho):
    """[U^T rhs, log gamma, log rho] for one subproblem."""
    return np.concatenate([U.T @ rhs, [math.log(gamma), math.log(rho)]])
