"""The warm-start network in FP32 and BF16 (MFMA matrix products, FP32
accumulation, FP32 master weights) against the FP64 oracle network at equal
weights and batch.

Bars: outputs and loss within 1e-5 (FP32) / 2e-2 (BF16) relative; every
parameter block's gradient within 1e-4 (FP32) / 2e-2 (BF16) relative in norm;
three FP32 Adam steps on the master weights equal to the oracle's Adam steps
to FP32 rounding; BF16 training lowers the loss like FP64 training does.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as om

pytestmark = pytest.mark.gpu
DEV = "cuda"

SHAPES = [(18, 32, 16, 37), (130, 256, 128, 300)]
BARS = {"f32": (1e-5, 1e-4), "bf16": (2e-2, 2e-2)}


@pytest.fixture(scope="module")
def N():
    from paper_2202_11599_amd import nysadmm
    return nysadmm


@pytest.fixture(scope="module")
def ctx(N):
    c = N.Context()
    yield c
    c.close()


def oracle_net(n_in, hidden, n_out, seed):
    m = om.init_mlp(n_in, hidden, n_out, seed=seed)
    r = np.random.default_rng(seed + 100)
    for b in (m.b1, m.b2, m.b3):
        b[:] = 0.1 * r.standard_normal(b.shape)
    return m


def flat(m):
    return np.concatenate([p.reshape(-1) for p in m.params()])


def make_data(n_in, n_out, batch, seed):
    r = np.random.default_rng(seed)
    X = 3.0 + 2.0 * r.standard_normal((batch, n_in))
    T = r.standard_normal((batch, n_out))
    W = r.uniform(0.5, 4.0, (batch, n_out))
    mu = X.mean(0)
    sd = X.std(0) + 0.1
    return X, T, W, mu, sd


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def prec_of(N, name):
    return {"f32": N.NYS_F32, "bf16": N.NYS_BF16}[name]


@pytest.mark.parametrize("name", ["f32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_forward_loss_and_gradients(N, ctx, shape, name):
    ni, h, no, B = shape
    out_bar, grad_bar = BARS[name]
    m = oracle_net(ni, h, no, seed=3)
    X, T, W, mu, sd = make_data(ni, no, B, seed=4)
    net = N.WarmStart(ctx, ni, h, no, flat(m), mu, sd)
    net.set_precision(prec_of(N, name))
    out = net.forward(dev(X)).cpu().numpy()
    ref, _ = om.forward(m, (X - mu) / sd)
    eo = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    loss, g = net.loss_grad(dev(X), dev(T), dev(W))
    L, grads = om.loss_and_grads(m, (X - mu) / sd, T, W)
    g = g.cpu().numpy()
    errs = []
    off = 0
    for q in grads:
        n = q.size
        ref_b = q.reshape(-1)
        errs.append(float(np.linalg.norm(g[off:off + n] - ref_b) / np.linalg.norm(ref_b)))
        off += n
    print(f"[ws {name}] {shape}: output rel err {eo:.2e}, loss {loss:.6e} vs {L:.6e}, gradient "
          f"block rel errs {[f'{e:.1e}' for e in errs]}", flush=True)
    assert eo <= out_bar
    assert abs(loss - L) <= out_bar * abs(L)
    assert max(errs) <= grad_bar
    # the parameters read back are the FP32 master weights
    assert np.abs(net.params().numpy() - flat(m)).max() <= 1e-6 * np.abs(flat(m)).max()
    net.close()


def test_fp32_adam_steps_match_oracle(N, ctx):
    # Adam on the FP32 master weights: three steps fed with the device's own
    # gradients (loss_grad gives the gradient train_step is about to use) move
    # the weights as the oracle's Adam moves an FP64 copy, to FP32 rounding
    ni, h, no, B = 18, 32, 16, 37
    m = oracle_net(ni, h, no, seed=5)
    X, T, W, mu, sd = make_data(ni, no, B, seed=6)
    net = N.WarmStart(ctx, ni, h, no, flat(m), mu, sd)
    net.set_precision(N.NYS_F32)
    shadow = oracle_net(ni, h, no, seed=5)
    opt = om.Adam(lr=1e-2)
    p0 = flat(shadow).copy()
    for _ in range(3):
        _, g = net.loss_grad(dev(X), dev(T), dev(W))
        g = g.cpu().numpy()
        blocks, off = [], 0
        for q in shadow.params():
            blocks.append(g[off:off + q.size].reshape(q.shape))
            off += q.size
        net.train_step(dev(X), dev(T), dev(W), lr=1e-2)
        opt.step(shadow.params(), blocks)
    p = net.params().numpy()
    step = np.abs(flat(shadow) - p0).max()
    diff = np.abs(p - flat(shadow)).max()
    print(f"[ws f32 adam] max param diff {diff:.2e} (largest step {step:.2e})", flush=True)
    assert step > 1e-3
    assert diff <= 1e-6 * max(np.abs(p0).max(), 1.0)
    net.close()


@pytest.mark.parametrize("name", ["f64", "f32", "bf16"])
def test_training_lowers_the_loss(N, ctx, name):
    # a linear target map plus noise: every precision fits it
    ni, h, no, B = 34, 64, 32, 256
    r = np.random.default_rng(7)
    X = r.standard_normal((2048, ni))
    M = r.standard_normal((ni, no)) / np.sqrt(ni)
    T = X @ M + 0.01 * r.standard_normal((2048, no))
    m = om.init_mlp(ni, h, no, seed=8)
    net = N.WarmStart(ctx, ni, h, no, flat(m), X.mean(0), X.std(0))
    if name != "f64":
        net.set_precision(prec_of(N, name))
    Xd, Td = dev(X), dev(T)
    first = net.loss_grad(Xd, Td, None, want_grad=False)[0]
    g = torch.Generator().manual_seed(9)
    for k in range(300):
        idx = torch.randint(0, 2048, (B,), generator=g).to(DEV)
        net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), None, lr=2e-3)
    last = net.loss_grad(Xd, Td, None, want_grad=False)[0]
    print(f"[ws train {name}] loss {first:.3e} -> {last:.3e}", flush=True)
    assert last < 0.05 * first
    net.close()
