"""Host driver of the learned warm start (data recording, training, arms).

The network, its training step and the candidate/judge inside each ADMM
subproblem all run in libnysadmm (nys_ws_*, admm_step with warm_start); this
module only orders the calls and prepares the training set:

  * record   runs ADMM on a family of subproblems (one fixed A and factor,
             several (b, gamma, rho)) and keeps, per subproblem, the features
             f = [U^T rhs, log gamma, log rho] and the target U^T x of the
             solution, both written on the device by the library;
  * fit      standardises features and targets, weights the squared error by
             (lambda_k + rho) / rho (the error of x0 = U c in the norm of
             H + rho I, up to a constant) and takes Adam steps on minibatches
             in the network's precision (BF16 MFMA products with FP32 master
             weights by default); with a validation set it keeps the weights
             of the best validation loss seen (early stopping: the recorded
             subproblems of one ADMM run are strongly correlated, so a network
             of this size memorises them long before it stops improving on
             new right-hand sides);
  * run_arm  solves a family with one start rule: the previous iterate only,
             the network's proposal judged against it, or the analytic proposal
             U (Lambda + rho I)^-1 U^T rhs judged against it.
"""
from __future__ import annotations

import math
import time
from typing import List, Sequence, Tuple

import torch

from . import nysadmm as N

Family = Tuple[torch.Tensor, float, float]   # (b, gamma, rho)


def record(ctx: N.Context, A: torch.Tensor, F: N.Factor, omega: torch.Tensor,
           families: Sequence[Family], iters: int, pcg=None):
    """ADMM runs of `iters` steps per family; returns (X, T) device tensors of
    shape (len(families) * iters, r + 2) and (..., r)."""
    r = F.info()["rank"]
    d = A.shape[1]
    m = len(families) * iters
    X = torch.empty(m, r + 2, dtype=torch.float64, device=A.device)
    T = torch.empty(m, r, dtype=torch.float64, device=A.device)
    row = 0
    for b, gamma, rho in families:
        prob = N.problem(A, b, gamma)
        st = N.State(d, A.device)
        for _ in range(iters):
            o = N.admm_opts(rho, r, omega, pcg=pcg or N.pcg_opts(tol=1e-6), factor=F,
                            ws_features=X[row], ws_target=T[row])
            N.admm_step(ctx, prob, o, F, st)
            row += 1
    ctx.synchronize()
    return X, T


def init_params(n_in: int, hidden: int, n_out: int, seed: int) -> torch.Tensor:
    """He-style initial weights (scale sqrt(2 / fan_in)), zero biases, flat FP64."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for fi, fo in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        parts.append(torch.randn(fi * fo, generator=g, dtype=torch.float64) * math.sqrt(2.0 / fi))
        parts.append(torch.zeros(fo, dtype=torch.float64))
    return torch.cat(parts)


def _targets(X, T, lam_t, analytic_skip):
    n_out = T.shape[1]
    rho = torch.exp(X[:, -1])
    if analytic_skip:
        T = T - X[:, :n_out] / (lam_t[None, :] + rho[:, None])
    return T, rho


def fit(ctx: N.Context, X: torch.Tensor, T: torch.Tensor, lam: Sequence[float],
        hidden: int = 256, steps: int = 2000, batch: int = 256, lr: float = 1e-3,
        seed: int = 0, log_every: int = 0, analytic_skip: bool = True,
        prec: int = N.NYS_BF16, val=None, val_every: int = 50):
    """Train a warm-start network on (X, T); returns (model, loss history).
    analytic_skip: the network learns c* - (Lambda + rho I)^-1 U^T rhs.
    prec: the network's arithmetic (NYS_BF16, NYS_F32 or NYS_F64).
    val: optional held-out (X, T) rows; the weights with the lowest
    validation loss (checked every val_every steps) are the ones returned."""
    n_in, n_out = X.shape[1], T.shape[1]
    lam_t = torch.as_tensor(list(lam), dtype=torch.float64, device=X.device)
    T, rho = _targets(X, T, lam_t, analytic_skip)
    mu = X.mean(0)
    sd = X.std(0).clamp_min(1e-12)
    s_out = T.std(0).clamp_min(1e-30)
    Tn = (T / s_out).contiguous()
    W = (lam_t[None, :] + rho[:, None]) / rho[:, None] * (s_out[None, :] ** 2)
    wscale = W.mean()
    W = (W / wscale).contiguous()
    if val is not None:
        Xv = val[0].contiguous()
        Tv, rv = _targets(Xv, val[1], lam_t, analytic_skip)
        Tvn = (Tv / s_out).contiguous()
        Wv = ((lam_t[None, :] + rv[:, None]) / rv[:, None] * (s_out[None, :] ** 2) /
              wscale).contiguous()
    params = init_params(n_in, hidden, n_out, seed)
    if analytic_skip:
        # start close to the analytic proposal: small last layer
        w3 = n_in * hidden + hidden + hidden * hidden + hidden
        params[w3:w3 + hidden * n_out] *= 0.01
    model = N.WarmStart(ctx, n_in, hidden, n_out, params, mu.cpu(), sd.cpu(), s_out.cpu(),
                        analytic_skip=analytic_skip)
    if prec != N.NYS_F64:
        model.set_precision(prec)
    g = torch.Generator().manual_seed(seed + 1)
    m = X.shape[0]
    hist = []
    perm = torch.randperm(m, generator=g)
    pos = 0
    best = (math.inf, None, -1)
    if val is not None:
        # the untrained network (close to the analytic start) is a candidate too
        lv, _ = model.loss_grad(Xv, Tvn, Wv, want_grad=False)
        best = (lv, model.params(), -1)
    for k in range(steps):
        if pos + batch > m:
            perm = torch.randperm(m, generator=g)
            pos = 0
        idx = perm[pos:pos + batch].to(X.device)
        pos += batch
        loss = model.train_step(X[idx].contiguous(), Tn[idx].contiguous(), W[idx].contiguous(),
                                lr=lr)
        if log_every and (k % log_every == 0 or k == steps - 1):
            hist.append((k, loss))
        if val is not None and (k % val_every == val_every - 1 or k == steps - 1):
            lv, _ = model.loss_grad(Xv, Tvn, Wv, want_grad=False)
            if lv < best[0]:
                best = (lv, model.params(), k)
    if val is not None and best[1] is not None:
        # the weights of the best validation loss, in the same precision
        model.close()
        model = N.WarmStart(ctx, n_in, hidden, n_out, best[1], mu.cpu(), sd.cpu(), s_out.cpu(),
                            analytic_skip=analytic_skip)
        if prec != N.NYS_F64:
            model.set_precision(prec)
        model.best_step = best[2]
        model.best_val_loss = best[0]
    return model, hist


def proposals(model, X: torch.Tensor, lam: Sequence[float]) -> torch.Tensor:
    """Coefficients c the model proposes for feature rows X (as in admm_step)."""
    r = model.n_out
    o = model.forward(X.contiguous()) * model.out_scale.to(X.device)
    if model.analytic_skip:
        lam_t = torch.as_tensor(list(lam), dtype=torch.float64, device=X.device)
        o = o + X[:, :r] / (lam_t[None, :] + torch.exp(X[:, -1])[:, None])
    return o


def analytic(X: torch.Tensor, lam: Sequence[float]) -> torch.Tensor:
    """(Lambda + rho I)^-1 U^T rhs for feature rows X."""
    r = X.shape[1] - 2
    lam_t = torch.as_tensor(list(lam), dtype=torch.float64, device=X.device)
    return X[:, :r] / (lam_t[None, :] + torch.exp(X[:, -1])[:, None])


def energy_error(C: torch.Tensor, X: torch.Tensor, T: torch.Tensor, lam: Sequence[float]) -> float:
    """Mean over rows of sum_k (lambda_k + rho)(c_k - c*_k)^2 / sum_k (lambda_k + rho) c*_k^2:
    the relative error of x0 = U c in the norm of H + rho I restricted to span(U)."""
    lam_t = torch.as_tensor(list(lam), dtype=torch.float64, device=X.device)
    w = lam_t[None, :] + torch.exp(X[:, -1])[:, None]
    num = (w * (C - T) ** 2).sum(1)
    den = (w * T ** 2).sum(1).clamp_min(1e-300)
    return float((num / den).mean())


def run_arm(ctx: N.Context, A: torch.Tensor, F: N.Factor, omega: torch.Tensor,
            families: Sequence[Family], iters: int, arm: str, model=None, pcg=None,
            every_step: bool = False):
    """Solve every family for `iters` ADMM steps with one start rule
    ("prev", "mlp" or "analytic"; the candidate is judged at the first step of
    each run, or at every step); returns totals and the final z of each."""
    r = F.info()["rank"]
    d = A.shape[1]
    tot = {"arm": arm, "solves": 0, "pcg_iters": 0, "ws_used": 0, "first_iters": 0}
    zs: List[torch.Tensor] = []
    ctx.synchronize()
    t0 = time.perf_counter()
    for b, gamma, rho in families:
        prob = N.problem(A, b, gamma)
        st = N.State(d, A.device)
        for k in range(iters):
            o = N.admm_opts(rho, r, omega, pcg=pcg or N.pcg_opts(tol=1e-6), factor=F,
                            warm_start=model if arm == "mlp" else None,
                            ws_analytic=(arm == "analytic"), ws_every_step=every_step)
            _, info = N.admm_step(ctx, prob, o, F, st)
            tot["solves"] += 1
            tot["pcg_iters"] += info.pcg_iters
            tot["ws_used"] += info.ws_used
            if k == 0:
                tot["first_iters"] += info.pcg_iters
        zs.append(st.z.clone())
    ctx.synchronize()
    tot["seconds"] = time.perf_counter() - t0
    return tot, zs
