"""Inexact (linearized) ADMM with Nystrom PCG for lasso and l1-logistic
regression, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

Follows Algorithm NysADMM (Section 2.3) on top of Algorithm Inexact ADMM
(Section 2.1):
  x-update   PCG on (ADMMSubProb); lasso (eq. 2): rhs = rho (z - u) + A^T b;
             elastic-net style smooth part g = c/2 ||x||^2 shifts the operator
             by c and leaves rhs unchanged (eq. 6 with c = 1 - gamma);
             logistic (eq. 9): t = A x, w = 1/(2 + e^-t + e^t),
             rhs = rho (z - u) + A^T (w t + b - sigma(t))  (= A^T diag(w) q),
             operator A^T diag(w) A + rho I.
  z-update   soft threshold S_{gamma/rho}(x + u)  (Section 2.1, h = gamma||.||_1)
  u-update   u + x - z
  residuals  r_p = x - z, r_d = rho (z_old - z), stop on
             ||r_p|| <= eps_abs + eps_rel max(||x||, ||z||),
             ||r_d|| <= eps_abs + eps_rel ||rho u||   (Section 2.1)
  accuracy   relative KKT residual eta of eq. (31) for lasso; the same form
             with the logistic gradient for logistic regression (our reading)
  schedule   optional eps^{k+1} = sqrt(||r_p^k|| ||r_d^k||) (Section 5 setup),
             absolute on ||w||, starting at 1e-2 ||rhs|| and floored at
             pcg_tol ||rhs|| (our reading).

Comparison form: cg=True runs the x-update by plain CG (no preconditioner,
no sketch) -- inexact ADMM with CG, the first row of Table
t-ComplexityComparison -- with the same stopping rule.

Readings: x = z = u = 0 initially; PCG is warm-started at the previous x; the
returned solution is z (sparse), x is reported too; the logistic model is
linearised at x (as printed); its factor is rebuilt every `resketch_every`
iterations, the weights every iteration.

Pins: orthonormal design (closed form S_gamma(A^T b)), gamma >= ||A^T b||_inf
gives 0, brute force over sign patterns for d <= 8, KKT/subgradient
conditions, the dual certificate rho u = -grad l(z), and for logistic the zero
solution above ||A^T (1/2 - b)||_inf and the weight identity.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

from .nystrom import rand_nys_appx, hessian_apply, precond_inverse_apply
from .pcg import nys_pcg, dense_solve


def soft_threshold(a, k):
    """prox of k ||.||_1: sign(a) max(|a| - k, 0)."""
    return np.sign(a) * np.maximum(np.abs(a) - k, 0.0)


def lasso_objective(A, b, gamma, x, c=0.0):
    r = A @ x - b
    return 0.5 * float(r @ r) + 0.5 * c * float(x @ x) + gamma * float(np.abs(x).sum())


def kkt_eta_lasso(A, b, gamma, x):
    """eq. (31)."""
    r = A @ x - b
    g = A.T @ r
    num = np.linalg.norm(x - soft_threshold(x - g, gamma))
    return float(num / (1.0 + np.linalg.norm(x) + np.linalg.norm(r)))


def sigmoid(t):
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def logistic_loss(t, b):
    """-sum(b t - log(1 + e^t)), evaluated stably."""
    return float(np.sum(np.log1p(np.exp(-np.abs(t))) + np.maximum(t, 0.0) - b * t))


def logistic_objective(A, b, gamma, x):
    return logistic_loss(A @ x, b) + gamma * float(np.abs(x).sum())


def logistic_weights(t, b):
    """w_i = 1/(2 + e^-t_i + e^t_i) = sigma(t)(1 - sigma(t)) and the right-hand
    side vector s = w q = w t + b - sigma(t) of Section 3.2 (formed without the
    division by w)."""
    sig = sigmoid(t)
    w = sig * sigmoid(-t)
    return w, w * t + b - sig


def kkt_eta_logistic(A, b, gamma, x):
    g = A.T @ (sigmoid(A @ x) - b)
    num = np.linalg.norm(x - soft_threshold(x - g, gamma))
    return float(num / (1.0 + np.linalg.norm(x) + np.linalg.norm(g)))


def rel_change_inf(z_old, z):
    """||z - z_old||_inf / ||z_old||_inf, the relative change of the iterate
    used as the stopping rule of the logistic experiments (Section 5); None
    when z_old = 0 (the rule cannot fire)."""
    den = float(np.abs(z_old).max())
    if den == 0.0:
        return None
    return float(np.abs(z - z_old).max()) / den


@dataclasses.dataclass
class ADMMResult:
    x: np.ndarray
    z: np.ndarray
    u: np.ndarray
    iters: int
    pcg_iters: list
    r_p: list
    r_d: list
    converged: bool = False
    factor: object = None
    tols: list = dataclasses.field(default_factory=list)   # absolute PCG tolerance per step
    z_hist: list = None                                     # z after each step (record=True)


def _stop(r_p, r_d, x, z, u, rho, eps_abs, eps_rel):
    if eps_abs is None or eps_rel is None:
        return False
    tp = eps_abs + eps_rel * max(np.linalg.norm(x), np.linalg.norm(z))
    td = eps_abs + eps_rel * np.linalg.norm(rho * u)
    return r_p <= tp and r_d <= td


def admm_lasso(A, b, gamma, rho, omega_raw=None, c=0.0, iters=300, pcg_tol=1e-8,
               exact=False, factor=None, eps_abs=None, eps_rel=None,
               tol_schedule=False, state=None, mantissa_bits=52,
               pcg_max_iter=1000, cg=False, record=False) -> ADMMResult:
    """Algorithm NysADMM for min 1/2||Ax - b||^2 + c/2||x||^2 + gamma||x||_1
    (cg=True: inexact ADMM with plain CG)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = A.shape[1]
    if not exact and not cg and factor is None:
        factor = rand_nys_appx(A, None, c, omega_raw, mantissa_bits)
    if state is None:
        x, z, u = np.zeros(d), np.zeros(d), np.zeros(d)
    else:
        x, z, u = (np.array(v, dtype=np.float64) for v in state)
    Atb = A.T @ b
    chol = None
    if exact:   # the subproblem matrix is constant for least squares: factor once
        chol = sla.cho_factor(A.T @ A + (c + rho) * np.eye(d))
    matvec = lambda p: hessian_apply(A, None, c, p) + rho * p
    precond = None if (exact or cg) else (
        lambda w: precond_inverse_apply(factor.U, factor.lam, rho, w))
    its, rps, rds, tols = [], [], [], []
    zh = [] if record else None
    eps_k = None
    converged = False
    for k in range(iters):
        rhs = rho * (z - u) + Atb
        if exact:
            x = sla.cho_solve(chol, rhs)
            its.append(0)
        else:
            nr = np.linalg.norm(rhs)
            if tol_schedule:
                tol_abs_val = 1e-2 * nr if eps_k is None else max(eps_k, pcg_tol * nr)
                res = nys_pcg(matvec, rhs, x, precond, tol_abs_val, pcg_max_iter, tol_abs=True)
                tols.append(tol_abs_val)
            else:
                res = nys_pcg(matvec, rhs, x, precond, pcg_tol, pcg_max_iter)
                tols.append(pcg_tol * nr)
            x = res.x
            its.append(res.iters)
        z_old = z
        z = soft_threshold(x + u, gamma / rho)
        u = u + x - z
        r_p = float(np.linalg.norm(x - z))
        r_d = float(rho * np.linalg.norm(z_old - z))
        rps.append(r_p)
        rds.append(r_d)
        if record:
            zh.append(z.copy())
        eps_k = math.sqrt(r_p * r_d)
        if _stop(r_p, r_d, x, z, u, rho, eps_abs, eps_rel):
            converged = True
            break
    return ADMMResult(x, z, u, len(its), its, rps, rds, converged, factor, tols, zh)


def admm_logistic(A, b, gamma, rho, omega_raw=None, iters=100, pcg_tol=1e-6,
                  resketch_every=10, exact=False, rel_change_tol=None, state=None,
                  mantissa_bits=52, pcg_max_iter=1000, cg=False, record=False) -> ADMMResult:
    """Linearised NysADMM for min -sum(b_i t_i - log(1 + e^t_i)) + gamma||x||_1,
    t = A x, labels b in {0, 1} (cg=True: inexact ADMM with plain CG)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = A.shape[1]
    if state is None:
        x, z, u = np.zeros(d), np.zeros(d), np.zeros(d)
    else:
        x, z, u = (np.array(v, dtype=np.float64) for v in state)
    factor = None
    its, rps, rds = [], [], []
    zh = [] if record else None
    converged = False
    for k in range(iters):
        t = A @ x
        w, s = logistic_weights(t, b)
        rhs = rho * (z - u) + A.T @ s
        if exact:
            x = dense_solve(A, w, 0.0, rho, rhs)
            its.append(0)
        else:
            if not cg and (factor is None or (resketch_every and k % resketch_every == 0)):
                factor = rand_nys_appx(A, w, 0.0, omega_raw, mantissa_bits)
            matvec = lambda p, w=w: hessian_apply(A, w, 0.0, p) + rho * p
            precond = None if cg else (
                lambda v, f=factor: precond_inverse_apply(f.U, f.lam, rho, v))
            res = nys_pcg(matvec, rhs, x, precond, pcg_tol, pcg_max_iter)
            x = res.x
            its.append(res.iters)
        z_old = z
        z = soft_threshold(x + u, gamma / rho)
        u = u + x - z
        rps.append(float(np.linalg.norm(x - z)))
        rds.append(float(rho * np.linalg.norm(z_old - z)))
        if record:
            zh.append(z.copy())
        if rel_change_tol is not None and k > 0:
            ch = rel_change_inf(z_old, z)
            if ch is not None and ch < rel_change_tol:
                converged = True
                break
    return ADMMResult(x, z, u, len(its), its, rps, rds, converged, factor, None, zh)
