"""Subproblem solves, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

  dense_solve  the subproblem (ADMMSubProb): (A^T D A + (c + rho) I) x = rhs by
               a dense Cholesky solve.  PCG reaches exactly this point.
  nys_pcg      Algorithm Nystrom PCG, with the factor as an input (NysADMM
               builds it once, before its loop) and the stopping test applied to
               the initial residual as well.

Reading of the stop: ||w||_2 <= tol ||rhs||_2 (relative to the right-hand side,
so a warm start is rewarded); tol_abs=True gives the printed absolute test
||w||_2 <= tol.  rhs = 0 returns x = 0 after 0 iterations.

Pins: dense Cholesky against scipy's LU solve, P = I against scipy's CG,
convergence in 1-2 steps when rank(H) < s, the error rate of Corollary
ADMMSubProb when the preconditioned condition number is <= 8, and the
iteration count of Theorem NysADMMConv.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .nystrom import hessian_dense, hessian_apply, precond_inverse_apply


def dense_solve(A, D, c, rho, rhs):
    Hs = hessian_dense(A, D, c) + rho * np.eye(A.shape[1])
    L = np.linalg.cholesky(Hs)
    z = np.linalg.solve(L, rhs)
    return np.linalg.solve(L.T, z)


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    res_hist: list
    breakdown: bool = False


def nys_pcg(matvec, rhs, x0, precond, tol, max_iter=1000, tol_abs=False,
            track=None) -> PCGResult:
    """Algorithm Nystrom PCG.  `matvec(p)` returns (H + rho I) p, `precond(w)`
    returns P^-1 w (identity when None).  `track(x)` is called after every
    update of x (used by the error-rate pins)."""
    rhs = np.asarray(rhs, dtype=np.float64)
    nr = float(np.linalg.norm(rhs))
    if nr == 0.0:
        return PCGResult(np.zeros_like(rhs), 0, [0.0])
    thr = tol if tol_abs else tol * nr
    Pinv = (lambda v: v) if precond is None else precond
    x = np.array(x0, dtype=np.float64, copy=True)
    w = rhs - matvec(x)
    hist = [float(np.linalg.norm(w))]
    if hist[-1] <= thr:
        return PCGResult(x, 0, hist)
    y = Pinv(w)
    p = y.copy()
    wy = float(w @ y)
    it = 0
    while it < max_iter:
        v = matvec(p)
        pv = float(p @ v)
        if not pv > 0.0:
            return PCGResult(x, it, hist, breakdown=True)
        alpha = wy / pv
        x = x + alpha * p
        w = w - alpha * v
        it += 1
        if track is not None:
            track(x)
        hist.append(float(np.linalg.norm(w)))
        if hist[-1] <= thr:
            break
        y = Pinv(w)
        wy_new = float(w @ y)
        beta = wy_new / wy
        p = y + beta * p
        wy = wy_new
    return PCGResult(x, it, hist)


def subproblem_matvec(A, D, c, rho):
    """p -> (A^T D A + (c + rho) I) p, the operator of (ADMMSubProb)."""
    return lambda p: hessian_apply(A, D, c, p) + rho * p


def nystrom_precond(factor, rho):
    return lambda w: precond_inverse_apply(factor.U, factor.lam, rho, w)
