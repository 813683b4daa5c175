"""Kernel SVM dual by NysADMM, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

Follows the support vector machine formulation of Section 3 (eq. 8):

    minimize    1/2 x^T diag(b) K diag(b) x - 1^T x
    subject to  x^T b = 0,  0 <= x <= C

split as l(x) = 1/2 x^T H x with H = diag(b) K diag(b), g(x) = -1^T x and h
the indicator of the constraint set, inside Algorithm NysADMM:

  x-update   PCG on (H + rho I) x = rho (z - u) + 1  (the linear g has
             gradient -1 and no curvature; l is quadratic, so the linearised
             model is exact), preconditioned by RandNysAppx of H
  z-update   projection of x + u onto {0 <= z <= C, b^T z = 0}
  u-update   u + x - z

Readings (the paper is silent on them):
  * projection: z(mu) = clip(v - mu b, 0, C) with the multiplier mu chosen so
    that b^T z(mu) = 0; b^T z(mu) is non-increasing in mu (b_i = +-1), found
    by bisection on a bracket where it changes sign, then one secant step on
    the final bracket.
  * stop ("ADMM dual gap 1e-4", as LIBSVM): the duality gap at the feasible z
    between the SVM primal with w = sum_i z_i b_i phi(a_i) and bias beta, and
    the dual:  P = 1/2 z^T H z + C sum_i max(0, 1 - b_i (g_i + beta)),
    D = 1^T z - 1/2 z^T H z, with g = K diag(b) z.  beta is the mean of
    b_i - g_i over the free variables 0 < z_i < C (LIBSVM's rule); with none,
    the midpoint of the interval the bound variables allow.  Relative gap
    (P - D) / (1 + |P|).
  * RBF kernel K_ij = exp(-gamma ||a_i - a_j||^2).

Pins (tests/test_oracle_pins_svm.py): the projection against a general QP
solver; the kernel against scipy's pairwise distances; the solution against
LIBSVM's SMO solver (scikit-learn's SVC on the precomputed kernel): equal dual
objective and decision values; weak duality of the gap and a zero gap at the
optimum; exact-solve and Nystrom-PCG ADMM agree.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .nystrom import nystrom_from_sketch, orthonormalize, precond_inverse_apply, NysFactor
from .pcg import nys_pcg


def rbf_kernel(X, gamma):
    """K_ij = exp(-gamma ||a_i - a_j||^2), rows a_i of X; by the definition,
    one row at a time."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    K = np.empty((n, n))
    for i in range(n):
        diff = X - X[i]
        K[i] = np.exp(-gamma * np.einsum("ij,ij->i", diff, diff))
    return K


def svm_hessian(K, b):
    """H = diag(b) K diag(b)."""
    b = np.asarray(b, dtype=np.float64)
    return (b[:, None] * np.asarray(K, dtype=np.float64)) * b[None, :]


def project(v, b, C, iters=200):
    """Projection of v onto {0 <= z <= C, b^T z = 0}, b_i in {-1, +1}."""
    v = np.asarray(v, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    phi = lambda mu: float(b @ np.clip(v - mu * b, 0.0, C))
    pos, neg = b > 0, b < 0
    # below lo every b = +1 entry sits at C and every b = -1 entry at 0, above
    # hi the reverse; phi(lo) >= 0 >= phi(hi)
    lo = min(np.min(v[pos] - C, initial=0.0), np.min(-v[neg], initial=0.0))
    hi = max(np.max(v[pos], initial=0.0), np.max(C - v[neg], initial=0.0))
    flo, fhi = phi(lo), phi(hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        f = phi(mid)
        if f > 0.0:
            lo, flo = mid, f
        else:
            hi, fhi = mid, f
    # phi is linear on a bracket that holds no breakpoint: one secant step
    mu = lo if flo == fhi else lo + flo * (hi - lo) / (flo - fhi)
    mu = min(max(mu, lo), hi)
    return np.clip(v - mu * b, 0.0, C), mu


@dataclasses.dataclass
class Gap:
    primal: float
    dual: float
    gap: float
    rel: float
    beta: float


def bias(g, b, z, C, tol=0.0):
    """LIBSVM's bias: mean of b_i - g_i over free variables, else the midpoint
    of the interval allowed by the bound ones."""
    free = (z > tol) & (z < C - tol)
    if free.any():
        return float(np.mean(b[free] - g[free]))
    # y_i (g_i + beta) >= 1 at z_i = 0, <= 1 at z_i = C
    r = b - g
    lo_set = ((z <= tol) & (b > 0)) | ((z >= C - tol) & (b < 0))
    hi_set = ((z <= tol) & (b < 0)) | ((z >= C - tol) & (b > 0))
    lo = np.max(r[lo_set]) if lo_set.any() else -np.inf
    hi = np.min(r[hi_set]) if hi_set.any() else np.inf
    if np.isfinite(lo) and np.isfinite(hi):
        return 0.5 * (lo + hi)
    return float(lo if np.isfinite(lo) else (hi if np.isfinite(hi) else 0.0))


def duality_gap(K, b, C, z) -> Gap:
    K = np.asarray(K, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    g = K @ (b * z)                      # decision values without the bias
    zHz = float((b * z) @ g)
    beta = bias(g, b, z, C)
    hinge = float(np.sum(np.maximum(0.0, 1.0 - b * (g + beta))))
    P = 0.5 * zHz + C * hinge
    D = float(np.sum(z)) - 0.5 * zHz
    return Gap(P, D, P - D, (P - D) / (1.0 + abs(P)), beta)


def dual_objective(K, b, z):
    """The maximised dual 1^T z - 1/2 z^T H z."""
    H = svm_hessian(K, b)
    return float(np.sum(z) - 0.5 * z @ H @ z)


@dataclasses.dataclass
class SVMResult:
    x: np.ndarray
    z: np.ndarray
    u: np.ndarray
    iters: int
    pcg_iters: list
    r_p: list
    r_d: list
    gaps: list
    converged: bool
    factor: object


def nys_factor_of(H, omega_raw, c=0.0, mantissa_bits=52) -> NysFactor:
    """Algorithm RandNysAppx for an explicit PSD matrix H + c I."""
    Omega = orthonormalize(np.asarray(omega_raw, dtype=np.float64))
    Y = H @ Omega + c * Omega
    U, lam, nu = nystrom_from_sketch(Y, Omega, mantissa_bits)
    return NysFactor(U, lam, nu, Omega, Y)


def admm_svm(K, b, C, rho, omega_raw=None, iters=100, pcg_tol=1e-8, exact=False,
             gap_tol=None, gap_every=10, pcg_max_iter=5000, mantissa_bits=52,
             factor=None) -> SVMResult:
    """Algorithm NysADMM on the kernel SVM dual (eq. 8); `factor` (of H) may
    be given instead of the Gaussian entries."""
    b = np.asarray(b, dtype=np.float64)
    H = svm_hessian(K, b)
    n = H.shape[0]
    x, z, u = np.zeros(n), np.zeros(n), np.zeros(n)
    if exact:
        L = np.linalg.cholesky(H + rho * np.eye(n))
    elif factor is None:
        factor = nys_factor_of(H, omega_raw, 0.0, mantissa_bits)
    matvec = lambda p: H @ p + rho * p
    precond = None if exact else (lambda w: precond_inverse_apply(factor.U, factor.lam, rho, w))
    its, rps, rds, gaps = [], [], [], []
    converged = False
    for k in range(iters):
        rhs = rho * (z - u) + 1.0
        if exact:
            x = np.linalg.solve(L.T, np.linalg.solve(L, rhs))
            its.append(0)
        else:
            res = nys_pcg(matvec, rhs, x, precond, pcg_tol, pcg_max_iter)
            x = res.x
            its.append(res.iters)
        z_old = z
        z, _ = project(x + u, b, C)
        u = u + x - z
        rps.append(float(np.linalg.norm(x - z)))
        rds.append(float(rho * np.linalg.norm(z_old - z)))
        if gap_tol is not None and (k + 1) % gap_every == 0:
            gp = duality_gap(K, b, C, z)
            gaps.append(gp.rel)
            if gp.rel <= gap_tol:
                converged = True
                break
    return SVMResult(x, z, u, len(its), its, rps, rds, gaps, converged, factor)
