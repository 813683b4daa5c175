"""Randomized Nystrom approximation and preconditioner, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

Follows Algorithm RandNysAppx (appendix "Randomized Nystrom approximation and
Nystrom PCG"), Algorithm AdaptiveRandNysAppx (appendix "AdaNysADMM"), the
Nystrom definition eq. (NysAppx) and the preconditioner eq. (Nyspreconditioner)
of Section 2.2.

Readings where the paper is loose (each one listed in the design notes):
  * shift: nu = sqrt(d) * eps(||Y||_2) in both algorithms (the adaptive
    algorithm prints sqrt(n) with n the dimension of H, the fixed one prints no
    factor); eps(x) = 2^(floor(log2 x) - p) with p = 52 for an FP64 sketch and
    p = 23 when Y was accumulated from FP32/BF16 data.
  * norm(Y, 2) is the spectral norm.
  * chol returns the upper factor C with C^T C = M; B = Y_nu / C is the right
    division B C = Y_nu.  M is symmetrised first.  If the Cholesky fails the
    shift is multiplied by 10 and the step retried, at most 3 times.
  * lambda_s is the smallest retained eigenvalue (entry s of the descending
    list, possibly 0 after the clamp).
  * the adaptive loop tests the tolerance before the s_max branch, and its
    tolerance Tol stands for 1 + epsilon of eq. (empCondNum).

Pins (tests/test_oracle_pins.py): exactness when rank(H) <= s, diagonal H with
coordinate test matrix, agreement with the pseudo-inverse definition, Loewner
order and eigenvalue interlacing (Lemma NysPropLemma), the condition-number
bound of Proposition NysPCGThm, P P^-1 = I and the spectrum of P^-1, and the
incremental sketch equal to the one-shot sketch.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla


class NotSPD(RuntimeError):
    pass


def eps_of(x: float, mantissa_bits: int = 52) -> float:
    """MATLAB-style eps(x): spacing of the floats of the binade holding x."""
    if not np.isfinite(x) or x <= 0:
        raise ValueError("eps_of needs a positive finite number")
    m, e = np.frexp(x)          # x = m 2^e, m in [0.5, 1)
    return float(np.ldexp(1.0, int(e) - 1 - mantissa_bits))


def orthonormalize(omega_raw: np.ndarray) -> np.ndarray:
    """Thin QR of the Gaussian test matrix (first two steps of RandNysAppx)."""
    q, _ = np.linalg.qr(omega_raw, mode="reduced")
    return q


def hessian_apply(A, D, c, X):
    """H X with H = A^T diag(D) A + c I (D None means the identity), the Hessian
    of the subproblem (ADMMSubProb) without the rho shift."""
    T = A @ X
    if D is not None:
        T = D.reshape(-1, *([1] * (T.ndim - 1))) * T
    return A.T @ T + c * X


def hessian_dense(A, D, c):
    d = A.shape[1]
    AD = A if D is None else (D[:, None] * A)
    return A.T @ AD + c * np.eye(d)


@dataclasses.dataclass
class NysFactor:
    U: np.ndarray        # d x s, orthonormal columns
    lam: np.ndarray      # s, descending, >= 0
    nu: float
    Omega: np.ndarray    # d x s test matrix actually used
    Y: np.ndarray        # d x s sketch H Omega

    @property
    def rank(self):
        return self.U.shape[1]

    @property
    def lam_s(self):
        return float(self.lam[-1])

    def dense(self):
        return (self.U * self.lam) @ self.U.T


def nystrom_from_sketch(Y: np.ndarray, Omega: np.ndarray, mantissa_bits: int = 52,
                        retries: int = 3):
    """Shift, Cholesky, right division, thin SVD and shift removal of
    Algorithm RandNysAppx, given the sketch Y = H Omega."""
    d = Y.shape[0]
    nrm = float(np.linalg.norm(Y, 2))
    nu = np.sqrt(d) * eps_of(nrm, mantissa_bits)
    for attempt in range(retries + 1):
        Ynu = Y + nu * Omega
        M = Omega.T @ Ynu
        M = 0.5 * (M + M.T)
        try:
            L = np.linalg.cholesky(M)
        except np.linalg.LinAlgError:
            if attempt == retries:
                raise NotSPD("Cholesky of Omega^T Y_nu failed after shift retries")
            nu *= 10.0
            continue
        C = L.T                                   # upper, C^T C = M
        B = sla.solve_triangular(C, Ynu.T, trans="T", lower=False).T   # B C = Y_nu
        U, S, _ = np.linalg.svd(B, full_matrices=False)
        lam = np.maximum(0.0, S * S - nu)
        return U, lam, nu
    raise AssertionError("unreachable")


def rand_nys_appx(A, D, c, omega_raw, mantissa_bits: int = 52) -> NysFactor:
    """Algorithm RandNysAppx for H = A^T diag(D) A + c I.  `omega_raw` holds
    the Gaussian entries (d x s); the orthonormalisation happens here."""
    Omega = orthonormalize(np.asarray(omega_raw, dtype=np.float64))
    Y = hessian_apply(A, D, c, Omega)
    U, lam, nu = nystrom_from_sketch(Y, Omega, mantissa_bits)
    return NysFactor(U, lam, nu, Omega, Y)


def nystrom_definition(H: np.ndarray, Omega: np.ndarray) -> np.ndarray:
    """eq. (NysAppx): H<Omega> = (H Omega) (Omega^T H Omega)^+ (H Omega)^T."""
    HO = H @ Omega
    return HO @ np.linalg.pinv(Omega.T @ HO) @ HO.T


def precond_inverse_apply(U, lam, rho, w):
    """P^-1 w with P^-1 = (lambda_s + rho) U (Lambda + rho I)^-1 U^T + (I - U U^T),
    eq. (Nyspreconditioner), second line, applied in O(ds)."""
    lam_s = float(lam[-1])
    c = U.T @ w
    return (lam_s + rho) * (U @ (c / (lam + rho))) + w - U @ c


def precond_dense(U, lam, rho):
    """Both printed forms of eq. (Nyspreconditioner) as dense d x d matrices."""
    d = U.shape[0]
    lam_s = float(lam[-1])
    P = (U * (lam + rho)) @ U.T / (lam_s + rho) + (np.eye(d) - U @ U.T)
    Pinv = (lam_s + rho) * (U / (lam + rho)) @ U.T + (np.eye(d) - U @ U.T)
    return P, Pinv


def adaptive_rand_nys_appx(A, D, c, omega_raw, rho, s0, s_max, tol,
                           mantissa_bits: int = 52):
    """Algorithm AdaptiveRandNysAppx.  Gaussian blocks are consecutive columns
    of `omega_raw` (d x s_max); each block is orthonormalised on its own and
    only its columns are sketched, the earlier sketch columns are reused.  The
    rank doubles (s0, 2 s0, 4 s0, ...) until (lambda_s + rho)/rho <= tol, the
    last step being cut to s_max.  Returns (factor, history) with history the
    list of (rank, empirical condition number)."""
    omega_raw = np.asarray(omega_raw, dtype=np.float64)
    Om_blocks, Y_blocks, hist = [], [], []
    s, m = 0, s0
    while True:
        blk = orthonormalize(omega_raw[:, s:s + m])
        Om_blocks.append(blk)
        Y_blocks.append(hessian_apply(A, D, c, blk))
        s += m
        Omega = np.concatenate(Om_blocks, axis=1)
        Y = np.concatenate(Y_blocks, axis=1)
        U, lam, nu = nystrom_from_sketch(Y, Omega, mantissa_bits)
        kappa = (float(lam[-1]) + rho) / rho
        hist.append((s, kappa))
        if kappa <= tol or s >= s_max:
            return NysFactor(U, lam, nu, Omega, Y), hist
        m = min(s, s_max - s)


def effective_dimension(H: np.ndarray, rho: float) -> float:
    """eq. (deff): d_eff(rho) = tr(H (H + rho I)^-1), from the eigenvalues."""
    ev = np.clip(np.linalg.eigvalsh(H), 0.0, None)
    return float(np.sum(ev / (ev + rho)))
