"""Seeded synthetic inputs shaped like the NysADMM workloads.

This module draws problem data only: feature matrices with a prescribed
singular-value decay, sparse ground truths, noise, labels, regularisation
levels and the Gaussian entries of the Nystrom test matrix.  It contains none
of the method's arithmetic (no sketch, no factorisation, no CG, no prox), so
the FP64 CPU oracle and the HIP library can both consume its arrays without
sharing any code path of the method itself.

Layout conventions (they match the C ABI):
  * A is row-major n x d (torch shape (n, d), contiguous).
  * The Gaussian test matrix is column-major d x s, i.e. torch shape (s, d):
    row k of the tensor is column k of Omega.  Blocks used by the adaptive
    sketch are consecutive columns.

Every draw uses its own torch.Generator seeded from (seed, tag), so adding a
draw never changes the others.  Generation runs on the device passed in:
"cpu" for test-sized problems, "cuda" for the full-size workloads (the QR of a
1e5 x 4000 Gaussian factor is too slow on a few host cores).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

_TAGS = {"G": 1, "Q1": 2, "Q2": 3, "support": 4, "xval": 5, "noise": 6,
         "omega": 7, "unif": 8, "shape": 9, "misc": 10}


def _gen(seed: int, tag: str, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1000003 + _TAGS[tag] * 7919) % (2**62))
    return g


def gaussian(shape, seed: int, tag: str = "G", device="cpu") -> torch.Tensor:
    """i.i.d. N(0,1) entries in FP64."""
    return torch.randn(*shape, generator=_gen(seed, tag, device), device=device,
                       dtype=torch.float64)


def haar_orthonormal(rows: int, cols: int, seed: int, tag: str, device="cpu") -> torch.Tensor:
    """rows x cols matrix with orthonormal columns, Haar distributed
    (Q factor of a Gaussian matrix with the signs of diag(R) made positive)."""
    g = gaussian((rows, cols), seed, tag, device)
    q, r = torch.linalg.qr(g, mode="reduced")
    sgn = torch.sign(torch.diagonal(r))
    sgn[sgn == 0] = 1
    return q * sgn


def decay_matrix(n: int, d: int, alpha: float, seed: int, device="cpu") -> torch.Tensor:
    """A = Q1 diag(j^-alpha) Q2^T with Haar factors (FP64, exact singular values
    j^-alpha, j = 1..min(n, d)); Q1 is n x k, Q2 is d x k, k = min(n, d)."""
    k = min(n, d)
    sigma = torch.arange(1, k + 1, device=device, dtype=torch.float64).pow(-alpha)
    q1 = haar_orthonormal(n, k, seed, "Q1", device)
    q2 = haar_orthonormal(d, k, seed, "Q2", device)
    a = (q1 * sigma) @ q2.T
    del q1
    return a


def column_decay_matrix(n: int, d: int, seed: int, device="cpu") -> torch.Tensor:
    """A = G diag(1/j) with G i.i.d. N(0,1): polynomial column decay."""
    g = gaussian((n, d), seed, "G", device)
    return g / torch.arange(1, d + 1, device=device, dtype=torch.float64)


def sparse_truth(d: int, frac: float, seed: int, device="cpu") -> torch.Tensor:
    k = max(1, int(round(frac * d)))
    perm = torch.randperm(d, generator=_gen(seed, "support", "cpu"))[:k]
    vals = torch.randn(k, generator=_gen(seed, "xval", "cpu"), dtype=torch.float64)
    x = torch.zeros(d, dtype=torch.float64)
    x[perm] = vals
    return x.to(device)


def omega_raw(d: int, s: int, seed: int, device="cpu") -> torch.Tensor:
    """Gaussian test-matrix entries, column-major d x s (torch shape (s, d))."""
    return gaussian((s, d), seed + 1, "omega", device)


@dataclasses.dataclass
class Problem:
    """One composite problem min l(Ax; b) + gamma ||x||_1 (+ c/2 ||x||^2)."""
    kind: str                    # "lasso" or "logistic"
    A: torch.Tensor              # (n, d), storage dtype of the workload
    b: torch.Tensor              # (n,) FP64; labels in {0, 1} for logistic
    gamma: float
    rho: float
    rank: int
    omega: torch.Tensor          # (s_max, d) FP64 Gaussian entries
    x_true: torch.Tensor         # (d,) FP64
    c: float = 0.0
    pcg_tol: float = 1e-6
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def d(self):
        return self.A.shape[1]


def _lasso_from_matrix(a64: torch.Tensor, dtype, frac, noise, gamma_frac, rho, rank,
                       s_max, seed, device, name, pcg_tol) -> Problem:
    n, d = a64.shape
    a = a64.to(dtype)
    a_up = a.to(torch.float64)             # b is consistent with the stored A
    x = sparse_truth(d, frac, seed, device)
    e = gaussian((n,), seed, "noise", device)
    b = a_up @ x + noise * e
    gamma = float(gamma_frac * (a_up.T @ b).abs().max())
    return Problem("lasso", a.contiguous(), b, gamma, rho, rank,
                   omega_raw(d, s_max, seed, device), x, 0.0, pcg_tol, name)


def lasso_c1(seed: int = 0, device="cpu", dtype=torch.float64, n=2000, d=500) -> Problem:
    """Lasso, 2000 x 500, A = G diag(1/j), 5% support, noise 0.01,
    gamma = 0.1 ||A^T b||_inf, rho = 1, rank 50, PCG tol 1e-8."""
    a64 = column_decay_matrix(n, d, seed, device)
    p = _lasso_from_matrix(a64, dtype, 0.05, 0.01, 0.1, 1.0, 50, 50, seed, device,
                           "lasso-colDecay-2000x500", 1e-8)
    return p


def lasso_decay(n: int, d: int, alpha: float = 0.8, seed: int = 0, device="cpu",
                dtype=torch.float32, frac=0.02, noise=0.01, gamma_frac=0.1,
                rho=1e-4, rank=50, s_max=800, pcg_tol=1e-6, name=None) -> Problem:
    """Lasso with A = Q1 diag(j^-alpha) Q2^T (the 100000 x 4000 FP32 workload
    uses alpha = 0.8, 2% support, noise 0.01, gamma = 0.1 ||A^T b||_inf,
    rho = 1e-4 and an adaptive rank from 50 up to 800)."""
    a64 = decay_matrix(n, d, alpha, seed, device)
    return _lasso_from_matrix(a64, dtype, frac, noise, gamma_frac, rho, rank, s_max,
                              seed, device, name or f"lasso-decay{alpha}-{n}x{d}", pcg_tol)


def logistic_decay(n: int, d: int, seed: int = 0, device="cpu", dtype=torch.float32,
                   frac=0.05, gamma_per_row=1e-3, rho=200.0, rank=200,
                   pcg_tol=1e-6, name=None) -> Problem:
    """l1 logistic regression: rows ~ N(0, Sigma), Sigma = Q diag(1/j) Q^T
    (A = G diag(j^-1/2) Q^T), y = sign(A x* + logistic noise), b = (1 + y)/2,
    gamma = 1e-3 n."""
    g = gaussian((n, d), seed, "G", device)
    q = haar_orthonormal(d, d, seed, "Q2", device)
    scale = torch.arange(1, d + 1, device=device, dtype=torch.float64).pow(-0.5)
    a64 = (g * scale) @ q.T
    del g
    a = a64.to(dtype).contiguous()
    a_up = a.to(torch.float64)
    x = sparse_truth(d, frac, seed, device)
    u = torch.rand(n, generator=_gen(seed, "unif", device), device=device,
                   dtype=torch.float64).clamp(1e-12, 1 - 1e-12)
    t = a_up @ x + torch.log(u / (1 - u))
    y = torch.where(t >= 0, 1.0, -1.0).to(torch.float64)
    b = (1 + y) / 2
    gamma = gamma_per_row * n
    return Problem("logistic", a, b, gamma, rho, rank, omega_raw(d, rank, seed, device),
                   x, 0.0, pcg_tol, name or f"logistic-{n}x{d}")


def batched_shapes(count: int, n_lo: int, n_hi: int, d_lo: int, d_hi: int, seed: int):
    """Uneven instance shapes, n ~ U{n_lo..n_hi}, d ~ U{d_lo..d_hi}."""
    g = _gen(seed, "shape", "cpu")
    ns = torch.randint(n_lo, n_hi + 1, (count,), generator=g).tolist()
    ds = torch.randint(d_lo, d_hi + 1, (count,), generator=g).tolist()
    return list(zip(ns, ds))


def gamma_grid(gmax: float, points: int = 16, lo: float = 1e-3, hi: float = 1e-1):
    """Log-spaced regularisation path in [lo, hi] * gmax, largest first."""
    if points == 1:
        return [hi * gmax]
    return [gmax * math.exp(math.log(hi) + (math.log(lo) - math.log(hi)) * k / (points - 1))
            for k in range(points)]


def batched_instances(count: int = 64, seed: int = 0, device="cpu", dtype=torch.float32,
                      n_range=(5000, 50000), d_range=(500, 3000), alpha=0.7,
                      rho=1e-3, rank=100, gamma_points=16):
    """Regularisation-path workload: `count` uneven lasso instances, each with
    its own gamma grid (stored in meta['gammas'])."""
    probs = []
    for k, (n, d) in enumerate(batched_shapes(count, *n_range, *d_range, seed)):
        p = lasso_decay(n, d, alpha, seed + k, device, dtype, rho=rho, rank=rank,
                        s_max=rank, name=f"path{k}-{n}x{d}")
        gmax = p.gamma / 0.1
        p.meta["gammas"] = gamma_grid(gmax, gamma_points)
        p.gamma = p.meta["gammas"][0]
        probs.append(p)
    return probs


def warmstart_draws(a: torch.Tensor, draws: int, per_draw: int, seed: int,
                    rho_range=(1e-5, 1e-3), gamma_range=(1e-3, 1e-1), frac=0.02, noise=0.01):
    """Training/test subproblem families for the learned warm start on one fixed
    A: `draws` right-hand sides b = A x + noise e (x sparse, each draw its own
    seed), each paired with `per_draw` (gamma, rho) with gamma log-uniform in
    gamma_range * ||A^T b||_inf and rho log-uniform in rho_range.
    Returns a list of (b, gamma, rho); b is FP64 on a's device."""
    n, d = a.shape
    dev = a.device
    a_up = a.to(torch.float64)
    out = []
    for k in range(draws):
        s = seed * 1009 + k
        x = sparse_truth(d, frac, s, dev)
        b = a_up @ x + noise * gaussian((n,), s, "noise", dev)
        gmax = float((a_up.T @ b).abs().max())
        u = torch.rand(2 * per_draw, generator=_gen(s, "misc", "cpu"), dtype=torch.float64)
        for j in range(per_draw):
            lg = math.log(gamma_range[0]) + float(u[2 * j]) * math.log(gamma_range[1] / gamma_range[0])
            lr = math.log(rho_range[0]) + float(u[2 * j + 1]) * math.log(rho_range[1] / rho_range[0])
            out.append((b, gmax * math.exp(lg), math.exp(lr)))
    return out


def svm_points(n: int, p: int, seed: int = 0, sep: float = 1.0, device="cpu"):
    """Two-class points for the kernel SVM: labels b = +-1 with probability
    1/2 each, features a_i = N(0, I_p) + sep * b_i * 1 / sqrt(p), stored FP32
    (n x p); labels FP64.  The classes overlap (margin violations at every
    C), so the dual has variables at 0, at C and in between."""
    u = torch.rand(n, generator=_gen(seed, "unif", device), device=device, dtype=torch.float64)
    b = torch.where(u < 0.5, -1.0, 1.0).to(torch.float64)
    X = gaussian((n, p), seed, "G", device) + sep * b[:, None] / math.sqrt(p)
    return X.to(torch.float32).contiguous(), b.contiguous()


def sparse_text_like(n: int, d: int, density: float, seed: int = 0, device="cpu",
                     zipf: float = 1.1):
    """A sparse n x d matrix shaped like bag-of-words data (E2006, sector):
    about density * d distinct columns per row, drawn with a Zipf popularity
    (column j with weight (j + 1)^-zipf, so a few columns are dense and most
    are rare), positive values |N(0, 1)| + 0.1, each row scaled to unit norm.
    Returns CSR arrays (rowptr int32 n + 1, colidx int32, val float32, sorted
    columns within each row)."""
    per = max(1, int(round(density * d)))
    g = _gen(seed, "shape", device)
    w = torch.arange(1, d + 1, device=device, dtype=torch.float64) ** (-zipf)
    cdf = torch.cumsum(w, 0)
    cdf = cdf / cdf[-1]
    u = torch.rand(n * per, generator=g, device=device, dtype=torch.float64)
    cols = torch.searchsorted(cdf, u).clamp_(max=d - 1)
    rows = torch.arange(n, device=device, dtype=torch.int64).repeat_interleave(per)
    key = torch.unique(rows * d + cols)            # sorted, distinct (row, col)
    r = key // d
    c = (key % d).to(torch.int32)
    counts = torch.bincount(r, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    v = gaussian((key.numel(),), seed, "misc", device).abs() + 0.1
    nrm = torch.zeros(n, dtype=torch.float64, device=device).index_add_(0, r, v * v).sqrt()
    v = v / nrm[r]
    return rowptr.to(torch.int32), c.contiguous(), v.to(torch.float32).contiguous()


def sparse_lasso(n: int, d: int, density: float, seed: int = 0, device="cpu", frac=0.01,
                 noise=0.01, gamma_frac=0.01):
    """Lasso data on a sparse_text_like matrix: x* with frac * d nonzeros
    N(0, 1) on the most popular columns' range, b = A x* + noise, gamma =
    gamma_frac ||A^T b||_inf.  Returns (rowptr, colidx, val, b, gamma, x*);
    A^T b is formed here from the CSR arrays in FP64 (input preparation, not
    the method)."""
    rowptr, col, val = sparse_text_like(n, d, density, seed, device)
    k = max(1, int(frac * d))
    xs = torch.zeros(d, dtype=torch.float64, device=device)
    idx = torch.randperm(min(d, 10 * k), generator=_gen(seed, "support", device),
                         device=device)[:k]
    xs[idx] = gaussian((k,), seed, "xval", device)
    counts = (rowptr[1:] - rowptr[:-1]).to(torch.int64)
    r = torch.arange(n, device=device).repeat_interleave(counts)
    ax = torch.zeros(n, dtype=torch.float64, device=device).index_add_(
        0, r, val.double() * xs[col.long()])
    b = ax + noise * gaussian((n,), seed, "noise", device)
    atb = torch.zeros(d, dtype=torch.float64, device=device).index_add_(
        0, col.long(), val.double() * b[r])
    gamma = float(gamma_frac * atb.abs().max())
    return rowptr, col, val, b, gamma, xs
