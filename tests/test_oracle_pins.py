"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
formula: they use closed forms, special cases that reduce to a library routine
(scipy CG, LU solve, L-BFGS-B), brute force on tiny inputs, and the
deterministic results of the analysis (Lemma NysPropLemma, Proposition
NysPCGThm, Lemma KeyLemma, the CG energy-norm bound used by Corollary
ADMMSubProb).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as sopt
import scipy.sparse.linalg as spla

from oracle import nystrom as ny
from oracle import pcg as pc
from oracle import admm as ad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


def decay_A(n, d, alpha, seed=0):
    r = rng(seed)
    q1, _ = np.linalg.qr(r.standard_normal((n, d)))
    q2, _ = np.linalg.qr(r.standard_normal((d, d)))
    return (q1 * np.arange(1, d + 1) ** -alpha) @ q2.T


# ---------------------------------------------------------------- eps / shift

def test_eps_matches_ieee_spacing():
    # MATLAB eps(x) is the IEEE spacing of the binade of x: numpy.spacing.
    for x in [1.0, 0.75, 3.0, 1e-7, 12345.678, 2.0 ** 40]:
        assert ny.eps_of(x, 52) == np.spacing(np.float64(x))
        assert ny.eps_of(x, 23) == float(np.spacing(np.float32(x)))


# ---------------------------------------------------------------- Nystrom

def test_nystrom_exact_when_rank_le_s():
    # Lemma NysPropLemma: H<Omega> depends on range(Omega); if range(H) lies in
    # range(H Omega) (rank(H) = k <= s, Gaussian Omega) then H<Omega> = H.
    r = rng(1)
    n, d, k, s = 80, 40, 7, 12
    A = r.standard_normal((n, k)) @ r.standard_normal((k, d))
    H = A.T @ A
    f = ny.rand_nys_appx(A, None, 0.0, r.standard_normal((d, s)))
    err = np.linalg.norm(f.dense() - H) / np.linalg.norm(H)
    assert err < 1e-10
    ev = np.sort(np.linalg.eigvalsh(H))[::-1][:k]
    assert np.allclose(f.lam[:k], ev, rtol=1e-9, atol=1e-12 * ev[0])
    assert np.all(f.lam[k:] <= 1e-10 * ev[0])


def test_nystrom_diagonal_coordinate_test_matrix():
    # H = diag(lambda), Omega = [e_1..e_s]: H Omega = Omega diag(lambda_1..s),
    # so U = [+-e_i] and Lambda = lambda_1..s exactly (Sigma^2 = lambda + nu).
    d, s = 30, 6
    lam = np.linspace(9.0, 0.5, d)
    A = np.diag(np.sqrt(lam))
    f = ny.rand_nys_appx(A, None, 0.0, np.eye(d)[:, :s])
    assert np.allclose(f.lam, lam[:s], rtol=1e-13)
    assert np.allclose(np.abs(f.U), np.eye(d)[:, :s], atol=1e-13)


def test_nystrom_stable_equals_pinv_definition():
    # Algorithm RandNysAppx is a stable evaluation of eq. (NysAppx).
    A = decay_A(300, 60, 0.8, seed=2)
    H = A.T @ A
    r = rng(3)
    f = ny.rand_nys_appx(A, None, 0.0, r.standard_normal((60, 15)))
    ref = ny.nystrom_definition(H, f.Omega)
    assert np.linalg.norm(f.dense() - ref) / np.linalg.norm(H) < 1e-10


def test_nystrom_loewner_and_interlacing():
    # Lemma NysPropLemma: H<Omega> is psd, rank <= s, H<Omega> <= H (Loewner),
    # lambda_j(H<Omega>) <= lambda_j(H).
    A = decay_A(400, 60, 0.5, seed=4)
    H = A.T @ A
    f = ny.rand_nys_appx(A, None, 0.0, rng(5).standard_normal((60, 20)))
    Hn = f.dense()
    scale = np.linalg.norm(H, 2)
    assert np.linalg.eigvalsh(H - Hn).min() > -1e-12 * scale
    assert np.linalg.eigvalsh(Hn).min() > -1e-12 * scale
    assert np.linalg.matrix_rank(Hn, tol=1e-9 * scale) <= 20
    eh = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert np.all(f.lam <= eh[:20] * (1 + 1e-12) + 1e-14 * scale)


def test_condition_number_bound():
    # Proposition NysPCGThm: kappa(P^-1/2 H_rho P^-1/2) <= (lam_s + rho + ||E||)/rho.
    A = decay_A(300, 50, 0.8, seed=6)
    H = A.T @ A
    rho = 1e-3
    f = ny.rand_nys_appx(A, None, 0.0, rng(7).standard_normal((50, 10)))
    E = H - f.dense()
    P, Pinv = ny.precond_dense(f.U, f.lam, rho)
    Pih = sla.sqrtm(Pinv).real
    M = Pih @ (H + rho * np.eye(50)) @ Pih
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    kappa = ev.max() / ev.min()
    bound = (f.lam_s + rho + np.linalg.norm(E, 2)) / rho
    assert kappa <= bound * (1 + 1e-8)


def test_preconditioner_forms_and_spectrum():
    # eq. (Nyspreconditioner): the two printed forms are inverses, the O(ds)
    # apply equals the dense inverse, and the spectrum of P^-1 is
    # {(lam_s + rho)/(lam_i + rho)} together with 1 (d - s times).
    A = decay_A(200, 40, 0.8, seed=8)
    rho = 1e-2
    f = ny.rand_nys_appx(A, None, 0.0, rng(9).standard_normal((40, 8)))
    P, Pinv = ny.precond_dense(f.U, f.lam, rho)
    assert np.allclose(P @ Pinv, np.eye(40), atol=1e-11)
    w = rng(10).standard_normal(40)
    assert np.allclose(ny.precond_inverse_apply(f.U, f.lam, rho, w), Pinv @ w, atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(Pinv))
    expect = np.sort(np.concatenate([(f.lam_s + rho) / (f.lam + rho), np.ones(32)]))
    assert np.allclose(ev, expect, atol=1e-11)
    assert ev.min() > 0


def test_adaptive_sketch_equals_definition_on_union_and_stops_early():
    # Algorithm AdaptiveRandNysAppx: reusing earlier sketch columns gives the
    # Nystrom approximation of range([Omega_1 .. Omega_k]) (eq. NysAppx), and
    # because lam_s(Hhat) <= lam_s(H) (Lemma NysPropLemma) the loop stops no
    # later than the first doubled rank s with lam_s(H) <= (Tol - 1) rho.
    d = 120
    A = decay_A(500, d, 1.0, seed=11)
    H = A.T @ A
    rho, tol = 1e-3, 2.0
    om = rng(12).standard_normal((d, 80))
    f, hist = ny.adaptive_rand_nys_appx(A, None, 0.0, om, rho, 5, 80, tol)
    ref = ny.nystrom_definition(H, f.Omega)
    assert np.linalg.norm(f.dense() - ref) / np.linalg.norm(H) < 1e-9
    ranks = [h[0] for h in hist]
    assert ranks[0] == 5 and all(b == min(2 * a, 80) for a, b in zip(ranks, ranks[1:]))
    eh = np.sort(np.linalg.eigvalsh(H))[::-1]
    first_ok = next(s for s in [5, 10, 20, 40, 80] if eh[s - 1] <= (tol - 1) * rho or s == 80)
    assert ranks[-1] <= first_ok
    # the blocks are consecutive columns, each orthonormal on its own
    for a, b in zip([0] + ranks[:-1], ranks):
        blk = f.Omega[:, a:b]
        assert np.allclose(blk.T @ blk, np.eye(b - a), atol=1e-12)


def test_effective_dimension_and_key_lemma():
    # eq. (deff) on a diagonal matrix, and Lemma KeyLemma:
    # j >= (1 + 1/g) d_eff(rho)  =>  lambda_j <= g rho.
    lam = np.arange(1, 301) ** -1.6
    rho = 1e-3
    de = ny.effective_dimension(np.diag(lam), rho)
    assert abs(de - np.sum(lam / (lam + rho))) < 1e-9
    for g in [0.1, 1 / 7, 1.0, 4.0]:
        j = int(math.ceil((1 + 1 / g) * de))
        if j <= 300:
            assert lam[j - 1] <= g * rho


# ---------------------------------------------------------------- PCG

def test_dense_solve_matches_lu():
    r = rng(13)
    A = r.standard_normal((60, 25))
    D = r.uniform(0.1, 2.0, 60)
    rhs = r.standard_normal(25)
    x = pc.dense_solve(A, D, 0.3, 0.7, rhs)
    K = A.T @ (D[:, None] * A) + 1.0 * np.eye(25)
    assert np.allclose(x, sla.lu_solve(sla.lu_factor(K), rhs), rtol=1e-12, atol=1e-12)


def test_pcg_identity_preconditioner_is_textbook_cg():
    # Algorithm Nystrom PCG with P = I is plain CG: iterates equal scipy's.
    A = decay_A(200, 40, 0.5, seed=14)
    rho = 1e-2
    mv = pc.subproblem_matvec(A, None, 0.0, rho)
    rhs = rng(15).standard_normal(40)
    ours = []
    pc.nys_pcg(mv, rhs, np.zeros(40), None, 1e-12, max_iter=12, track=lambda x: ours.append(x.copy()))
    theirs = []
    K = A.T @ A + rho * np.eye(40)
    spla.cg(K, rhs, x0=np.zeros(40), rtol=1e-14, atol=0.0, maxiter=12,
            callback=lambda x: theirs.append(np.array(x)))
    for a, b in zip(ours[:12], theirs[:12]):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


def test_pcg_reaches_dense_solution():
    # PCG reaches the (ADMMSubProb) solution: error <= kappa(H_rho) * tol.
    A = decay_A(300, 80, 0.8, seed=16)
    rho = 1e-4
    f = ny.rand_nys_appx(A, None, 0.0, rng(17).standard_normal((80, 20)))
    rhs = rng(18).standard_normal(80)
    res = pc.nys_pcg(pc.subproblem_matvec(A, None, 0.0, rho), rhs, np.zeros(80),
                     pc.nystrom_precond(f, rho), 1e-10)
    xs = pc.dense_solve(A, None, 0.0, rho, rhs)
    kap = np.linalg.cond(A.T @ A + rho * np.eye(80))
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= kap * 1e-10
    assert res.iters < 60


def test_pcg_low_rank_one_or_two_steps():
    # rank(H) < s: H_hat = H, P^-1 H_rho = (lam_s + rho) I on range(U) and rho
    # on the complement... with lam_s = 0 both equal rho: one CG step in exact
    # arithmetic (allow 2 in FP64).
    r = rng(19)
    A = r.standard_normal((90, 6)) @ r.standard_normal((6, 50))
    f = ny.rand_nys_appx(A, None, 0.0, r.standard_normal((50, 10)))
    rhs = r.standard_normal(50)
    res = pc.nys_pcg(pc.subproblem_matvec(A, None, 0.0, 0.1), rhs, np.zeros(50),
                     pc.nystrom_precond(f, 0.1), 1e-10)
    assert res.iters <= 2


def test_pcg_energy_norm_rate_when_kappa_small():
    # Corollary ADMMSubProb's proof: with kappa = kappa(P^-1/2 H_rho P^-1/2),
    # ||x_t - x*||_{H_rho} <= 2 ((sqrt k - 1)/(sqrt k + 1))^t ||x*||_{H_rho},
    # which is <= (1/2)^(t-1) once kappa <= 8.
    A = decay_A(400, 100, 1.0, seed=20)
    rho = 1e-3
    f = ny.rand_nys_appx(A, None, 0.0, rng(21).standard_normal((100, 40)))
    K = A.T @ A + rho * np.eye(100)
    _, Pinv = ny.precond_dense(f.U, f.lam, rho)
    Pih = sla.sqrtm(Pinv).real
    ev = np.linalg.eigvalsh(Pih @ K @ Pih)
    kap = ev.max() / ev.min()
    assert kap <= 8.0
    rhs = rng(22).standard_normal(100)
    xs = np.linalg.solve(K, rhs)
    en = lambda v: math.sqrt(v @ K @ v)
    its = []
    pc.nys_pcg(pc.subproblem_matvec(A, None, 0.0, rho), rhs, np.zeros(100),
               pc.nystrom_precond(f, rho), 1e-13, track=lambda x: its.append(x.copy()))
    q = (math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)
    for t, x in enumerate(its, start=1):
        if en(x - xs) < 1e-12 * en(xs):
            break
        assert en(x - xs) <= 2 * q ** t * en(xs) * (1 + 1e-6)
        assert en(x - xs) <= 0.5 ** (t - 1) * en(xs) * (1 + 1e-6)


def test_pcg_zero_rhs_and_warm_start_zero_iterations():
    A = decay_A(50, 10, 0.5, seed=23)
    mv = pc.subproblem_matvec(A, None, 0.0, 1.0)
    res = pc.nys_pcg(mv, np.zeros(10), np.ones(10), None, 1e-8)
    assert res.iters == 0 and np.all(res.x == 0)
    rhs = rng(24).standard_normal(10)
    xs = pc.dense_solve(A, None, 0.0, 1.0, rhs)
    res = pc.nys_pcg(mv, rhs, xs, None, 1e-8)
    assert res.iters == 0


# ---------------------------------------------------------------- lasso

def lasso_brute_force(A, b, gamma):
    """Enumerate sign patterns: on support S with signs s the stationarity
    A_S^T (A_S x - b) + gamma s = 0 fixes x_S; keep sign-consistent points and
    return the one with the smallest objective."""
    d = A.shape[1]
    best, bx = np.inf, None
    for pat in itertools.product((-1, 0, 1), repeat=d):
        S = [j for j in range(d) if pat[j] != 0]
        x = np.zeros(d)
        if S:
            AS = A[:, S]
            sg = np.array([pat[j] for j in S], dtype=float)
            xs = np.linalg.solve(AS.T @ AS, AS.T @ b - gamma * sg)
            if np.any(np.sign(xs) != sg):
                continue
            x[S] = xs
        f = 0.5 * np.sum((A @ x - b) ** 2) + gamma * np.abs(x).sum()
        if f < best:
            best, bx = f, x
    return bx


def test_lasso_orthonormal_design_closed_form():
    r = rng(25)
    Q, _ = np.linalg.qr(r.standard_normal((60, 12)))
    b = r.standard_normal(60)
    gamma = 0.3
    res = ad.admm_lasso(Q, b, gamma, 1.0, exact=True, iters=400, eps_abs=1e-13, eps_rel=1e-13)
    assert np.allclose(res.z, ad.soft_threshold(Q.T @ b, gamma), atol=1e-10)
    assert ad.kkt_eta_lasso(Q, b, gamma, res.z) < 1e-10


def test_lasso_large_gamma_gives_zero():
    r = rng(26)
    A = r.standard_normal((40, 10))
    b = r.standard_normal(40)
    gamma = 1.0001 * np.abs(A.T @ b).max()
    res = ad.admm_lasso(A, b, gamma, 1.0, omega_raw=r.standard_normal((10, 4)), iters=50)
    assert np.all(res.z == 0)


def test_lasso_brute_force_small():
    r = rng(27)
    for trial in range(3):
        A = r.standard_normal((30, 6))
        b = r.standard_normal(30)
        gamma = 0.3 * np.abs(A.T @ b).max()
        xb = lasso_brute_force(A, b, gamma)
        res = ad.admm_lasso(A, b, gamma, 1.0, omega_raw=r.standard_normal((6, 3)),
                            iters=3000, pcg_tol=1e-12, eps_abs=1e-13, eps_rel=1e-12)
        assert np.linalg.norm(res.z - xb) <= 1e-8 * max(1.0, np.linalg.norm(xb))


def test_lasso_kkt_and_dual_certificate():
    # At the ADMM fixed point rho u = -A^T (A z - b): the dual certificate, and
    # |(A^T(Az - b))_j| <= gamma with equality and opposite sign on the support.
    A = decay_A(200, 30, 0.5, seed=28)
    r = rng(29)
    b = A @ (r.standard_normal(30) * (r.uniform(size=30) < 0.3)) + 0.01 * r.standard_normal(200)
    gamma = 0.05 * np.abs(A.T @ b).max()
    rho = 0.5
    res = ad.admm_lasso(A, b, gamma, rho, omega_raw=r.standard_normal((30, 10)), iters=5000,
                        pcg_tol=1e-12, eps_abs=1e-12, eps_rel=1e-12)
    g = A.T @ (A @ res.z - b)
    assert np.allclose(rho * res.u, -g, atol=1e-8)
    on = res.z != 0
    assert np.all(np.abs(g) <= gamma * (1 + 1e-7))
    assert np.allclose(g[on], -gamma * np.sign(res.z[on]), atol=1e-7 * gamma)
    assert ad.kkt_eta_lasso(A, b, gamma, res.z) < 1e-9


def test_lasso_matches_lbfgsb_split_form():
    # Independent solver: x = p - q, p, q >= 0, smooth objective, L-BFGS-B.
    A = decay_A(300, 40, 0.8, seed=30)
    r = rng(31)
    b = A @ (r.standard_normal(40) * (r.uniform(size=40) < 0.2)) + 0.01 * r.standard_normal(300)
    gamma = 0.02 * np.abs(A.T @ b).max()

    def fg(v):
        p, q = v[:40], v[40:]
        res = A @ (p - q) - b
        g = A.T @ res
        return 0.5 * res @ res + gamma * v.sum(), np.concatenate([g + gamma, -g + gamma])

    sol = sopt.minimize(fg, np.zeros(80), jac=True, method="L-BFGS-B",
                        bounds=[(0, None)] * 80, options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    xl = sol.x[:40] - sol.x[40:]
    res = ad.admm_lasso(A, b, gamma, 0.05, omega_raw=r.standard_normal((40, 10)), iters=4000,
                        pcg_tol=1e-12, eps_abs=1e-12, eps_rel=1e-12)
    fo = ad.lasso_objective(A, b, gamma, res.z)
    fl = ad.lasso_objective(A, b, gamma, xl)
    assert fo <= fl + 1e-9 * abs(fl)
    assert np.linalg.norm(res.z - xl) <= 1e-4 * np.linalg.norm(xl)


def test_inexact_and_exact_admm_agree_on_small_c1_shape():
    # Inexact ADMM with PCG at tight tolerance tracks exact-solve ADMM
    # (Algorithm Inexact ADMM with eps^k -> 0).
    r = rng(32)
    G = r.standard_normal((400, 100))
    A = G / np.arange(1, 101)
    x = np.zeros(100)
    x[r.choice(100, 5, replace=False)] = r.standard_normal(5)
    b = A @ x + 0.01 * r.standard_normal(400)
    gamma = 0.1 * np.abs(A.T @ b).max()
    ex = ad.admm_lasso(A, b, gamma, 1.0, exact=True, iters=100)
    nx = ad.admm_lasso(A, b, gamma, 1.0, omega_raw=r.standard_normal((100, 10)), iters=100,
                       pcg_tol=1e-12)
    assert np.linalg.norm(ex.z - nx.z) <= 1e-8 * np.linalg.norm(ex.z)


def test_cg_admm_tracks_exact_admm():
    # Inexact ADMM with plain CG (Table t-ComplexityComparison, first row) at a
    # tight tolerance tracks exact-solve ADMM and builds no factor.
    r = rng(34)
    A = r.standard_normal((300, 80)) / np.sqrt(np.arange(1, 81))
    x = np.zeros(80)
    x[r.choice(80, 5, replace=False)] = r.standard_normal(5)
    b = A @ x + 0.01 * r.standard_normal(300)
    gamma = 0.1 * np.abs(A.T @ b).max()
    ex = ad.admm_lasso(A, b, gamma, 0.5, exact=True, iters=80)
    cg = ad.admm_lasso(A, b, gamma, 0.5, iters=80, pcg_tol=1e-13, cg=True)
    assert cg.factor is None
    assert np.linalg.norm(ex.z - cg.z) <= 1e-8 * np.linalg.norm(ex.z)
    assert min(cg.pcg_iters[1:]) > 0
    bl = (np.sign(A @ x + 0.3 * r.standard_normal(300)) + 1) / 2
    exl = ad.admm_logistic(A, bl, 0.5, 1.0, iters=40, exact=True)
    cgl = ad.admm_logistic(A, bl, 0.5, 1.0, iters=40, pcg_tol=1e-13, cg=True)
    assert cgl.factor is None
    assert np.linalg.norm(exl.z - cgl.z) <= 1e-8 * max(np.linalg.norm(exl.z), 1e-300)


# ---------------------------------------------------------------- logistic

def test_logistic_weight_identity_and_rhs():
    # Section 3.2: w = 1/(2 + e^-t + e^t) = sigma(t)(1 - sigma(t)), and
    # w q = w t + b - sigma(t) with q = t + (b - sigma(t))/w.
    t = np.linspace(-12, 12, 97)
    b = (np.arange(97) % 2).astype(float)
    w, s = ad.logistic_weights(t, b)
    assert np.allclose(w, 1.0 / (2.0 + np.exp(-t) + np.exp(t)), rtol=1e-13)
    sig = 1.0 / (1.0 + np.exp(-t))
    q = t + (b - sig) / w
    assert np.allclose(s, w * q, rtol=1e-9, atol=1e-12)


def test_logistic_gradient_finite_difference():
    r = rng(33)
    A = r.standard_normal((50, 8))
    b = (r.uniform(size=50) < 0.5).astype(float)
    x = r.standard_normal(8) * 0.3
    g = A.T @ (ad.sigmoid(A @ x) - b)
    h = 1e-6
    fd = np.array([(ad.logistic_loss(A @ (x + h * e), b) - ad.logistic_loss(A @ (x - h * e), b)) / (2 * h)
                   for e in np.eye(8)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_logistic_zero_solution_above_threshold():
    r = rng(34)
    A = r.standard_normal((80, 12))
    b = (r.uniform(size=80) < 0.4).astype(float)
    gamma = 1.0001 * np.abs(A.T @ (0.5 - b)).max()
    res = ad.admm_logistic(A, b, gamma, 1.0, omega_raw=r.standard_normal((12, 4)), iters=30)
    assert np.all(res.z == 0)


def test_logistic_matches_lbfgsb_and_kkt():
    r = rng(35)
    n, d = 400, 20
    A = r.standard_normal((n, d)) * np.arange(1, d + 1) ** -0.5
    xt = r.standard_normal(d) * (r.uniform(size=d) < 0.3)
    b = (A @ xt + r.logistic(size=n) > 0).astype(float)
    gamma = 0.1 * np.abs(A.T @ (0.5 - b)).max()

    def fg(v):
        p, q = v[:d], v[d:]
        t = A @ (p - q)
        g = A.T @ (ad.sigmoid(t) - b)
        return ad.logistic_loss(t, b) + gamma * v.sum(), np.concatenate([g + gamma, -g + gamma])

    sol = sopt.minimize(fg, np.zeros(2 * d), jac=True, method="L-BFGS-B",
                        bounds=[(0, None)] * (2 * d), options=dict(maxiter=50000, ftol=1e-16, gtol=1e-12))
    xl = sol.x[:d] - sol.x[d:]
    res = ad.admm_logistic(A, b, gamma, 5.0, omega_raw=r.standard_normal((d, 8)), iters=3000,
                           pcg_tol=1e-12, resketch_every=10)
    assert ad.kkt_eta_logistic(A, b, gamma, res.z) < 1e-8
    assert np.linalg.norm(res.z - xl) <= 1e-4 * np.linalg.norm(xl)
    assert ad.logistic_objective(A, b, gamma, res.z) <= ad.logistic_objective(A, b, gamma, xl) + 1e-9


# ---------------------------------------------------------------- golden fixtures

def test_golden_closed_form_fixtures():
    # Hand-derived values (see each fixture's "source"): a 2x2 lasso with
    # orthonormal design and a diagonal Nystrom case.
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        fx = json.load(fh)
    for case in fx["lasso_orthonormal"]:
        A = np.array(case["A"], dtype=float)
        b = np.array(case["b"], dtype=float)
        res = ad.admm_lasso(A, b, case["gamma"], 1.0, exact=True, iters=500,
                            eps_abs=1e-14, eps_rel=1e-14)
        assert np.allclose(res.z, case["x_star"], atol=1e-10)
    for case in fx["nystrom_diagonal"]:
        lam = np.array(case["lambda"], dtype=float)
        A = np.diag(np.sqrt(lam))
        f = ny.rand_nys_appx(A, None, 0.0, np.eye(len(lam))[:, :case["s"]])
        assert np.allclose(f.lam, case["lambda_hat"], rtol=1e-12)
        _, Pinv = ny.precond_dense(f.U, f.lam, case["rho"])
        assert np.allclose(np.sort(np.linalg.eigvalsh(Pinv)), np.sort(case["pinv_eigs"]), atol=1e-12)
