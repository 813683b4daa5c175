"""Pins of the oracle's ADMM branches that the basic lasso/logistic pins do not
reach: the elastic-net shift (eq. 6), the subproblem tolerance schedule and the
residual stop (Section 2.1 and the experimental setup of Section 5), the
relative-change stop of the logistic experiments (Section 5) and the logistic
KKT residual (our reading of eq. 31 for a non-quadratic loss).

Each pin is a closed form, a brute force, or a trace computed step by step in
the test from the definitions, chosen so that a plausible slip in the branch
(the shift put on the right-hand side, squared norms, a 2-norm in place of the
infinity norm, a dropped term of the denominator) fails it.
"""
import itertools
import math

import numpy as np
import scipy.optimize as sopt

from oracle import admm as ad


def rng(seed):
    return np.random.default_rng(seed)


def soft(a, k):
    # written out again on purpose: the pins must not lean on the oracle's helper
    return np.array([math.copysign(max(abs(v) - k, 0.0), v) for v in a])


# ------------------------------------------------------------ elastic net (eq. 6)

def test_elastic_net_orthonormal_closed_form():
    # A^T A = I: 1/2||Ax-b||^2 + c/2||x||^2 + gamma||x||_1 separates into
    # (1+c)/2 x_j^2 - a_j x_j + gamma|x_j| with a = A^T b, whose minimiser is
    # x_j = S_gamma(a_j) / (1 + c).  Putting c on the right-hand side, or
    # leaving it out of the operator, moves the fixed point off this value.
    r = rng(101)
    Q, _ = np.linalg.qr(r.standard_normal((80, 14)))
    b = r.standard_normal(80) * 2.0
    gamma, c = 1.2, 0.7
    x_star = soft(Q.T @ b, gamma) / (1.0 + c)
    assert np.count_nonzero(x_star) >= 3 and np.count_nonzero(x_star == 0) >= 3
    for exact in (True, False):
        res = ad.admm_lasso(Q, b, gamma, 0.8, omega_raw=r.standard_normal((14, 5)), c=c,
                            iters=3000, pcg_tol=1e-13, exact=exact, eps_abs=1e-14,
                            eps_rel=1e-13)
        assert np.allclose(res.z, x_star, atol=1e-10), exact
        assert ad.lasso_objective(Q, b, gamma, res.z, c=c) <= \
            ad.lasso_objective(Q, b, gamma, x_star, c=c) + 1e-12


def elastic_brute_force(A, b, gamma, c):
    # every sign pattern s: on the support S the optimality condition is
    # (A_S^T A_S + c I) x_S = A_S^T b - gamma s_S; keep sign-consistent
    # candidates and take the smallest objective
    d = A.shape[1]
    best, bx = np.inf, None
    for s in itertools.product((-1, 0, 1), repeat=d):
        s = np.array(s, dtype=float)
        S = s != 0
        x = np.zeros(d)
        if S.any():
            AS = A[:, S]
            xs = np.linalg.solve(AS.T @ AS + c * np.eye(S.sum()), AS.T @ b - gamma * s[S])
            if np.any(np.sign(xs) != s[S]):
                continue
            x[S] = xs
        f = 0.5 * np.sum((A @ x - b) ** 2) + 0.5 * c * (x @ x) + gamma * np.abs(x).sum()
        if f < best:
            best, bx = f, x
    return bx


def test_elastic_net_brute_force_small():
    r = rng(102)
    for trial in range(3):
        A = r.standard_normal((25, 6)) * np.array([3.0, 1.0, 0.5, 2.0, 0.3, 1.5])
        b = r.standard_normal(25)
        gamma = 0.25 * np.abs(A.T @ b).max()
        c = [0.3, 1.0, 2.5][trial]
        xb = elastic_brute_force(A, b, gamma, c)
        res = ad.admm_lasso(A, b, gamma, 1.0, omega_raw=r.standard_normal((6, 3)), c=c,
                            iters=4000, pcg_tol=1e-13, eps_abs=1e-14, eps_rel=1e-13)
        assert np.linalg.norm(res.z - xb) <= 1e-9 * max(1.0, np.linalg.norm(xb)), trial


# ------------------------------------------ tolerance schedule and residual stop

def test_tolerance_schedule_and_residual_stop_trace():
    # Orthonormal columns make the subproblem operator (1 + rho) I, so each PCG
    # solve is exact after one iteration and the whole ADMM trace can be
    # written out by hand: x^{k+1} = rhs^k / (1 + rho), z = S_{gamma/rho}(x + u),
    # u += x - z, r_p = ||x - z||, r_d = rho ||z_old - z||, except that PCG
    # returns the warm start untouched when its residual ||rhs - (1 + rho) x||
    # already meets the tolerance (the test comes before the first iteration).
    # The schedule is eps^0 = 1e-2 ||rhs^0||,
    # eps^{k+1} = max(sqrt(r_p^k r_d^k), tol ||rhs^{k+1}||) (norms, not squares).
    r = rng(103)
    Q, _ = np.linalg.qr(r.standard_normal((50, 10)))
    b = r.standard_normal(50) * 3.0
    gamma, rho, ptol = 0.9, 0.6, 1e-9
    atb = Q.T @ b
    x = np.zeros(10); z = np.zeros(10); u = np.zeros(10)
    want_tol, want_rp, want_rd, eps, kept = [], [], [], None, 0
    for k in range(4):
        rhs = rho * (z - u) + atb
        nr = np.linalg.norm(rhs)
        want_tol.append(1e-2 * nr if eps is None else max(eps, ptol * nr))
        if np.linalg.norm(rhs - (1.0 + rho) * x) > want_tol[-1]:
            x = rhs / (1.0 + rho)
        else:
            kept += 1
        z_old = z
        z = soft(x + u, gamma / rho)
        u = u + x - z
        rp = np.linalg.norm(x - z)
        rd = rho * np.linalg.norm(z_old - z)
        want_rp.append(rp)
        want_rd.append(rd)
        eps = math.sqrt(rp * rd)
    # the trace must exercise the schedule branch, not its floor, and tell
    # sqrt(r_p r_d) from r_p r_d
    assert want_tol[1] > 10 * ptol * np.linalg.norm(atb)
    assert abs(want_rp[0] * want_rd[0] - want_tol[1]) > 0.1 * want_tol[1]
    assert 1 <= kept <= 2   # both branches of the PCG stop test occur
    res = ad.admm_lasso(Q, b, gamma, rho, omega_raw=r.standard_normal((10, 4)), iters=4,
                        pcg_tol=ptol, tol_schedule=True)
    assert np.allclose(res.tols, want_tol, rtol=1e-9)
    assert np.allclose(res.r_p, want_rp, rtol=1e-9)
    assert np.allclose(res.r_d, want_rd, rtol=1e-9)
    assert np.allclose(res.z, z, atol=1e-12)

    # residual stop of Section 2.1: ||r_p|| <= eps_abs + eps_rel max(||x||, ||z||)
    # and ||r_d|| <= eps_abs + eps_rel ||rho u||, checked after every step.
    # Run the hand trace on and report the first step at which both hold.
    eps_abs, eps_rel = 1e-6, 1e-4
    rho = 5.0   # far from 1, so ||rho u|| and ||u|| give different stops
    x = np.zeros(10); z = np.zeros(10); u = np.zeros(10)
    stop_at = None
    for k in range(2000):
        rhs = rho * (z - u) + atb
        x = rhs / (1.0 + rho)
        z_old = z
        z = soft(x + u, gamma / rho)
        u = u + x - z
        rp = np.linalg.norm(x - z)
        rd = rho * np.linalg.norm(z_old - z)
        if rp <= eps_abs + eps_rel * max(np.linalg.norm(x), np.linalg.norm(z)) and \
                rd <= eps_abs + eps_rel * np.linalg.norm(rho * u):
            stop_at = k + 1
            break
    assert stop_at is not None and stop_at > 3
    res = ad.admm_lasso(Q, b, gamma, rho, omega_raw=r.standard_normal((10, 4)), iters=2000,
                        pcg_tol=1e-14, eps_abs=eps_abs, eps_rel=eps_rel)
    assert res.converged and res.iters == stop_at


# ------------------------------------------------- relative-change stop (Section 5)

def test_relative_change_is_infinity_norm_hand_vectors():
    # ||z - z_old||_inf / ||z_old||_inf with hand-built vectors where the
    # 2-norm form decides the other way
    z_old = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
    z = np.array([1.0, 9e-4, 9e-4, 9e-4, 9e-4])
    assert ad.rel_change_inf(z_old, z) == 9e-4           # 2-norm form: 1.8e-3
    z_old = np.array([1.0, -1.0, 1.0, -1.0])
    z = np.array([1.0015, -1.0, 1.0, -1.0])
    assert math.isclose(ad.rel_change_inf(z_old, z), 1.5e-3, rel_tol=1e-12)   # 2-norm: 7.5e-4
    assert ad.rel_change_inf(np.zeros(3), np.ones(3)) is None


def test_logistic_relative_change_stop_index():
    # The run stops at the first step k >= 1 whose z moved by less than tol
    # relative to the previous z in the infinity norm, and not earlier.
    r = rng(104)
    n, d = 300, 12
    A = r.standard_normal((n, d)) * np.arange(1, d + 1) ** -0.5
    xt = r.standard_normal(d) * (r.uniform(size=d) < 0.5)
    b = (A @ xt + r.logistic(size=n) > 0).astype(float)
    gamma = 0.05 * np.abs(A.T @ (0.5 - b)).max()
    om = r.standard_normal((d, 5))
    full = ad.admm_logistic(A, b, gamma, 2.0, omega_raw=om, iters=60, pcg_tol=1e-12,
                            record=True)
    tol = 1e-3
    first = None
    for k in range(1, 60):
        zo, zn = full.z_hist[k - 1], full.z_hist[k]
        den = np.max(np.abs(zo))
        if den > 0 and np.max(np.abs(zn - zo)) / den < tol:
            first = k
            break
    assert first is not None and first >= 3
    res = ad.admm_logistic(A, b, gamma, 2.0, omega_raw=om, iters=60, pcg_tol=1e-12,
                           rel_change_tol=tol)
    assert res.converged and res.iters == first + 1
    assert np.array_equal(res.z, full.z_hist[first])


# ------------------------------------------------------- logistic KKT residual

def test_logistic_eta_hand_value_2x2():
    # eta = ||x - S_gamma(x - g)|| / (1 + ||x|| + ||g||), g = A^T (sigma(Ax) - b),
    # evaluated by hand on A = [[1, 2], [3, 4]], x = (0.5, -0.25), b = (1, 0),
    # gamma = 0.1:  t = (0, 0.5), sigma(t) = (1/2, 1/(1 + e^-0.5)),
    # g = (-1/2 + 3 s, -1 + 4 s) with s = sigma(0.5).
    s = 1.0 / (1.0 + math.exp(-0.5))
    g1, g2 = -0.5 + 3.0 * s, -1.0 + 4.0 * s
    a1, a2 = 0.5 - g1, -0.25 - g2                      # both below -gamma
    p1, p2 = a1 + 0.1, a2 + 0.1                        # S_gamma of negative entries
    num = math.hypot(0.5 - p1, -0.25 - p2)
    den = 1.0 + math.hypot(0.5, 0.25) + math.hypot(g1, g2)
    want = num / den
    assert abs(want - 0.52522) < 1e-4                  # the value worked out on paper
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    eta = ad.kkt_eta_logistic(A, np.array([1.0, 0.0]), 0.1, np.array([0.5, -0.25]))
    assert math.isclose(eta, want, rel_tol=1e-13)


def test_logistic_eta_vanishes_at_independent_optimum():
    # zero (to the solver's accuracy) at the L-BFGS-B optimum of the split
    # smooth form, and clearly positive a small step away from it
    r = rng(105)
    n, d = 200, 8
    A = r.standard_normal((n, d))
    b = (A @ (r.standard_normal(d) * (r.uniform(size=d) < 0.5)) + r.logistic(size=n) > 0)
    b = b.astype(float)
    gamma = 0.2 * np.abs(A.T @ (0.5 - b)).max()

    def fg(v):
        p, q = v[:d], v[d:]
        t = A @ (p - q)
        g = A.T @ (ad.sigmoid(t) - b)
        return ad.logistic_loss(t, b) + gamma * v.sum(), np.concatenate([g + gamma, -g + gamma])

    sol = sopt.minimize(fg, np.zeros(2 * d), jac=True, method="L-BFGS-B",
                        bounds=[(0, None)] * (2 * d),
                        options=dict(maxiter=50000, ftol=1e-16, gtol=1e-13))
    xl = sol.x[:d] - sol.x[d:]
    assert np.count_nonzero(np.abs(xl) > 1e-6) >= 2
    assert ad.kkt_eta_logistic(A, b, gamma, xl) < 1e-6
    assert ad.kkt_eta_logistic(A, b, gamma, xl + 1e-2 * r.standard_normal(d)) > 1e-4
