"""Pins of the kernel SVM oracle (oracle/svm.py) against things other than
itself: scipy's pairwise distances, a general QP solver, and LIBSVM's SMO
solver (scikit-learn's SVC on the precomputed kernel)."""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.distance import cdist

from oracle import svm

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def two_blobs(n, p, seed, sep=1.0):
    r = np.random.default_rng(seed)
    b = np.where(r.random(n) < 0.5, -1.0, 1.0)
    X = r.standard_normal((n, p)) + sep * b[:, None] * np.ones(p) / np.sqrt(p)
    return X, b


def test_rbf_kernel_matches_pairwise_distances():
    X, _ = two_blobs(40, 7, 1)
    K = svm.rbf_kernel(X, 0.3)
    assert np.allclose(K, np.exp(-0.3 * cdist(X, X, "sqeuclidean")), rtol=1e-13, atol=0)
    assert np.allclose(np.diag(K), 1.0) and np.allclose(K, K.T)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_projection_matches_qp_solver(seed):
    r = np.random.default_rng(10 + seed)
    n, C = 12, 0.7
    b = np.where(r.random(n) < 0.5, -1.0, 1.0)
    b[0], b[1] = 1.0, -1.0
    v = r.standard_normal(n) * 1.5
    z, mu = svm.project(v, b, C)
    assert abs(b @ z) <= 1e-12 and z.min() >= 0.0 and z.max() <= C
    qp = minimize(lambda t: 0.5 * np.sum((t - v) ** 2), np.full(n, C / 2), jac=lambda t: t - v,
                  method="SLSQP", bounds=[(0.0, C)] * n,
                  constraints=[{"type": "eq", "fun": lambda t: b @ t, "jac": lambda t: b}],
                  options={"ftol": 1e-15, "maxiter": 500})
    assert np.linalg.norm(z - qp.x) <= 1e-6
    # the projection is no worse than the QP solver's point
    assert np.sum((z - v) ** 2) <= np.sum((qp.x - v) ** 2) + 1e-12


def test_gap_weak_duality_and_zero_at_libsvm_optimum():
    sk = pytest.importorskip("sklearn.svm")
    X, b = two_blobs(120, 5, 4, sep=1.5)
    K = svm.rbf_kernel(X, 0.4)
    C = 1.0
    r = np.random.default_rng(5)
    for _ in range(5):
        z, _ = svm.project(r.random(120) * 2 * C - 0.5 * C, b, C)
        assert svm.duality_gap(K, b, C, z).gap >= -1e-12
    m = sk.SVC(kernel="precomputed", C=C, tol=1e-12, shrinking=False).fit(K, b)
    a = np.zeros(120)
    a[m.support_] = np.abs(m.dual_coef_[0])
    g = svm.duality_gap(K, b, C, a)
    assert g.rel <= 1e-6
    # decision values agree with LIBSVM's up to its bias choice
    dec = K @ (b * a) + g.beta
    assert np.max(np.abs(dec - m.decision_function(K))) <= 1e-4 * max(1.0, np.abs(dec).max())


def test_admm_reaches_libsvm_dual_objective():
    sk = pytest.importorskip("sklearn.svm")
    X, b = two_blobs(150, 6, 7, sep=1.2)
    K = svm.rbf_kernel(X, 0.25)
    C = 2.0
    m = sk.SVC(kernel="precomputed", C=C, tol=1e-12, shrinking=False).fit(K, b)
    a = np.zeros(150)
    a[m.support_] = np.abs(m.dual_coef_[0])
    d_sk = svm.dual_objective(K, b, a)
    ex = svm.admm_svm(K, b, C, 1.0, iters=20000, exact=True, gap_tol=1e-10, gap_every=50)
    assert ex.converged
    d_ex = svm.dual_objective(K, b, ex.z)
    assert abs(d_ex - d_sk) <= 1e-7 * abs(d_sk)
    assert abs(b @ ex.z) <= 1e-10 and ex.z.min() >= 0 and ex.z.max() <= C
    # Nystrom-PCG ADMM tracks the exact-solve run
    om = np.random.default_rng(8).standard_normal((150, 30))
    ny = svm.admm_svm(K, b, C, 1.0, omega_raw=om, iters=200, pcg_tol=1e-12)
    ex2 = svm.admm_svm(K, b, C, 1.0, iters=200, exact=True)
    assert np.linalg.norm(ny.z - ex2.z) <= 1e-8 * np.linalg.norm(ex2.z)
