"""Argument checks and failure reporting of the C ABI on the GPU.

* D >= 0 (H^l of a convex loss is positive semidefinite, Section 2.1): a
  negative weight gives NYS_ERR_INVALID, a NaN or infinite one
  NYS_ERR_NONFINITE, at every entry point that takes a caller's D.
* logistic labels b in {0, 1} (eq. 9), and no ridge term for the logistic loss.
* NaN in A or b surfaces as NYS_ERR_NONFINITE.
* a subproblem that stops at PCG's max_iter above tolerance is counted in
  maxiter_solves and makes the status sticky NYS_ERR_MAXITER, on the single,
  batched and SVM drivers.
"""
import pytest
import torch

from paper_2202_11599_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def N():
    from paper_2202_11599_amd import nysadmm
    return nysadmm


@pytest.fixture(scope="module")
def ctx(N):
    c = N.Context()
    yield c
    c.close()


def small(seed=21, n=600, d=80):
    return synth.lasso_decay(n, d, 0.5, seed=seed, dtype=torch.float64, frac=0.1, rho=0.5,
                             rank=10, s_max=10, pcg_tol=1e-8)


def status_of(N, fn):
    try:
        fn()
    except N.NysError as e:
        return e.status
    return N.NYS_OK


def test_weights_checked_at_every_entry_point(N, ctx):
    p = small()
    A, om = p.A.to(DEV), p.omega.to(DEV)
    x = torch.zeros(p.d, dtype=torch.float64, device=DEV)
    rhs = torch.ones(p.d, dtype=torch.float64, device=DEV)
    good = torch.rand(p.n, dtype=torch.float64, device=DEV)
    for bad_value, want in ((-1e-3, N.NYS_ERR_INVALID), (float("nan"), N.NYS_ERR_NONFINITE),
                            (float("inf"), N.NYS_ERR_NONFINITE)):
        D = good.clone()
        D[p.n - 7] = bad_value
        print(f"[validation] D entry {bad_value}", flush=True)
        calls = {
            "nys_sketch": lambda: N.nys_sketch(ctx, A, om, D=D, prec=N.NYS_F64),
            "nys_sketch_adaptive": lambda: N.nys_sketch_adaptive(ctx, A, om, 5, 10, 0.5, 2.0, D=D),
            "nys_hessian_apply": lambda: N.nys_hessian_apply(ctx, A, x, rho=1.0, D=D),
            "pcg_solve": lambda: N.pcg_solve(ctx, A, rhs, x.clone(), 1.0, D=D),
        }
        for name, fn in calls.items():
            assert status_of(N, fn) == want, (name, bad_value)
    # zero weights are allowed (a convex loss can have a flat direction)
    D = good.clone()
    D[:10] = 0.0
    N.pcg_solve(ctx, A, rhs, x.clone(), 1.0, D=D)
    N.nys_sketch(ctx, A, om, D=D, prec=N.NYS_F64).close()


def test_logistic_labels_and_ridge_checked(N, ctx):
    p = synth.logistic_decay(800, 40, seed=4, dtype=torch.float64, rank=8, rho=5.0)
    A, om = p.A.to(DEV), p.omega.to(DEV)
    opts = N.admm_opts(p.rho, 8, om, max_iter=3)
    for bad_value, want in ((2.0, N.NYS_ERR_INVALID), (-1.0, N.NYS_ERR_INVALID),
                            (0.5, N.NYS_ERR_INVALID), (float("nan"), N.NYS_ERR_NONFINITE)):
        b = p.b.to(DEV).clone()
        b[13] = bad_value
        prob = N.problem(A, b, p.gamma, loss=N.NYS_LOSS_LOGISTIC)
        st = N.State(p.d, DEV)
        assert status_of(N, lambda: N.admm_solve(ctx, [prob], [opts], [st])) == want
        assert status_of(N, lambda: N.admm_step(ctx, prob, opts, None, st)) == want
    prob = N.problem(A, p.b.to(DEV), p.gamma, loss=N.NYS_LOSS_LOGISTIC, c=0.1)
    assert status_of(N, lambda: N.admm_solve(ctx, [prob], [opts], [N.State(p.d, DEV)])) == \
        N.NYS_ERR_INVALID
    # the valid problem runs
    prob = N.problem(A, p.b.to(DEV), p.gamma, loss=N.NYS_LOSS_LOGISTIC)
    info = N.admm_solve(ctx, [prob], [opts], [N.State(p.d, DEV)])[0]
    assert info.iters == 3 and info.status == N.NYS_OK


def test_nan_in_data_is_nonfinite(N, ctx):
    p = small(seed=22)
    om = p.omega.to(DEV)
    opts = N.admm_opts(p.rho, 10, om, max_iter=5)
    b = p.b.to(DEV).clone()
    b[5] = float("nan")
    st = N.State(p.d, DEV)
    assert status_of(N, lambda: N.admm_solve(ctx, [N.problem(p.A.to(DEV), b, p.gamma)], [opts],
                                             [st])) == N.NYS_ERR_NONFINITE
    A = p.A.to(DEV).clone()
    A[17, 3] = float("nan")
    x = torch.zeros(p.d, dtype=torch.float64, device=DEV)
    rhs = torch.ones(p.d, dtype=torch.float64, device=DEV)
    assert status_of(N, lambda: N.pcg_solve(ctx, A, rhs, x, 1.0)) == N.NYS_ERR_NONFINITE
    assert status_of(N, lambda: N.nys_sketch(ctx, A, om, prec=N.NYS_F64)) == N.NYS_ERR_NONFINITE
    A32 = p.A.to(DEV).float()
    A32[0, 0] = float("inf")
    assert status_of(N, lambda: N.nys_sketch(ctx, A32, om, prec=N.NYS_F32)) == \
        N.NYS_ERR_NONFINITE


def test_maxiter_subproblems_are_counted(N, ctx):
    # PCG capped at 2 iterations at a 1e-13 tolerance cannot converge: every
    # subproblem is counted and the status stays NYS_ERR_MAXITER (the run goes on)
    p = small(seed=23)
    A, b, om = p.A.to(DEV), p.b.to(DEV), p.omega.to(DEV)
    pcg = N.pcg_opts(tol=1e-13, max_iter=2)
    opts = N.admm_opts(p.rho, 10, om, pcg=pcg, max_iter=6)
    info = N.admm_solve(ctx, [N.problem(A, b, p.gamma)], [opts], [N.State(p.d, DEV)])[0]
    assert info.iters == 6 and info.maxiter_solves == 6 and info.status == N.NYS_ERR_MAXITER
    # a loose tolerance: none counted
    opts = N.admm_opts(p.rho, 10, om, pcg=N.pcg_opts(tol=1e-6), max_iter=6)
    info = N.admm_solve(ctx, [N.problem(A, b, p.gamma)], [opts], [N.State(p.d, DEV)])[0]
    assert info.maxiter_solves == 0 and info.status == N.NYS_OK
    # batched path (two instances, lockstep): counted per instance
    q = small(seed=24, n=700, d=90)
    probs = [N.problem(A, b, p.gamma), N.problem(q.A.to(DEV), q.b.to(DEV), q.gamma)]
    opts = [N.admm_opts(p.rho, 10, om, pcg=pcg, max_iter=4),
            N.admm_opts(q.rho, 10, q.omega.to(DEV), pcg=pcg, max_iter=4)]
    infos = N.admm_solve(ctx, probs, opts, [N.State(p.d, DEV), N.State(q.d, DEV)])
    for info in infos:
        assert info.iters == 4 and info.maxiter_solves == 4 and info.status == N.NYS_ERR_MAXITER
    # admm_step: per step
    F, info = N.admm_step(ctx, N.problem(A, b, p.gamma), N.admm_opts(p.rho, 10, om, pcg=pcg),
                          None, N.State(p.d, DEV))
    assert info.maxiter_solves == 1 and info.status == N.NYS_ERR_MAXITER
    F.close()


def test_svm_maxiter_counted(N, ctx):
    X, b = synth.svm_points(300, 6, seed=25)
    Xd = X.to(DEV).float().contiguous()
    bd = b.to(DEV)
    H = N.kernel_rbf(ctx, Xd, 1.0 / 6, b=bd)
    st = N.State(300, DEV)
    o = N.svm_opts(1.0, 0, pcg=N.pcg_opts(tol=1e-14, max_iter=2), max_iter=5)
    info = N.svm_solve(ctx, H, bd, 1.0, o, st)
    assert info.iters == 5 and info.maxiter_solves == 5 and info.status == N.NYS_ERR_MAXITER
