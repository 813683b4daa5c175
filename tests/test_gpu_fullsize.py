"""Full-size parity of the 100000 x 4000 FP32 lasso workload the bench times
(A = Q1 diag(j^-0.8) Q2^T stored in FP32, x* 2% sparse, b = A x* + 0.01 noise,
gamma = 0.01 ||A^T b||_inf, rho = 1e-4, adaptive rank 50 -> 800 with Tol = 2).

  * Sketch (Algorithm AdaptiveRandNysAppx): the FP32-MFMA form against the
    oracle's adaptive sketch of the upcast A on the same Gaussian blocks and
    the FP32 shift: the same rank, ||H_hat - H_hat_oracle|| <= 1e-5 ||H_hat_oracle||,
    the top eigenvalues within 1e-5, P^-1 v on probe vectors reported.
  * Optimum (Algorithm NysADMM): the library run to the KKT residual eq. (31)
    eta <= 1e-10 with PCG at 1e-10 against the oracle's exact-solve ADMM (one
    Cholesky of A^T A + rho I in FP64 on the host) run to eta <= 1e-13:
    |f(z) - f*| <= 1e-6 |f*| and ||z - x*|| <= 1e-5 ||x*||, both evaluated in
    FP64 by the oracle.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle import admm as ad
from oracle import nystrom as ny
from paper_2202_11599_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def N():
    from paper_2202_11599_amd import nysadmm
    return nysadmm


@pytest.fixture(scope="module")
def workload():
    print("[fullsize] generating 100000 x 4000", flush=True)
    p = synth.lasso_decay(100000, 4000, 0.8, seed=0, device=DEV, dtype=torch.float32,
                          frac=0.02, noise=0.01, gamma_frac=0.01, rho=1e-4, rank=50, s_max=800,
                          pcg_tol=1e-6)
    A64 = p.A.double().cpu().numpy()
    return p, A64, p.b.cpu().numpy(), p.omega.cpu().numpy().T


@pytest.mark.timeout(900)
def test_fullsize_sketch_and_optimum(N, workload):
    p, A, b, om = workload
    ctx = N.Context()
    F = N.nys_sketch_adaptive(ctx, p.A, p.omega.contiguous(), 50, 800, p.rho, 2.0,
                              prec=N.NYS_F32)
    inf = F.info()
    U = F.U(ctx).cpu().numpy().T
    lam = np.array(inf["lam"])
    print(f"[fullsize] gpu rank {inf['rank']}; oracle sketch", flush=True)
    f, hist = ny.adaptive_rand_nys_appx(A, None, 0.0, om, p.rho, 50, 800, 2.0, mantissa_bits=23)
    print(f"[fullsize] oracle ranks {hist}", flush=True)
    assert inf["rank"] == f.rank
    H = (U * lam) @ U.T
    Ho = (f.U * f.lam) @ f.U.T
    eh = float(np.linalg.norm(H - Ho) / np.linalg.norm(Ho))
    el = float(np.max(np.abs(lam[:20] - f.lam[:20]) / f.lam[:20]))
    g = np.random.default_rng(1)
    ep = 0.0
    for _ in range(4):
        w = g.standard_normal(4000)
        y = N.nys_precond_apply(ctx, F, p.rho, torch.tensor(w, device=DEV)).cpu().numpy()
        yo = ny.precond_inverse_apply(f.U, f.lam, p.rho, w)
        ep = max(ep, float(np.linalg.norm(y - yo) / np.linalg.norm(yo)))
    print(f"[fullsize] sketch: rel(Hhat) {eh:.2e}, top-20 eigenvalues {el:.2e}, P^-1 v {ep:.2e}, "
          f"nu {inf['nu']:.3e}/{f.nu:.3e}", flush=True)
    assert eh <= 1e-5 and el <= 1e-5
    assert ep <= 1e-4

    # library: NysADMM with this factor to eta <= 1e-10
    st = N.State(4000, DEV)
    o = N.admm_opts(p.rho, inf["rank"], p.omega, factor=F, pcg=N.pcg_opts(tol=1e-10),
                    max_iter=3000, kkt_tol=1e-10, kkt_every=10)
    info = N.admm_solve(ctx, [N.problem(p.A, p.b, p.gamma)], [o], [st])[0]
    z = st.z.cpu().numpy()
    print(f"[fullsize] gpu admm: {info.iters} iterations, eta {info.eta:.2e}, "
          f"{info.pcg_iters / max(info.iters, 1):.1f} PCG per solve", flush=True)
    assert info.converged == 1 and info.status == N.NYS_OK and info.eta <= 1e-10

    # oracle: exact-solve ADMM on the upcast A
    G = A.T @ A
    ch = sla.cho_factor(G + p.rho * np.eye(4000))
    atb = A.T @ b
    x = np.zeros(4000)
    zo = np.zeros(4000)
    u = np.zeros(4000)
    eta = 1.0
    for k in range(1, 5001):
        x = sla.cho_solve(ch, p.rho * (zo - u) + atb)
        zo = ad.soft_threshold(x + u, p.gamma / p.rho)
        u = u + x - zo
        if k % 50 == 0:
            eta = ad.kkt_eta_lasso(A, b, p.gamma, zo)
            if eta <= 1e-13:
                break
    print(f"[fullsize] oracle exact ADMM: {k} iterations, eta {eta:.2e}, nnz {(zo != 0).sum()}",
          flush=True)
    assert eta <= 1e-13
    fs = ad.lasso_objective(A, b, p.gamma, zo)
    fz = ad.lasso_objective(A, b, p.gamma, z)
    ex = float(np.linalg.norm(z - zo) / np.linalg.norm(zo))
    print(f"[fullsize] |f - f*|/|f*| {abs(fz - fs) / abs(fs):.2e}, ||z - x*||/||x*|| {ex:.2e}, "
          f"library eta vs oracle eta of z: {info.eta:.3e}/{ad.kkt_eta_lasso(A, b, p.gamma, z):.3e}",
          flush=True)
    assert abs(fz - fs) <= 1e-6 * abs(fs)
    assert ex <= 1e-5
    F.close()
    ctx.close()
