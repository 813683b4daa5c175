"""GPU parity of the wide form of the matvec pair (d above one workgroup's row:
8192 FP32 / 4096 FP64 columns), the shapes of the paper's random-feature data
(Table dataset: 13000 x 27648, 60000 x 60000, ...), against the oracle.

The wide form splits the pair at the row dot (row dots per column block, the
mode's epilogue, then the A^T pass per block) with FP64 products and sums, so
the bar is that of the fused pass: 1e-12 relative to the FP64 oracle.  ADMM
runs on wide matrices (lasso and logistic, whose epilogues differ) are
compared with the oracle's iterates.
"""
import ctypes

import numpy as np
import pytest
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
def ctx(N):
    c = N.Context()
    yield c
    c.close()


@pytest.mark.parametrize("n,d,dt,offset,withD", [
    (3001, 27648, torch.float32, 0, True),      # STL-10 width
    (700, 60000, torch.float32, 0, False),      # 60000-column width, ragged last block
    (1500, 9001, torch.float32, 1, True),       # rows 4 bytes off the 16-byte grid
    (1200, 5000, torch.float64, 0, True),       # FP64 above 4096 columns
    (999, 4099, torch.float64, 1, False),       # FP64, unaligned, one column past a block
])
def test_wide_pair_matches_oracle(N, ctx, n, d, dt, offset, withD):
    print(f"[wide pair] n={n} d={d} {dt} offset={offset} D={withD}", flush=True)
    g = torch.Generator().manual_seed(n + d)
    base = torch.randn(n, d + offset, generator=g, dtype=torch.float64).to(dt)
    Ad = base.to(DEV)[:, offset:]               # a view: same ld, start shifted
    A = base[:, offset:].double().numpy()
    p = torch.randn(d, generator=g, dtype=torch.float64)
    D = torch.rand(n, generator=g, dtype=torch.float64) if withD else None
    c, rho = 0.25, 0.5
    v, pv = N.nys_hessian_apply(ctx, Ad, p.to(DEV), rho=rho, D=None if D is None else D.to(DEV),
                                c=c, want_pv=True)
    ref = ny.hessian_apply(A, None if D is None else D.numpy(), c, p.numpy()) + rho * p.numpy()
    err = float(np.linalg.norm(v.cpu().numpy() - ref) / np.linalg.norm(ref))
    print(f"[wide pair]   rel err {err:.2e}", flush=True)
    assert err <= 1e-12
    assert abs(pv - float(p.numpy() @ ref)) <= 1e-12 * abs(float(p.numpy() @ ref))
    # bit-for-bit repeatable (fixed-order sums)
    v2 = N.nys_hessian_apply(ctx, Ad, p.to(DEV), rho=rho, D=None if D is None else D.to(DEV), c=c)
    assert torch.equal(v, v2)


def test_wide_lasso_admm_matches_oracle(N, ctx):
    n, d, r = 2000, 12000, 40
    a64 = synth.column_decay_matrix(n, d, seed=17)
    p = synth._lasso_from_matrix(a64, torch.float32, 0.01, 0.01, 0.005, 1.0, r, r, 17, "cpu",
                                 "lasso-wide", 1e-10)
    A = p.A.double().numpy()
    b = p.b.numpy()
    its = 20
    ora = ad.admm_lasso(A, b, p.gamma, p.rho, omega_raw=p.omega.numpy().T, iters=its,
                        pcg_tol=1e-10, mantissa_bits=23)
    st = N.State(d, DEV)
    o = N.admm_opts(p.rho, r, p.omega.to(DEV), sketch_prec=N.NYS_F32,
                    pcg=N.pcg_opts(tol=1e-10), max_iter=its)
    info = N.admm_solve(ctx, [N.problem(p.A.to(DEV), p.b.to(DEV), p.gamma)], [o], [st])[0]
    z = st.z.cpu().numpy()
    ez = float(np.linalg.norm(z - ora.z) / np.linalg.norm(ora.z))
    eta_o = ad.kkt_eta_lasso(A, b, p.gamma, z)
    print(f"[wide lasso] rel z diff {ez:.2e} eta {info.eta:.4e}/{eta_o:.4e} nnz "
          f"{(z != 0).sum()} pcg {info.pcg_iters}/{sum(ora.pcg_iters)}", flush=True)
    assert info.status == N.NYS_OK and info.iters == its
    assert (z != 0).sum() > 3
    assert ez <= 1e-7
    assert abs(info.eta - eta_o) <= 1e-8 * eta_o


def test_wide_logistic_admm_matches_oracle(N, ctx):
    n, d, r = 3000, 9500, 30
    g = torch.Generator().manual_seed(23)
    A64 = torch.randn(n, d, generator=g, dtype=torch.float64) / np.sqrt(d) * 4.0
    xt = torch.zeros(d, dtype=torch.float64)
    xt[:40] = torch.randn(40, generator=g, dtype=torch.float64) * 3
    t = A64 @ xt
    u = torch.rand(n, generator=g, dtype=torch.float64).clamp(1e-12, 1 - 1e-12)
    b = ((t + torch.log(u / (1 - u))) > 0).double()
    gamma = float(0.2 * (A64.T @ (0.5 - b)).abs().max())
    om = torch.randn(r, d, generator=g, dtype=torch.float64)
    A = A64.numpy()
    its = 15
    ora = ad.admm_logistic(A, b.numpy(), gamma, 5.0, omega_raw=om.numpy().T, iters=its,
                           pcg_tol=1e-10, resketch_every=5)
    st = N.State(d, DEV)
    o = N.admm_opts(5.0, r, om.to(DEV), resketch_every=5, pcg=N.pcg_opts(tol=1e-10),
                    max_iter=its)
    prob = N.problem(A64.to(DEV), b.to(DEV), gamma, loss=N.NYS_LOSS_LOGISTIC)
    info = N.admm_solve(ctx, [prob], [o], [st])[0]
    z = st.z.cpu().numpy()
    ez = float(np.linalg.norm(z - ora.z) / max(np.linalg.norm(ora.z), 1e-300))
    eta_o = ad.kkt_eta_logistic(A, b.numpy(), gamma, z)
    print(f"[wide logistic] rel z diff {ez:.2e} eta {info.eta:.4e}/{eta_o:.4e} nnz "
          f"{(z != 0).sum()}", flush=True)
    assert info.status == N.NYS_OK
    assert (z != 0).sum() > 3
    assert ez <= 1e-7
    assert abs(info.eta - eta_o) <= 1e-8 * eta_o
    assert abs(info.obj - ad.logistic_objective(A, b.numpy(), gamma, z)) <= 1e-10 * abs(info.obj)
