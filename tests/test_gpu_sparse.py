"""Sparse A (CSR) through the NysADMM hot path on the GPU against the FP64
oracle run on the same matrix densified, through the C ABI.

Parity contract: the matvec pair A^T (D (A p)) + (c + rho) p at 1e-12
relative (rows of 24..45 entries, empty columns, a column present in every
row); the FP64 sketch's H-hat at 1e-10 with nu equal (the NYS_F32 factor
of a sparse A: the same U, Lambda, nu, and P^-1 w at 1e-13 against the
oracle's with U rounded to FP32); lasso and logistic NysADMM iterates within
1e-8 of the oracle's after the same iterations (lasso also with the FP32 U);
malformed CSR input is rejected with NYS_ERR_INVALID before any slot is
written; two handles of the same matrix give bit-for-bit equal results.
"""
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


def densify(rowptr, col, val, n, d):
    A = np.zeros((n, d))
    rp = rowptr.numpy()
    for i in range(n):
        A[i, col[rp[i]:rp[i + 1]].numpy()] = val[rp[i]:rp[i + 1]].double().numpy()
    return A


def make(N, ctx, n, d, density, seed):
    rp, c, v = synth.sparse_text_like(n, d, density, seed=seed)
    S = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v.to(DEV), (n, d))
    return S, densify(rp, c, v, n, d)


@pytest.mark.parametrize("n,d,dens", [(2000, 5000, 0.01), (333, 7001, 0.004), (4100, 900, 0.05)])
def test_sparse_pair_matches_oracle(N, ctx, n, d, dens):
    S, A = make(N, ctx, n, d, dens, seed=n)
    r = np.random.default_rng(1)
    p = r.standard_normal(d)
    D = r.random(n) + 0.1
    v = N.nys_hessian_apply(ctx, S, torch.tensor(p, device=DEV), rho=0.3,
                            D=torch.tensor(D, device=DEV), c=0.2)
    ref = A.T @ (D * (A @ p)) + 0.5 * p
    e = np.linalg.norm(v.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"[sparse pair] {n}x{d} nnz {S.nnz} rel err {e:.2e}", flush=True)
    assert e < 1e-12
    S.close()


@pytest.mark.parametrize("r", [60, 130, 300])   # 1, 3 and 4 column groups per lane, 2 chunks
def test_sparse_sketch_matches_oracle(N, ctx, r):
    n, d = 1500, 3000
    S, A = make(N, ctx, n, d, 0.01, seed=5)
    om = synth.omega_raw(d, r, seed=6)
    F = N.nys_sketch(ctx, S, om.to(DEV), prec=N.NYS_F64)
    f = ny.rand_nys_appx(A, None, 0.0, om.numpy().T)
    U = F.U(ctx).cpu().numpy().T
    lam = np.array(F.info()["lam"])
    e = np.linalg.norm((U * lam) @ U.T - f.dense()) / np.linalg.norm(f.dense())
    print(f"[sparse sketch] r={r} rel(Hhat) {e:.2e} nu {F.info()['nu']:.3e}/{f.nu:.3e}", flush=True)
    assert e < 1e-10 and F.info()["nu"] == f.nu
    # NYS_F32 on a sparse A: the same FP64 products and core (U, Lambda and nu
    # bit-for-bit those of the FP64 factor), and the preconditioner applies
    # the FP32 copy of U: P^-1 w equals the oracle's P^-1 with U rounded to
    # FP32 (FP64 arithmetic on those values)
    F32 = N.nys_sketch(ctx, S, om.to(DEV), prec=N.NYS_F32)
    assert torch.equal(F32.U(ctx), F.U(ctx))
    assert F32.info()["lam"] == F.info()["lam"] and F32.info()["nu"] == F.info()["nu"]
    w = np.random.default_rng(r).standard_normal(d)
    y = N.nys_precond_apply(ctx, F32, 0.5, torch.tensor(w, device=DEV)).cpu().numpy()
    U32 = U.astype(np.float32).astype(np.float64)
    ref32 = ny.precond_inverse_apply(U32, lam, 0.5, w)
    ref64 = ny.precond_inverse_apply(U, lam, 0.5, w)
    e32 = np.linalg.norm(y - ref32) / np.linalg.norm(ref32)
    e64 = np.linalg.norm(y - ref64) / np.linalg.norm(ref64)
    print(f"[sparse sketch] r={r} FP32-U P^-1 w rel err {e32:.2e} (vs FP64 U {e64:.2e})", flush=True)
    assert e32 < 1e-13 and e64 < 1e-5
    with pytest.raises(N.NysError):      # BF16 rounds A, which a sparse A does not take
        N.nys_sketch(ctx, S, om.to(DEV), prec=N.NYS_BF16)
    F32.close()
    F.close()
    S.close()


def test_sparse_lasso_and_logistic_match_oracle(N, ctx):
    n, d, r, its = 2500, 4000, 50, 40
    rp, c, v, b, gamma, _ = synth.sparse_lasso(n, d, 0.01, seed=7)
    A = densify(rp, c, v, n, d)
    S = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v.to(DEV), (n, d))
    om = synth.omega_raw(d, r, seed=8)
    rho = 0.05
    ora = ad.admm_lasso(A, b.numpy(), gamma, rho, omega_raw=om.numpy().T, iters=its,
                        pcg_tol=1e-10)
    st = N.State(d, DEV)
    o = N.admm_opts(rho, r, om.to(DEV), pcg=N.pcg_opts(tol=1e-10), max_iter=its,
                    sketch_prec=N.NYS_F64)
    info = N.admm_solve(ctx, [N.problem(S, b.to(DEV), gamma)], [o], [st])[0]
    z = st.z.cpu().numpy()
    ez = np.linalg.norm(z - ora.z) / np.linalg.norm(ora.z)
    print(f"[sparse lasso] rel z diff {ez:.2e} nnz(z) {(z != 0).sum()} pcg {info.pcg_iters} vs "
          f"{sum(ora.pcg_iters)} eta {info.eta:.2e}", flush=True)
    assert info.iters == its and ez < 1e-8
    assert abs(info.eta - ad.kkt_eta_lasso(A, b.numpy(), gamma, z)) <= 1e-9 * info.eta
    # logistic on the same rows with labels from the sign of A x* + noise
    bl = (np.sign(b.numpy() - np.median(b.numpy())) + 1) / 2
    gl = 0.02 * np.abs(A.T @ (0.5 - bl)).max()
    oral = ad.admm_logistic(A, bl, gl, 1.0, omega_raw=om.numpy().T, iters=20, pcg_tol=1e-10,
                            resketch_every=10)
    st = N.State(d, DEV)
    o = N.admm_opts(1.0, r, om.to(DEV), pcg=N.pcg_opts(tol=1e-10), max_iter=20,
                    resketch_every=10, sketch_prec=N.NYS_F64)
    N.admm_solve(ctx, [N.problem(S, torch.tensor(bl, device=DEV), gl,
                                 loss=N.NYS_LOSS_LOGISTIC)], [o], [st])
    zl = st.z.cpu().numpy()
    el = np.linalg.norm(zl - oral.z) / np.linalg.norm(oral.z)
    print(f"[sparse logistic] rel z diff {el:.2e} nnz(z) {(zl != 0).sum()}", flush=True)
    assert el < 1e-8
    # lasso again with the FP32 copy of U in the preconditioner: PCG solves to
    # the same tolerance, so the iterates stay within 1e-8 of the oracle's
    st = N.State(d, DEV)
    o = N.admm_opts(rho, r, om.to(DEV), pcg=N.pcg_opts(tol=1e-10), max_iter=its,
                    sketch_prec=N.NYS_F32)
    info = N.admm_solve(ctx, [N.problem(S, b.to(DEV), gamma)], [o], [st])[0]
    e32 = np.linalg.norm(st.z.cpu().numpy() - ora.z) / np.linalg.norm(ora.z)
    print(f"[sparse lasso FP32 U] rel z diff {e32:.2e} pcg {info.pcg_iters}", flush=True)
    assert info.iters == its and e32 < 1e-8
    S.close()


def test_sparse_deterministic_and_invalid(N, ctx):
    n, d = 1200, 2500
    rp, c, v = synth.sparse_text_like(n, d, 0.02, seed=9)
    S1 = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v.to(DEV), (n, d))
    S2 = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v.to(DEV), (n, d))
    p = torch.randn(d, dtype=torch.float64, device=DEV)
    y1 = N.nys_hessian_apply(ctx, S1, p, rho=1.0)
    y2 = N.nys_hessian_apply(ctx, S2, p, rho=1.0)
    assert torch.equal(y1, y2)
    S1.close()
    S2.close()
    bad_col = c.clone()
    bad_col[5] = d                         # column out of range
    with pytest.raises(N.NysError):
        N.SparseMatrix(ctx, rp.to(DEV), bad_col.to(DEV), v.to(DEV), (n, d))
    bad_rp = rp.clone()
    r10, r11 = int(rp[10]), int(rp[11])
    bad_rp[10] = r11 + 1                   # rowptr[10] > rowptr[11]: decreasing
    bad_rp[11] = r10
    with pytest.raises(N.NysError):
        N.SparseMatrix(ctx, bad_rp.to(DEV), c.to(DEV), v.to(DEV), (n, d))
    short = rp.clone()
    short[-1] -= 1                         # does not end at nnz
    with pytest.raises(N.NysError):
        N.SparseMatrix(ctx, short.to(DEV), c.to(DEV), v.to(DEV), (n, d))


def test_sparse_large_d_pcg(N, ctx):
    # d > 32768: the PCG scalars are summed by a one-workgroup kernel and U^T w
    # is split into more slices; iterates against the oracle's PCG
    from oracle import pcg as opcg
    n, d, r, rho = 1000, 40000, 30, 1e-2
    S, A = make(N, ctx, n, d, 0.002, seed=12)
    om = synth.omega_raw(d, r, seed=13)
    F = N.nys_sketch(ctx, S, om.to(DEV), prec=N.NYS_F64)
    f = ny.rand_nys_appx(A, None, 0.0, om.numpy().T)
    rhs_np = np.random.default_rng(14).standard_normal(d)
    x = torch.zeros(d, dtype=torch.float64, device=DEV)
    info = N.pcg_solve(ctx, S, torch.tensor(rhs_np, device=DEV), x, rho, F,
                       opts=N.pcg_opts(tol=1e-10, max_iter=2000))
    ora = opcg.nys_pcg(lambda v: A.T @ (A @ v) + rho * v, rhs_np, np.zeros(d),
                       lambda w: ny.precond_inverse_apply(f.U, f.lam, rho, w), 1e-10, 2000)
    e = np.linalg.norm(x.cpu().numpy() - ora.x) / np.linalg.norm(ora.x)
    print(f"[sparse large d] iters {info.iters} oracle {ora.iters} rel diff {e:.2e} true res "
          f"{info.true_res_norm / info.rhs_norm:.2e}", flush=True)
    assert abs(info.iters - ora.iters) <= max(1, int(np.ceil(0.03 * ora.iters)))
    assert info.true_res_norm <= 1e-10 * info.rhs_norm * (1 + 1e-6)
    assert e < 1e-7
    F.close()
    S.close()


@pytest.mark.parametrize("n,d", [(20000, 30000), (5000, 16384), (777, 16385)])
def test_sparse_pair_persistent_rows_and_head(N, ctx, n, d):
    # the row pass runs persistent workgroups (several rows per wavefront at
    # n = 20000) with p[0, 16384) staged in LDS and the rest gathered from
    # memory; d = 16384 / 16385 put the last column exactly at / past the
    # staged head
    import scipy.sparse as sps
    rp, c, v32 = synth.sparse_text_like(n, d, 0.003, seed=d % 1000)
    S = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v32.to(DEV), (n, d))
    A = sps.csr_matrix((v32.double().numpy(), c.numpy(), rp.numpy()), shape=(n, d))
    r = np.random.default_rng(2)
    p = r.standard_normal(d)
    D = r.random(n) + 0.1
    v = N.nys_hessian_apply(ctx, S, torch.tensor(p, device=DEV), rho=0.7,
                            D=torch.tensor(D, device=DEV))
    ref = A.T @ (D * (A @ p)) + 0.7 * p
    e = np.linalg.norm(v.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"[sparse pair persistent] {n}x{d} nnz {S.nnz} rel err {e:.2e}", flush=True)
    assert e < 1e-12
    S.close()


@pytest.mark.parametrize("n,d,dens,seed", [(1, 9, 0.5, 1), (7, 300, 0.01, 2), (3000, 50, 0.5, 3),
                                           (20000, 40, 0.3, 4), (17000, 2000, 0.02, 5)])
def test_sparse_pair_elementwise_edges(N, ctx, n, d, dens, seed):
    # element by element against the FP64 product: a single row, mostly empty
    # columns (each kept as one zero entry in the CSC copy), columns longer
    # than a wavefront's share of the entries (their partial sums combined
    # across wavefronts), fewer entries than workgroups, and n above the
    # LDS-staged part of s
    import scipy.sparse as sps
    r = np.random.default_rng(seed)
    M = sps.random(n, d, density=dens, format="csr", random_state=seed, dtype=np.float64)
    M.data = (np.abs(r.standard_normal(M.nnz)) + 0.1).astype(np.float32).astype(np.float64)
    M.sort_indices()
    rp = torch.tensor(M.indptr, dtype=torch.int32)
    c = torch.tensor(M.indices, dtype=torch.int32)
    v32 = torch.tensor(M.data, dtype=torch.float32)
    S = N.SparseMatrix(ctx, rp.to(DEV), c.to(DEV), v32.to(DEV), (n, d))
    p = r.standard_normal(d)
    D = r.random(n) + 0.1
    v = N.nys_hessian_apply(ctx, S, torch.tensor(p, device=DEV), rho=0.4,
                            D=torch.tensor(D, device=DEV)).cpu().numpy()
    ref = M.T @ (D * (M @ p)) + 0.4 * p
    scale = abs(M).T @ (D * (abs(M) @ np.abs(p))) + 0.4 * np.abs(p)
    err = np.abs(v - ref)
    print(f"[sparse pair edges] {n}x{d} nnz {M.nnz} max err/scale {np.max(err / scale):.2e}",
          flush=True)
    assert np.all(err <= 1e-13 * scale + 1e-300)
    S.close()


def test_sparse_pair_no_rows_and_one_column(N, ctx):
    # n = 0: every column of the CSC copy is its zero entry and s is empty, so
    # the pair is rho p exactly; d = 1 with every row in the one column: one
    # workgroup owns all entries, split over its sixteen wavefronts
    d = 5
    rp = torch.zeros(1, dtype=torch.int32)
    S = N.SparseMatrix(ctx, rp.to(DEV), torch.zeros(0, dtype=torch.int32, device=DEV),
                       torch.zeros(0, dtype=torch.float32, device=DEV), (0, d))
    p = torch.arange(1, d + 1, dtype=torch.float64, device=DEV)
    v = N.nys_hessian_apply(ctx, S, p, rho=0.5)
    assert torch.equal(v, 0.5 * p)
    S.close()
    n = 5000
    r = np.random.default_rng(3)
    vals = (np.abs(r.standard_normal(n)) + 0.1).astype(np.float32)
    rp = torch.arange(n + 1, dtype=torch.int32)
    S = N.SparseMatrix(ctx, rp.to(DEV), torch.zeros(n, dtype=torch.int32, device=DEV),
                       torch.tensor(vals, device=DEV), (n, 1))
    D = r.random(n) + 0.1
    v = N.nys_hessian_apply(ctx, S, torch.tensor([0.7], dtype=torch.float64, device=DEV), rho=0.0,
                            D=torch.tensor(D, device=DEV)).item()
    a = vals.astype(np.float64)
    ref = float(np.sum(a * D * a) * 0.7)
    assert abs(v - ref) <= 1e-13 * abs(ref)
    S.close()
