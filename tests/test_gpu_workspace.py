"""Caller-supplied device memory: nys_workspace_query and nys_ctx_set_workspace.

With a workspace set, every device buffer of a call -- the context's own, the
factor and its sketch state, the batched path's, a sparse handle's CSC copy --
is carved from the caller's tensor.  Checked here:
  * the queried size suffices (peak use <= query) for the lasso workload with
    the adaptive FP32 sketch, the FP32 logistic workload with factor refreshes
    (old and new factor alive together), a batched run of three instances and
    a sparse A;
  * the device's free memory does not change during such a call (the library
    made no hipMalloc of its own);
  * results are bit-for-bit those of a context that allocates for itself (the
    same launch shapes: NYSADMM_TUNE=0 for both);
  * a workspace that is too small gives NYS_ERR_NOMEM, and dropping the
    workspace returns to the library's own allocation.
"""
import numpy as np
import pytest
import torch

from paper_2202_11599_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def N():
    from paper_2202_11599_amd import nysadmm
    return nysadmm


@pytest.fixture(autouse=True)
def fixed_shapes(monkeypatch):
    monkeypatch.setenv("NYSADMM_TUNE", "0")


def solve(N, ctx, A, b, gamma, opts, loss=None):
    st = N.State(A.shape[1], DEV)
    prob = N.problem(A, b, gamma, loss=N.NYS_LOSS_LS if loss is None else loss)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    info = N.admm_solve(ctx, [prob], [opts], [st])[0]
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return st, info, free0 - free1


def with_workspace(N, A, r_max, count=1):
    ctx = N.Context()
    q = ctx.workspace_query(A, r_max, count)
    buf = torch.empty(q, dtype=torch.uint8, device=DEV)
    ctx.set_workspace(buf)
    return ctx, q, buf


def test_lasso_adaptive_fp32_in_workspace(N):
    p = synth.lasso_decay(30000, 1500, 0.8, seed=3, device=DEV, dtype=torch.float32,
                          gamma_frac=0.01, rho=1e-4, rank=50, s_max=400, pcg_tol=1e-6)
    mk = lambda: N.admm_opts(p.rho, 50, p.omega, rank_max=400, ada_tol=2.0,
                             sketch_prec=N.NYS_F32, max_iter=15)
    ref_ctx = N.Context()
    st0, info0, _ = solve(N, ref_ctx, p.A, p.b, p.gamma, mk())
    ctx, q, buf = with_workspace(N, p.A, 400)
    st1, info1, grew = solve(N, ctx, p.A, p.b, p.gamma, mk())
    peak = ctx.workspace_peak()
    print(f"[workspace lasso] query {q / 2**20:.1f} MiB peak {peak / 2**20:.1f} MiB rank "
          f"{info1.rank} device memory change {grew}", flush=True)
    assert info1.status == N.NYS_OK and info1.rank == info0.rank
    assert 0 < peak <= q
    assert grew == 0
    assert torch.equal(st1.z, st0.z) and torch.equal(st1.x, st0.x)
    assert info1.pcg_iters == info0.pcg_iters
    # back to the library's own memory: the same answer again
    ctx.set_workspace(None)
    st2, info2, _ = solve(N, ctx, p.A, p.b, p.gamma, mk())
    assert torch.equal(st2.z, st0.z)
    ctx.close()
    ref_ctx.close()


def test_logistic_refresh_in_workspace(N):
    p = synth.logistic_decay(20000, 400, seed=8, device=DEV, dtype=torch.float32, rho=20.0,
                             rank=40, pcg_tol=1e-8)
    mk = lambda: N.admm_opts(p.rho, 40, p.omega, resketch_every=5, sketch_prec=N.NYS_F32,
                             pcg=N.pcg_opts(tol=1e-8), max_iter=12)
    ref_ctx = N.Context()
    st0, info0, _ = solve(N, ref_ctx, p.A, p.b, p.gamma, mk(), loss=N.NYS_LOSS_LOGISTIC)
    ctx, q, buf = with_workspace(N, p.A, 40)
    st1, info1, grew = solve(N, ctx, p.A, p.b, p.gamma, mk(), loss=N.NYS_LOSS_LOGISTIC)
    peak = ctx.workspace_peak()
    print(f"[workspace logistic] query {q / 2**20:.1f} MiB peak {peak / 2**20:.1f} MiB "
          f"device memory change {grew}", flush=True)
    assert info1.status == N.NYS_OK and 0 < peak <= q and grew == 0
    assert torch.equal(st1.z, st0.z)
    ctx.close()
    ref_ctx.close()


def test_batched_in_workspace(N):
    probs = [synth.lasso_decay(8000 + 1000 * k, 600, 0.7, seed=40 + k, device=DEV,
                               dtype=torch.float32, rho=1e-3, rank=30, s_max=30)
             for k in range(3)]
    # the query is per shape: size it for the largest instance
    big = probs[-1]
    ctx, q, buf = with_workspace(N, big.A, 30, count=3)
    P = [N.problem(p.A, p.b, p.gamma) for p in probs]
    O = [N.admm_opts(p.rho, 30, p.omega, sketch_prec=N.NYS_F32, max_iter=10) for p in probs]
    S = [N.State(p.d, DEV) for p in probs]
    infos = N.admm_solve(ctx, P, O, S)
    peak = ctx.workspace_peak()
    print(f"[workspace batched] query {q / 2**20:.1f} MiB peak {peak / 2**20:.1f} MiB", flush=True)
    assert all(i.status == N.NYS_OK and i.iters == 10 for i in infos)
    assert 0 < peak <= q
    ref_ctx = N.Context()
    S0 = [N.State(p.d, DEV) for p in probs]
    N.admm_solve(ref_ctx, P, O, S0)
    for a, b in zip(S, S0):
        assert torch.equal(a.z, b.z)
    ctx.close()
    ref_ctx.close()


def test_sparse_in_workspace(N):
    n, d, r = 3000, 9000, 20
    rp, c, v, b, gamma, _ = synth.sparse_lasso(n, d, 0.01, seed=5)
    rp, c, v, b = rp.to(DEV), c.to(DEV), v.to(DEV), b.to(DEV)
    om = synth.omega_raw(d, r, seed=5, device=DEV)
    ctx0 = N.Context()
    S0 = N.SparseMatrix(ctx0, rp, c, v, (n, d))
    ctx = N.Context()
    # the handle is created after the workspace is set, so its CSC copy is carved too
    q = ctx.workspace_query(S0, r)
    buf = torch.empty(q, dtype=torch.uint8, device=DEV)
    ctx.set_workspace(buf)
    S1 = N.SparseMatrix(ctx, rp, c, v, (n, d))
    mk = lambda: N.admm_opts(1.0, r, om, max_iter=8)
    st0, info0, _ = solve(N, ctx0, S0, b, gamma, mk())
    st1, info1, grew = solve(N, ctx, S1, b, gamma, mk())
    peak = ctx.workspace_peak()
    print(f"[workspace sparse] query {q / 2**20:.1f} MiB peak {peak / 2**20:.1f} MiB", flush=True)
    assert info1.status == N.NYS_OK and 0 < peak <= q and grew == 0
    assert torch.equal(st1.z, st0.z)
    S1.close()
    S0.close()
    ctx.close()
    ctx0.close()


def test_too_small_workspace_is_nomem(N):
    p = synth.lasso_decay(5000, 300, 0.8, seed=6, device=DEV, dtype=torch.float32, rank=20,
                          s_max=20)
    ctx = N.Context()
    buf = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    ctx.set_workspace(buf)
    st = N.State(p.d, DEV)
    with pytest.raises(N.NysError) as ei:
        N.admm_solve(ctx, [N.problem(p.A, p.b, p.gamma)], [N.admm_opts(p.rho, 20, p.omega)], [st])
    assert ei.value.status == N.NYS_ERR_NOMEM
    # host memory is refused by the library itself
    import ctypes
    host = torch.empty(4096, dtype=torch.uint8)
    assert N.lib().nys_ctx_set_workspace(ctx.h, ctypes.c_void_p(host.data_ptr()), 4096) == \
        N.NYS_ERR_INVALID
    ctx.close()
