"""nys_hessian_apply_noalloc against nys_hessian_apply through the C ABI.

Both compute v = (A^T diag(D) A + (c + rho) I) p with FP64 products of the
stored A and FP64 sums; they may use different workgroup counts, so the sums
are added in different orders and the bar is rounding of the sums, not bit
equality: ||v_noalloc - v|| <= 1e-12 ||v||.  Two calls in a row, the second
on a smaller matrix, then the limits.
"""
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def N():
    from paper_2202_11599_amd import nysadmm
    return nysadmm


def rel(a, b):
    return float((a - b).norm() / b.norm())


def test_noalloc_matches_allocating_entry_point(N):
    ctx = N.Context()
    g = torch.Generator(device=DEV).manual_seed(7)
    cases = [  # (n, d, dtype, with D, c, rho)
        (60000, 4000, torch.float32, True, 0.25, 1e-3),
        (5003, 701, torch.float64, False, 0.0, 0.5),
    ]
    for n, d, dt, withD, c, rho in cases:
        print(f"[noalloc] n={n} d={d} {dt} D={withD}", flush=True)
        A = torch.randn(n, d, generator=g, device=DEV, dtype=torch.float64).to(dt)
        p = torch.randn(d, generator=g, device=DEV, dtype=torch.float64)
        D = torch.rand(n, generator=g, device=DEV, dtype=torch.float64) if withD else None
        v0, pv0 = N.nys_hessian_apply(ctx, A, p, rho=rho, D=D, c=c, want_pv=True)
        out = torch.full((d,), float("nan"), dtype=torch.float64, device=DEV)
        v1, pv1 = N.nys_hessian_apply_noalloc(ctx, A, p, out, rho=rho, D=D, c=c, want_pv=True)
        torch.cuda.synchronize()
        assert v1 is out
        e = rel(v1, v0)
        print(f"[noalloc]   rel diff {e:.2e}  pv {pv1:.6e} vs {pv0:.6e}", flush=True)
        assert e <= 1e-12
        assert abs(pv1 - pv0) <= 1e-12 * abs(pv0)
        # an FP64 reference on the device as a third opinion
        Ad = A.double()
        t = Ad @ p
        if D is not None:
            t = D * t
        ref = Ad.T @ t + (rho + c) * p
        assert rel(v1, ref) <= 1e-12
    ctx.close()


def test_noalloc_limits_and_empty(N):
    ctx = N.Context()
    p = torch.ones(8193, dtype=torch.float64, device=DEV)
    out = torch.empty_like(p)
    A = torch.ones(4, 8193, dtype=torch.float32, device=DEV)
    with pytest.raises(N.NysError) as ei:
        N.nys_hessian_apply_noalloc(ctx, A, p, out)
    assert ei.value.status == N.NYS_ERR_INVALID
    A = torch.ones(4, 4097, dtype=torch.float64, device=DEV)
    with pytest.raises(N.NysError):
        N.nys_hessian_apply_noalloc(ctx, A, p[:4097], out[:4097])
    D = torch.ones(4, dtype=torch.float64, device=DEV)
    D[1] = -1.0
    A = torch.ones(4, 16, dtype=torch.float32, device=DEV)
    with pytest.raises(N.NysError) as ei:
        N.nys_hessian_apply_noalloc(ctx, A, p[:16], out[:16], D=D)
    assert ei.value.status == N.NYS_ERR_INVALID
    # no rows: v = (rho + c) p.  torch gives a zero-row tensor a null data
    # pointer, so the descriptor is built by hand on a live buffer.
    import ctypes
    buf = torch.ones(1, 16, dtype=torch.float32, device=DEV)
    dA = N.Dense(0, 16, 16, N.NYS_F32, buf.data_ptr())
    v = out[:16]
    st = N.lib().nys_hessian_apply_noalloc(ctx.h, ctypes.byref(dA), None, 0.5, 2.0,
                                           ctypes.c_void_p(p.data_ptr()),
                                           ctypes.c_void_p(v.data_ptr()), None)
    torch.cuda.synchronize()
    assert st == N.NYS_OK
    assert torch.equal(v, torch.full((16,), 2.5, dtype=torch.float64, device=DEV))
    ctx.close()
