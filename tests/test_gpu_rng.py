"""The device Gaussian stream (nys_gaussian: Philox4x32-10 and Box-Muller)
against the oracle's independent statement of the same stream, through the C
ABI, and a sketch built on a test matrix drawn by the library.

Parity contract: every sample within 1e-13 absolute of the oracle's (the
32-bit words must agree exactly for that: a wrong word moves a sample by
O(1)); offsets, the counter's second word and a key with a nonzero high word
covered; invalid arguments rejected; the FP64 sketch (Algorithm RandNysAppx)
on a device-drawn test matrix equal to the oracle's on the oracle-drawn one
(H-hat within 1e-10).
"""
import numpy as np
import pytest
import torch

from oracle import nystrom as ny
from oracle import rng as orng
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


@pytest.mark.parametrize("seed,offset,count", [(0, 0, 1), (1, 0, 4), (123, 5, 1001),
                                               ((1 << 40) + 7, (1 << 34) - 3, 4099),
                                               (2**64 - 1, 2**40 + 2, 257)])
def test_gaussian_matches_oracle(N, ctx, seed, offset, count):
    z = N.nys_gaussian(ctx, seed, count, offset=offset).cpu().numpy()
    ref = orng.gaussian(seed, offset, count)
    err = np.max(np.abs(z - ref))
    print(f"[gaussian] seed {seed} offset {offset} count {count} max abs err {err:.2e}", flush=True)
    assert err <= 1e-13


def test_gaussian_offsets_and_invalid(N, ctx):
    full = N.nys_gaussian(ctx, 9, 3000)
    part = N.nys_gaussian(ctx, 9, 1234, offset=1000)
    assert torch.equal(full[1000:2234], part)
    assert N.nys_gaussian(ctx, 9, 0).numel() == 0
    with pytest.raises(N.NysError):
        N._check(N.lib().nys_gaussian(ctx.h, 9, 0, -1, None), "nys_gaussian")
    with pytest.raises(N.NysError):
        N._check(N.lib().nys_gaussian(ctx.h, 9, 0, 5, None), "nys_gaussian")
    with pytest.raises(N.NysError):
        N._check(N.lib().nys_gaussian(ctx.h, 9, 2**64 - 2, 5, full.data_ptr()), "nys_gaussian")


def test_sketch_on_device_drawn_test_matrix(N, ctx):
    n, d, r, seed = 1500, 400, 37, 77
    A = synth.column_decay_matrix(n, d, seed=3)
    om = N.gaussian_omega(ctx, d, r, seed)
    F = N.nys_sketch(ctx, A.to(DEV), om, prec=N.NYS_F64)
    om_ref = orng.gaussian(seed, 0, d * r).reshape(r, d)
    f = ny.rand_nys_appx(A.numpy(), None, 0.0, om_ref.T)
    U = F.U(ctx).cpu().numpy().T
    info = F.info()
    nu, lam = info["nu"], np.asarray(info["lam"])
    H = (U * lam) @ U.T
    Hr = (f.U * f.lam) @ f.U.T
    e = np.linalg.norm(H - Hr) / np.linalg.norm(Hr)
    print(f"[gaussian sketch] rel err {e:.2e} nu {nu:.3e} vs {f.nu:.3e}", flush=True)
    assert e < 1e-10
    assert nu == pytest.approx(f.nu, rel=1e-12)
    F.close()
