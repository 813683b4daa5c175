"""Batched lockstep NysADMM (admm_solve with count > 1) against one-at-a-time
solves and the FP64 oracle, through the C ABI.

Instances have uneven shapes (ragged widths, rows not 16-byte aligned, FP32
and FP64 storage) so that several row-width buckets, both load paths and the
per-instance convergence masks are exercised.
"""
import numpy as np
import pytest
import torch

from oracle import admm as ad
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


SHAPES = [(3000, 120, torch.float64), (9000, 337, torch.float32), (5000, 700, torch.float32),
          (12000, 250, torch.float32), (4100, 513, torch.float32), (7000, 1100, torch.float32)]


def make(shapes, rho=0.05, rank=30):
    probs = []
    for k, (n, d, dt) in enumerate(shapes):
        p = synth.lasso_decay(n, d, 0.7, seed=100 + k, dtype=dt, rho=rho, rank=rank, s_max=rank,
                              pcg_tol=1e-10)
        probs.append(p)
    return probs


def to_dev(N, ctx, probs, prec_for):
    A = [p.A.to(DEV) for p in probs]
    b = [p.b.to(DEV) for p in probs]
    om = [p.omega.to(DEV) for p in probs]
    F = [N.nys_sketch(ctx, A[k], om[k], prec=prec_for(p)) for k, p in enumerate(probs)]
    return A, b, om, F


def prec_for(N):
    return lambda p: N.NYS_F64 if p.A.dtype == torch.float64 else N.NYS_F32


def test_batched_equals_sequential_and_oracle(N, ctx):
    probs = make(SHAPES)
    A, b, om, F = to_dev(N, ctx, probs, prec_for(N))
    its = 25
    mk_opts = lambda k: N.admm_opts(probs[k].rho, 30, om[k], pcg=N.pcg_opts(tol=1e-10),
                                    max_iter=its, factor=F[k],
                                    sketch_prec=prec_for(N)(probs[k]))
    # batched
    st_b = [N.State(p.d, DEV) for p in probs]
    info_b = N.admm_solve(ctx, [N.problem(A[k], b[k], probs[k].gamma) for k in range(len(probs))],
                          [mk_opts(k) for k in range(len(probs))], st_b)
    # one at a time, same factors
    for k, p in enumerate(probs):
        st = N.State(p.d, DEV)
        info = N.admm_solve(ctx, [N.problem(A[k], b[k], p.gamma)], [mk_opts(k)], [st])[0]
        zb, zs = st_b[k].z.cpu().numpy(), st.z.cpu().numpy()
        e = np.linalg.norm(zb - zs) / max(np.linalg.norm(zs), 1e-300)
        print(f"[batched] inst {k} {p.n}x{p.d} {p.A.dtype}: rel z diff {e:.2e}, pcg "
              f"{info_b[k].pcg_iters} vs {info.pcg_iters}", flush=True)
        assert info_b[k].iters == its
        assert e < 1e-9
        assert abs(info_b[k].pcg_iters - info.pcg_iters) <= 2
        assert abs(info_b[k].eta - info.eta) <= 1e-6 * info.eta + 1e-14
    # the oracle on two of them (its own factor from the same Gaussian entries)
    for k in (0, 2):
        p = probs[k]
        ora = ad.admm_lasso(p.A.double().numpy(), p.b.numpy(), p.gamma, p.rho,
                            omega_raw=p.omega.numpy().T, iters=its, pcg_tol=1e-10,
                            mantissa_bits=52 if p.A.dtype == torch.float64 else 23)
        zb = st_b[k].z.cpu().numpy()
        assert np.linalg.norm(zb - ora.z) <= 1e-7 * np.linalg.norm(ora.z)
    for f in F:
        f.close()


def test_regularisation_path_warm_started(N, ctx):
    # gamma on a decreasing grid per instance, states carried from one gamma to
    # the next, the factor of A^T A built once and reused; each point is
    # compared with the oracle's exact-solve optimum.
    shapes = [(4000, 150, torch.float32), (6000, 260, torch.float32), (3000, 90, torch.float64)]
    probs = make(shapes, rho=0.1, rank=20)
    A, b, om, F = to_dev(N, ctx, probs, prec_for(N))
    states = [N.State(p.d, DEV) for p in probs]
    gmax = [float(np.abs(p.A.double().numpy().T @ p.b.numpy()).max()) for p in probs]
    for frac in (0.3, 0.1, 0.03):
        gam = [frac * g for g in gmax]
        opts = [N.admm_opts(p.rho, 20, om[k], pcg=N.pcg_opts(tol=1e-10), max_iter=4000,
                            eps_abs=1e-12, eps_rel=1e-10, factor=F[k],
                            sketch_prec=prec_for(N)(p)) for k, p in enumerate(probs)]
        infos = N.admm_solve(ctx, [N.problem(A[k], b[k], gam[k]) for k in range(len(probs))],
                             opts, states)
        for k, p in enumerate(probs):
            Ad = p.A.double().numpy()
            ex = ad.admm_lasso(Ad, p.b.numpy(), gam[k], p.rho, exact=True, iters=100000,
                               eps_abs=1e-15, eps_rel=1e-14)
            z = states[k].z.cpu().numpy()
            fs = ad.lasso_objective(Ad, p.b.numpy(), gam[k], ex.z)
            f = ad.lasso_objective(Ad, p.b.numpy(), gam[k], z)
            print(f"[path] frac {frac} inst {k}: iters {infos[k].iters} converged "
                  f"{infos[k].converged} rel obj {abs(f - fs) / abs(fs):.2e}", flush=True)
            assert infos[k].converged == 1
            assert abs(f - fs) <= 1e-6 * abs(fs)
            assert np.linalg.norm(z - ex.z) <= 1e-5 * max(np.linalg.norm(ex.z), 1e-12)
    for f in F:
        f.close()


def test_batched_true_residual_cadence(N, ctx):
    # lockstep run with the residual of each solve carried to the next step and
    # the true residual checked every 7th step (and at the last): the same
    # iterates as the run that checks every step
    probs = make(SHAPES[:4])
    A, b, om, F = to_dev(N, ctx, probs, prec_for(N))
    its = 20
    out = {}
    for every in (1, 7):
        opts = [N.admm_opts(p.rho, 30, om[k], pcg=N.pcg_opts(tol=1e-10), max_iter=its,
                            factor=F[k], sketch_prec=prec_for(N)(p), true_res_every=every)
                for k, p in enumerate(probs)]
        st = [N.State(p.d, DEV) for p in probs]
        infos = N.admm_solve(ctx, [N.problem(A[k], b[k], p.gamma) for k, p in enumerate(probs)],
                             opts, st)
        out[every] = ([s.z.cpu().numpy() for s in st], infos)
    for k in range(len(probs)):
        z1, z7 = out[1][0][k], out[7][0][k]
        i1, i7 = out[1][1][k], out[7][1][k]
        e = np.linalg.norm(z1 - z7) / max(np.linalg.norm(z1), 1e-300)
        print(f"[batched cadence] inst {k}: rel z diff {e:.2e} pcg {i1.pcg_iters}/{i7.pcg_iters} "
              f"true res max {i1.true_res_max:.2e}/{i7.true_res_max:.2e}", flush=True)
        assert i1.iters == its and i7.iters == its
        assert i1.status == N.NYS_OK and i7.status == N.NYS_OK
        assert e < 1e-8
        assert abs(i1.pcg_iters - i7.pcg_iters) <= 2
        for i in (i1, i7):
            assert 0.0 < i.true_res_max <= 1e-10 * (1 + 1e-6)
    for f in F:
        f.close()
