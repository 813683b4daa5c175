"""ctypes binding of libnysadmm (C ABI in include/nysadmm.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.  The
library is loaded on first use and a missing build raises ImportError (there is
no fallback path).

Entry points keep the C names: nys_sketch, nys_sketch_adaptive,
nys_precond_apply, nys_hessian_apply, pcg_solve, admm_step, admm_solve, plus
the context/factor helpers.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnysadmm.so")
_lib = None

NYS_OK, NYS_ERR_INVALID, NYS_ERR_HIP, NYS_ERR_NOT_SPD, NYS_ERR_BREAKDOWN, NYS_ERR_MAXITER, \
    NYS_ERR_NONFINITE, NYS_ERR_NOMEM, NYS_ERR_NOT_CONVERGED = range(9)
NYS_F32, NYS_F64, NYS_BF16, NYS_CSR = 0, 1, 2, 3
NYS_LOSS_LS, NYS_LOSS_LOGISTIC = 0, 1

EXPORTS = [
    "nys_status_string", "nys_ctx_create", "nys_ctx_destroy", "nys_ctx_set_stream",
    "nys_ctx_workspace_bytes", "nys_ctx_profile_start", "nys_ctx_profile_stop", "nys_ctx_profile_pcg", "nys_ctx_profile_pcg_enable", "nys_sketch", "nys_sketch_adaptive", "nys_factor_import",
    "nys_factor_info", "nys_factor_get_U", "nys_factor_destroy", "nys_hessian_apply",
    "nys_precond_apply", "pcg_solve", "admm_step", "admm_solve", "nys_ws_param_count",
    "nys_ws_create", "nys_ws_get_params", "nys_ws_forward", "nys_ws_loss_grad",
    "nys_ws_train_step", "nys_ws_destroy", "nys_kernel_rbf", "nys_sketch_sym", "pcg_solve_sym",
    "svm_solve", "nys_sparse_create", "nys_sparse_destroy", "nys_hessian_apply_noalloc",
    "nys_workspace_query", "nys_ctx_set_workspace", "nys_ctx_workspace_peak",
    "nys_ws_set_precision", "nys_gaussian",
]


class NysError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)})")


class Dense(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int), ("data", C.c_void_p)]


class PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_abs", C.c_int), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("true_residual", C.c_int), ("max_restarts", C.c_int)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("rhs_norm", C.c_double),
                ("res_norm", C.c_double), ("true_res_norm", C.c_double), ("status", C.c_int)]


class Problem(C.Structure):
    _fields_ = [("loss", C.c_int), ("A", Dense), ("b", C.c_void_p), ("gamma", C.c_double),
                ("c", C.c_double)]


class AdmmOpts(C.Structure):
    _fields_ = [("rho", C.c_double), ("rank", C.c_int), ("rank_max", C.c_int),
                ("ada_tol", C.c_double), ("resketch_every", C.c_int), ("sketch_prec", C.c_int),
                ("omega", C.c_void_p), ("pcg", PcgOpts), ("tol_schedule", C.c_int),
                ("max_iter", C.c_int), ("eps_abs", C.c_double), ("eps_rel", C.c_double),
                ("rel_change_tol", C.c_double), ("kkt_tol", C.c_double), ("kkt_every", C.c_int),
                ("factor", C.c_void_p), ("warm_start", C.c_void_p), ("ws_analytic", C.c_int),
                ("ws_every_step", C.c_int), ("ws_features", C.c_void_p),
                ("ws_target", C.c_void_p), ("true_res_every", C.c_int)]


class SvmProblem(C.Structure):
    _fields_ = [("H", Dense), ("b", C.c_void_p), ("C", C.c_double)]


class SvmOpts(C.Structure):
    _fields_ = [("rho", C.c_double), ("rank", C.c_int), ("omega", C.c_void_p), ("pcg", PcgOpts),
                ("max_iter", C.c_int), ("gap_tol", C.c_double), ("gap_every", C.c_int),
                ("true_res_every", C.c_int), ("factor", C.c_void_p)]


class SvmInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("pcg_iters", C.c_long), ("pcg_max", C.c_int),
                ("r_p", C.c_double), ("r_d", C.c_double), ("primal", C.c_double),
                ("dual", C.c_double), ("gap", C.c_double), ("gap_rel", C.c_double),
                ("bias", C.c_double), ("rank", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("true_res_max", C.c_double), ("maxiter_solves", C.c_int)]


class AdmmState(C.Structure):
    _fields_ = [("x", C.c_void_p), ("z", C.c_void_p), ("u", C.c_void_p), ("k", C.c_int)]


class AdmmInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("pcg_iters", C.c_long), ("pcg_max", C.c_int),
                ("r_p", C.c_double), ("r_d", C.c_double), ("eta", C.c_double),
                ("obj", C.c_double), ("rank", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("ws_used", C.c_int), ("true_res_max", C.c_double),
                ("maxiter_solves", C.c_int)]


def lib():
    """Load libnysadmm.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run python -m paper_2202_11599_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "nys_status_string": (C.c_char_p, [i32]),
        "nys_ctx_create": (i32, [i32, vp, P(vp)]),
        "nys_ctx_destroy": (i32, [vp]),
        "nys_ctx_set_stream": (i32, [vp, vp]),
        "nys_ctx_workspace_bytes": (C.c_size_t, [vp]),
        "nys_workspace_query": (i32, [vp, P(Dense), i32, i32, P(C.c_size_t)]),
        "nys_ctx_set_workspace": (i32, [vp, vp, C.c_size_t]),
        "nys_ctx_workspace_peak": (C.c_size_t, [vp]),
        "nys_ctx_profile_start": (i32, [vp]),
        "nys_ctx_profile_stop": (i32, [vp, P(C.c_long), P(dbl)]),
        "nys_ctx_profile_pcg": (i32, [vp, P(C.c_long), P(dbl)]),
        "nys_ctx_profile_pcg_enable": (i32, [vp, i32]),
        "nys_sketch": (i32, [vp, P(Dense), vp, dbl, vp, i32, i32, P(vp)]),
        "nys_sketch_adaptive": (i32, [vp, P(Dense), vp, dbl, vp, i32, i32, dbl, dbl, i32, P(vp)]),
        "nys_factor_import": (i32, [vp, i64, i32, vp, P(dbl), dbl, P(vp)]),
        "nys_factor_info": (i32, [vp, P(i32), P(dbl), P(dbl), P(dbl)]),
        "nys_factor_get_U": (i32, [vp, vp, vp]),
        "nys_factor_destroy": (i32, [vp]),
        "nys_hessian_apply": (i32, [vp, P(Dense), vp, dbl, dbl, vp, vp, P(dbl)]),
        "nys_hessian_apply_noalloc": (i32, [vp, P(Dense), vp, dbl, dbl, vp, vp, P(dbl)]),
        "nys_precond_apply": (i32, [vp, vp, dbl, vp, vp]),
        "pcg_solve": (i32, [vp, P(Dense), vp, dbl, dbl, vp, vp, vp, P(PcgOpts), P(PcgInfo)]),
        "admm_step": (i32, [vp, P(Problem), P(AdmmOpts), P(vp), P(AdmmState), P(AdmmInfo)]),
        "admm_solve": (i32, [vp, i32, P(Problem), P(AdmmOpts), P(AdmmState), P(AdmmInfo)]),
        "nys_ws_param_count": (C.c_size_t, [i32, i32, i32]),
        "nys_ws_create": (i32, [vp, i32, i32, i32, P(dbl), P(dbl), P(dbl), P(dbl), i32, P(vp)]),
        "nys_ws_get_params": (i32, [vp, vp, P(dbl)]),
        "nys_ws_set_precision": (i32, [vp, vp, i32]),
        "nys_ws_forward": (i32, [vp, vp, vp, i32, vp]),
        "nys_ws_loss_grad": (i32, [vp, vp, vp, vp, vp, i32, P(dbl), vp]),
        "nys_ws_train_step": (i32, [vp, vp, vp, vp, vp, i32, dbl, P(dbl)]),
        "nys_ws_destroy": (i32, [vp]),
        "nys_kernel_rbf": (i32, [vp, vp, i64, i64, i64, vp, dbl, vp, i64]),
        "nys_sketch_sym": (i32, [vp, P(Dense), dbl, vp, i32, i32, P(vp)]),
        "pcg_solve_sym": (i32, [vp, P(Dense), dbl, dbl, vp, vp, vp, P(PcgOpts), P(PcgInfo)]),
        "svm_solve": (i32, [vp, P(SvmProblem), P(SvmOpts), P(AdmmState), P(SvmInfo)]),
        "nys_sparse_create": (i32, [vp, i64, i64, i64, vp, vp, vp, P(vp)]),
        "nys_sparse_destroy": (i32, [vp]),
        "nys_gaussian": (i32, [vp, C.c_uint64, C.c_uint64, i64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().nys_status_string(int(s)).decode()


def _check(status, where, ok=(NYS_OK,)):
    if status not in ok:
        raise NysError(status, where)
    return status


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _vec(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of {n} elements")
    return t


def dense(A) -> Dense:
    """Describe a row-major (n, d) tensor (contiguous rows, any row stride), or
    a SparseMatrix."""
    if isinstance(A, SparseMatrix):
        return A.descriptor()
    if A.dim() != 2 or not A.is_cuda or A.stride(1) != 1:
        raise ValueError("A must be a 2-D CUDA tensor with unit column stride")
    dt = {torch.float32: NYS_F32, torch.float64: NYS_F64}.get(A.dtype)
    if dt is None:
        raise ValueError("A must be float32 or float64")
    ld = A.stride(0) if A.shape[0] > 1 else A.shape[1]
    return Dense(A.shape[0], A.shape[1], max(ld, A.shape[1]), dt, A.data_ptr())


class Context:
    """nys_ctx bound to the current torch device and stream."""

    def __init__(self, device: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None):
        L = lib()
        self.device = torch.cuda.current_device() if device is None else device
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        h = C.c_void_p()
        _check(L.nys_ctx_create(self.device, C.c_void_p(s.cuda_stream), C.byref(h)),
               "nys_ctx_create")
        self.h = h

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        _check(lib().nys_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)), "nys_ctx_set_stream")

    def profile_start(self):
        """Time every matvec-pair launch with HIP events from now on."""
        _check(lib().nys_ctx_profile_start(self.h), "nys_ctx_profile_start")

    def profile_stop(self):
        """(launches, total_ms) of the matvec-pair kernel since profile_start."""
        n, ms = C.c_long(), C.c_double()
        _check(lib().nys_ctx_profile_stop(self.h, C.byref(n), C.byref(ms)), "nys_ctx_profile_stop")
        return n.value, ms.value

    def profile_pcg_enable(self, on: bool = True):
        """Time each ADMM subproblem's PCG solve with HIP events (clears the record)."""
        _check(lib().nys_ctx_profile_pcg_enable(self.h, int(bool(on))), "nys_ctx_profile_pcg_enable")

    def profile_pcg(self):
        """(solves, total_ms) of the PCG solves timed since profile_pcg_enable."""
        n, ms = C.c_long(), C.c_double()
        _check(lib().nys_ctx_profile_pcg(self.h, C.byref(n), C.byref(ms)), "nys_ctx_profile_pcg")
        return n.value, ms.value

    def workspace_bytes(self) -> int:
        return int(lib().nys_ctx_workspace_bytes(self.h))

    def workspace_query(self, A, r_max: int, count: int = 1) -> int:
        """Device bytes admm_solve needs for `count` problems shaped like A at
        rank <= r_max when the memory comes from set_workspace."""
        dA = dense(A)
        out = C.c_size_t()
        _check(lib().nys_workspace_query(self.h, C.byref(dA), int(r_max), int(count),
                                         C.byref(out)), "nys_workspace_query")
        return int(out.value)

    def set_workspace(self, buf: Optional[torch.Tensor]):
        """Carve every device buffer of this context from `buf` (a CUDA tensor
        the caller keeps alive; its bytes are used); None returns to the
        library's own allocation."""
        if buf is None:
            _check(lib().nys_ctx_set_workspace(self.h, None, 0), "nys_ctx_set_workspace")
            self._workspace = None
            return
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("workspace must be a contiguous CUDA tensor")
        _check(lib().nys_ctx_set_workspace(self.h, C.c_void_p(buf.data_ptr()),
                                           buf.numel() * buf.element_size()),
               "nys_ctx_set_workspace")
        self._workspace = buf

    def workspace_peak(self) -> int:
        return int(lib().nys_ctx_workspace_peak(self.h))

    def synchronize(self):
        self._stream.synchronize()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().nys_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SparseMatrix:
    """A CSR matrix on the device (int32 rowptr and column indices, float32
    values, CUDA tensors kept alive here) with the library's column-major copy
    for the A^T pass.  Accepted wherever an A is."""

    def __init__(self, ctx: "Context", rowptr: torch.Tensor, colidx: torch.Tensor, val: torch.Tensor,
                 shape):
        n, d = int(shape[0]), int(shape[1])
        for t, dt, name in ((rowptr, torch.int32, "rowptr"), (colidx, torch.int32, "colidx"),
                            (val, torch.float32, "val")):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous CUDA {dt} tensor")
        if rowptr.numel() != n + 1 or colidx.numel() != val.numel():
            raise ValueError("rowptr needs n + 1 entries and colidx/val one per nonzero")
        self._keep = (rowptr, colidx, val)
        self.shape = (n, d)
        self.nnz = int(val.numel())
        h = C.c_void_p()
        _check(lib().nys_sparse_create(ctx.h, n, d, self.nnz, _ptr(rowptr), _ptr(colidx), _ptr(val),
                                       C.byref(h)), "nys_sparse_create")
        self.h = h

    @staticmethod
    def from_torch(ctx: "Context", M: torch.Tensor) -> "SparseMatrix":
        """From a torch sparse CSR tensor (any device/dtype; moved to CUDA FP32)."""
        M = M.to_sparse_csr()
        return SparseMatrix(ctx, M.crow_indices().to(torch.int32).cuda().contiguous(),
                            M.col_indices().to(torch.int32).cuda().contiguous(),
                            M.values().to(torch.float32).cuda().contiguous(), M.shape)

    def descriptor(self) -> Dense:
        return Dense(self.shape[0], self.shape[1], self.shape[1], NYS_CSR, self.h.value)

    def close(self):
        if self.h:
            lib().nys_sparse_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """Owning wrapper of a nys_factor handle."""

    def __init__(self, h: C.c_void_p, d: int):
        self.h = h
        self.d = d

    def info(self):
        r, nu, ls = C.c_int(), C.c_double(), C.c_double()
        _check(lib().nys_factor_info(self.h, C.byref(r), C.byref(nu), C.byref(ls), None),
               "nys_factor_info")
        lam = (C.c_double * r.value)()
        lib().nys_factor_info(self.h, None, None, None, lam)
        return {"rank": r.value, "nu": nu.value, "lambda_s": ls.value, "lam": list(lam)}

    def U(self, ctx: Context) -> torch.Tensor:
        """U as a (rank, d) FP64 tensor: row k is column k of U."""
        r = self.info()["rank"]
        out = torch.empty(r, self.d, dtype=torch.float64, device=f"cuda:{ctx.device}")
        _check(lib().nys_factor_get_U(ctx.h, self.h, _ptr(out)), "nys_factor_get_U")
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().nys_factor_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nys_gaussian(ctx: Context, seed: int, count: int, offset: int = 0,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Samples offset .. offset + count - 1 of the device Gaussian stream of
    `seed` (FP64, on the context's device, ordered on its stream)."""
    if out is None:
        out = torch.empty(count, dtype=torch.float64, device=f"cuda:{ctx.device}")
    elif out.dtype != torch.float64 or not out.is_contiguous() or out.numel() < count:
        raise ValueError("out: contiguous FP64 tensor with at least count entries")
    _check(lib().nys_gaussian(ctx.h, int(seed) & (2**64 - 1), int(offset), int(count),
                              _ptr(out) if count > 0 else None), "nys_gaussian")
    return out


def gaussian_omega(ctx: Context, d: int, s: int, seed: int) -> torch.Tensor:
    """A d x s Gaussian test matrix drawn on the device, column-major (torch
    shape (s, d): row k of the tensor is column k of Omega)."""
    return nys_gaussian(ctx, seed, d * s).view(s, d)


def nys_factor_import(ctx: Context, U_rows: torch.Tensor, lam: Sequence[float], nu: float = 0.0) -> Factor:
    """Factor from U given as (r, d) FP64 rows (column-major d x r) and lambda."""
    r, d = U_rows.shape
    _vec(U_rows.reshape(-1), r * d, "U")
    lam_arr = (C.c_double * r)(*[float(v) for v in lam])
    h = C.c_void_p()
    _check(lib().nys_factor_import(ctx.h, d, r, _ptr(U_rows), lam_arr, float(nu), C.byref(h)),
           "nys_factor_import")
    return Factor(h, d)


def nys_sketch(ctx: Context, A: torch.Tensor, omega_rows: torch.Tensor, D: Optional[torch.Tensor] = None,
               c: float = 0.0, prec: int = NYS_F64, factor: Optional[Factor] = None) -> Factor:
    """Algorithm RandNysAppx (or one appended block if `factor` is given).
    omega_rows: (r, d) FP64 Gaussian entries."""
    dA = dense(A)
    r, d = omega_rows.shape
    _vec(omega_rows.reshape(-1), r * d, "omega")
    if D is not None:
        _vec(D, A.shape[0], "D")
    h = C.c_void_p(None if factor is None else factor.h.value)
    _check(lib().nys_sketch(ctx.h, C.byref(dA), _ptr(D), float(c), _ptr(omega_rows), int(r), int(prec),
                            C.byref(h)), "nys_sketch")
    if factor is not None:
        factor.h = h
        return factor
    return Factor(h, d)


def nys_sketch_adaptive(ctx: Context, A: torch.Tensor, omega_rows: torch.Tensor, s0: int, s_max: int,
                        rho: float, tol: float, D: Optional[torch.Tensor] = None, c: float = 0.0,
                        prec: int = NYS_F64) -> Factor:
    dA = dense(A)
    s, d = omega_rows.shape
    if s < s_max:
        raise ValueError("omega must hold s_max columns")
    _vec(omega_rows.reshape(-1), s * d, "omega")
    h = C.c_void_p()
    _check(lib().nys_sketch_adaptive(ctx.h, C.byref(dA), _ptr(D), float(c), _ptr(omega_rows), int(s0),
                                     int(s_max), float(rho), float(tol), int(prec), C.byref(h)),
           "nys_sketch_adaptive")
    return Factor(h, d)


def nys_hessian_apply(ctx: Context, A: torch.Tensor, p: torch.Tensor, rho: float = 0.0,
                      D: Optional[torch.Tensor] = None, c: float = 0.0, out: Optional[torch.Tensor] = None,
                      want_pv: bool = False):
    dA = dense(A)
    _vec(p, A.shape[1], "p")
    v = torch.empty_like(p) if out is None else out
    pv = C.c_double()
    _check(lib().nys_hessian_apply(ctx.h, C.byref(dA), _ptr(D), float(c), float(rho), _ptr(p), _ptr(v),
                                   C.byref(pv) if want_pv else None), "nys_hessian_apply")
    return (v, pv.value) if want_pv else v


def nys_hessian_apply_noalloc(ctx: Context, A: torch.Tensor, p: torch.Tensor, out: torch.Tensor,
                              rho: float = 0.0, D: Optional[torch.Tensor] = None, c: float = 0.0,
                              want_pv: bool = False):
    """nys_hessian_apply without device allocation in the library (scratch is
    the library's static array); `out` is the caller's FP64 d-vector."""
    dA = dense(A)
    _vec(p, A.shape[1], "p")
    _vec(out, A.shape[1], "out")
    if D is not None:
        _vec(D, A.shape[0], "D")
    pv = C.c_double()
    _check(lib().nys_hessian_apply_noalloc(ctx.h, C.byref(dA), _ptr(D), float(c), float(rho),
                                           _ptr(p), _ptr(out), C.byref(pv) if want_pv else None),
           "nys_hessian_apply_noalloc")
    return (out, pv.value) if want_pv else out


def nys_precond_apply(ctx: Context, F: Factor, rho: float, w: torch.Tensor,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _vec(w, F.d, "w")
    y = torch.empty_like(w) if out is None else out
    _check(lib().nys_precond_apply(ctx.h, F.h, float(rho), _ptr(w), _ptr(y)), "nys_precond_apply")
    return y


def pcg_opts(tol=1e-6, tol_abs=False, max_iter=1000, check_every=0, true_residual=True,
             max_restarts=2) -> PcgOpts:
    return PcgOpts(float(tol), int(bool(tol_abs)), int(max_iter), int(check_every),
                   int(bool(true_residual)), int(max_restarts))


def pcg_solve(ctx: Context, A: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor, rho: float,
              F: Optional[Factor] = None, D: Optional[torch.Tensor] = None, c: float = 0.0,
              opts: Optional[PcgOpts] = None, allow=(NYS_OK,)) -> PcgInfo:
    """Solve (A^T D A + (c + rho) I) x = rhs in place (x holds x0)."""
    dA = dense(A)
    _vec(rhs, A.shape[1], "rhs")
    _vec(x, A.shape[1], "x")
    if D is not None:
        _vec(D, A.shape[0], "D")
    o = opts or pcg_opts()
    info = PcgInfo()
    st = lib().pcg_solve(ctx.h, C.byref(dA), _ptr(D), float(c), float(rho),
                         None if F is None else F.h, _ptr(rhs), _ptr(x), C.byref(o), C.byref(info))
    _check(st, "pcg_solve", ok=tuple(allow))
    return info


def kernel_rbf(ctx: Context, X: torch.Tensor, gamma: float, b: Optional[torch.Tensor] = None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """H = diag(b) K diag(b) (K without b) for the RBF kernel of the rows of
    X (CUDA float32, n x p, unit column stride); returns the FP32 n x n matrix."""
    if X.dim() != 2 or not X.is_cuda or X.dtype != torch.float32 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D CUDA float32 tensor with unit column stride")
    n, p = X.shape
    if b is not None:
        _vec(b, n, "b")
    H = torch.empty((n, n), dtype=torch.float32, device=X.device) if out is None else out
    if H.shape != (n, n) or H.dtype != torch.float32 or H.stride(1) != 1:
        raise ValueError("out must be a float32 n x n tensor with unit column stride")
    ldx = X.stride(0) if n > 1 else p
    _check(lib().nys_kernel_rbf(ctx.h, _ptr(X), n, p, max(ldx, p), _ptr(b), float(gamma), _ptr(H),
                                H.stride(0) if n > 1 else n), "nys_kernel_rbf")
    return H


def nys_sketch_sym(ctx: Context, K: torch.Tensor, omega_rows: torch.Tensor, c: float = 0.0,
                   factor: Optional["Factor"] = None, prec: int = NYS_F64) -> "Factor":
    """Algorithm RandNysAppx of the explicit symmetric K + c I (FP64 core;
    K Omega in FP64, or in FP32 with prec=NYS_F32)."""
    dK = dense(K)
    r, d = omega_rows.shape
    _vec(omega_rows.reshape(-1), r * d, "omega")
    h = C.c_void_p(None if factor is None else factor.h.value)
    _check(lib().nys_sketch_sym(ctx.h, C.byref(dK), float(c), _ptr(omega_rows), int(r), int(prec),
                                C.byref(h)), "nys_sketch_sym")
    if factor is not None:
        factor.h = h
        return factor
    return Factor(h, d)


def pcg_solve_sym(ctx: Context, K: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor, rho: float,
                  F: Optional["Factor"] = None, c: float = 0.0, opts: Optional[PcgOpts] = None,
                  allow=(NYS_OK,)) -> PcgInfo:
    """Solve (K + (c + rho) I) x = rhs in place for an explicit symmetric K."""
    dK = dense(K)
    _vec(rhs, K.shape[0], "rhs")
    _vec(x, K.shape[0], "x")
    o = opts or pcg_opts()
    info = PcgInfo()
    st = lib().pcg_solve_sym(ctx.h, C.byref(dK), float(c), float(rho), None if F is None else F.h,
                             _ptr(rhs), _ptr(x), C.byref(o), C.byref(info))
    _check(st, "pcg_solve_sym", ok=tuple(allow))
    return info


def _keep(struct, *objs):
    """Attach the tensors and handles whose addresses `struct` holds, so that
    they live as long as the struct does (ctypes stores only the raw pointer)."""
    struct._keep = tuple(o for o in objs if o is not None)
    return struct


def svm_opts(rho, rank, omega_rows: Optional[torch.Tensor] = None, pcg: Optional[PcgOpts] = None,
             max_iter=100, gap_tol=0.0, gap_every=10, true_res_every=1,
             factor: Optional["Factor"] = None) -> SvmOpts:
    o = SvmOpts(float(rho), int(rank), None if omega_rows is None else omega_rows.data_ptr(),
                pcg or pcg_opts(), int(max_iter), float(gap_tol), int(gap_every),
                int(true_res_every), None if factor is None else factor.h.value)
    return _keep(o, omega_rows, factor)


def svm_solve(ctx: Context, H: torch.Tensor, b: torch.Tensor, Cbox: float, opts: SvmOpts,
              state: "State", allow=(NYS_OK,)) -> SvmInfo:
    """NysADMM on the kernel SVM dual with H = diag(b) K diag(b)."""
    _vec(b, H.shape[0], "b")
    P = SvmProblem(dense(H), b.data_ptr(), float(Cbox))
    S = state.c()
    info = SvmInfo()
    _check(lib().svm_solve(ctx.h, C.byref(P), C.byref(opts), C.byref(S), C.byref(info)),
           "svm_solve", ok=tuple(allow))
    state.k = S.k
    return info


def admm_opts(rho, rank, omega_rows: Optional[torch.Tensor], rank_max=0, ada_tol=0.0, resketch_every=0,
              sketch_prec=NYS_F64, pcg: Optional[PcgOpts] = None, tol_schedule=False, max_iter=100,
              eps_abs=0.0, eps_rel=0.0, rel_change_tol=0.0, kkt_tol=0.0, kkt_every=10,
              factor: Optional["Factor"] = None, warm_start: Optional["WarmStart"] = None,
              ws_analytic=False, ws_every_step=False, ws_features: Optional[torch.Tensor] = None,
              ws_target: Optional[torch.Tensor] = None, true_res_every=1) -> AdmmOpts:
    for t, name in ((ws_features, "ws_features"), (ws_target, "ws_target")):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous CUDA float64 tensor")
    o = AdmmOpts(float(rho), int(rank), int(rank_max), float(ada_tol), int(resketch_every),
                 int(sketch_prec), None if omega_rows is None else omega_rows.data_ptr(),
                 pcg or pcg_opts(), int(bool(tol_schedule)),
                 int(max_iter), float(eps_abs), float(eps_rel), float(rel_change_tol),
                 float(kkt_tol), int(kkt_every), None if factor is None else factor.h.value,
                 None if warm_start is None else warm_start.h.value, int(bool(ws_analytic)),
                 int(bool(ws_every_step)),
                 None if ws_features is None else ws_features.data_ptr(),
                 None if ws_target is None else ws_target.data_ptr(), int(true_res_every))
    return _keep(o, omega_rows, factor, warm_start, ws_features, ws_target)


def problem(A: torch.Tensor, b: torch.Tensor, gamma: float, loss=NYS_LOSS_LS, c: float = 0.0) -> Problem:
    _vec(b, A.shape[0], "b")
    return _keep(Problem(int(loss), dense(A), b.data_ptr(), float(gamma), float(c)), A, b)


class State:
    """Caller-owned ADMM state (x, z, u) on the device."""

    def __init__(self, d: int, device, x=None, z=None, u=None, k: int = 0):
        z0 = lambda: torch.zeros(d, dtype=torch.float64, device=device)
        self.x = z0() if x is None else x
        self.z = z0() if z is None else z
        self.u = z0() if u is None else u
        self.k = k

    def c(self) -> AdmmState:
        return AdmmState(self.x.data_ptr(), self.z.data_ptr(), self.u.data_ptr(), int(self.k))


def admm_step(ctx: Context, prob: Problem, opts: AdmmOpts, F: Optional[Factor], state: State,
              allow=(NYS_OK,)):
    """One NysADMM iteration; returns (factor, info)."""
    h = C.c_void_p(None if F is None else F.h.value)
    cs = state.c()
    info = AdmmInfo()
    st = lib().admm_step(ctx.h, C.byref(prob), C.byref(opts), C.byref(h), C.byref(cs), C.byref(info))
    _check(st, "admm_step", ok=tuple(allow))
    state.k = cs.k
    if F is None:
        F = Factor(h, prob.A.d) if h.value else None
    else:
        F.h = h
    return F, info


def admm_solve(ctx: Context, probs: Sequence[Problem], opts: Sequence[AdmmOpts], states: Sequence[State],
               allow=(NYS_OK,)):
    n = len(probs)
    P = (Problem * n)(*probs)
    O = (AdmmOpts * n)(*opts)
    S = (AdmmState * n)(*[s.c() for s in states])
    I = (AdmmInfo * n)()
    st = lib().admm_solve(ctx.h, n, P, O, S, I)
    _check(st, "admm_solve", ok=tuple(allow))
    for s, cs in zip(states, S):
        s.k = cs.k
    return list(I)


def nys_ws_param_count(n_in: int, hidden: int, n_out: int) -> int:
    return int(lib().nys_ws_param_count(int(n_in), int(hidden), int(n_out)))


def _host_f64(a, n, name):
    if a is None:
        return None
    t = torch.as_tensor(a, dtype=torch.float64).contiguous().cpu()
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} values")
    return t


class WarmStart:
    """Warm-start network on the device (nys_ws_*): n_in -> hidden -> hidden ->
    n_out with GELU, FP64 parameters W1 b1 W2 b2 W3 b3 (row-major, flat).
    analytic_skip: the proposal is the analytic coefficients plus the output."""

    def __init__(self, ctx: "Context", n_in: int, hidden: int, n_out: int, params,
                 in_mean=None, in_std=None, out_scale=None, analytic_skip=False):
        self.ctx = ctx
        self.n_in, self.hidden, self.n_out = int(n_in), int(hidden), int(n_out)
        self.count = nys_ws_param_count(n_in, hidden, n_out)
        self.analytic_skip = bool(analytic_skip)
        P = _host_f64(params, self.count, "params")
        mu = _host_f64(in_mean, n_in, "in_mean")
        sd = _host_f64(in_std, n_in, "in_std")
        so = _host_f64(out_scale, n_out, "out_scale")
        self.out_scale = so if so is not None else torch.ones(n_out, dtype=torch.float64)
        dp = lambda t: None if t is None else C.cast(t.data_ptr(), C.POINTER(C.c_double))
        self.h = C.c_void_p()
        _check(lib().nys_ws_create(ctx.h, self.n_in, self.hidden, self.n_out, dp(P), dp(mu),
                                   dp(sd), dp(so), int(bool(analytic_skip)), C.byref(self.h)),
               "nys_ws_create")

    def _rows(self, X, n, name):
        if X.dtype != torch.float64 or not X.is_cuda or not X.is_contiguous() or X.dim() != 2 \
                or X.shape[1] != n:
            raise ValueError(f"{name} must be a contiguous CUDA float64 (batch, {n}) tensor")
        return X

    def set_precision(self, prec: int):
        """NYS_F64 (default), NYS_F32 or NYS_BF16 (FP32 master weights, MFMA products)."""
        _check(lib().nys_ws_set_precision(self.ctx.h, self.h, int(prec)), "nys_ws_set_precision")
        self.prec = int(prec)

    def params(self) -> torch.Tensor:
        out = torch.empty(self.count, dtype=torch.float64)
        _check(lib().nys_ws_get_params(self.ctx.h, self.h,
                                       C.cast(out.data_ptr(), C.POINTER(C.c_double))),
               "nys_ws_get_params")
        return out

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        self._rows(X, self.n_in, "X")
        out = torch.empty(X.shape[0], self.n_out, dtype=torch.float64, device=X.device)
        _check(lib().nys_ws_forward(self.ctx.h, self.h, _ptr(X), X.shape[0], _ptr(out)),
               "nys_ws_forward")
        self.ctx.synchronize()
        return out

    def loss_grad(self, X, T, W=None, want_grad=True):
        self._rows(X, self.n_in, "X")
        self._rows(T, self.n_out, "T")
        if W is not None:
            self._rows(W, self.n_out, "W")
        loss = C.c_double()
        g = torch.empty(self.count, dtype=torch.float64, device=X.device) if want_grad else None
        _check(lib().nys_ws_loss_grad(self.ctx.h, self.h, _ptr(X), _ptr(T), _ptr(W), X.shape[0],
                                      C.byref(loss), _ptr(g)), "nys_ws_loss_grad")
        self.ctx.synchronize()
        return loss.value, g

    def train_step(self, X, T, W=None, lr=1e-3) -> float:
        self._rows(X, self.n_in, "X")
        self._rows(T, self.n_out, "T")
        if W is not None:
            self._rows(W, self.n_out, "W")
        loss = C.c_double()
        _check(lib().nys_ws_train_step(self.ctx.h, self.h, _ptr(X), _ptr(T), _ptr(W), X.shape[0],
                                       float(lr), C.byref(loss)), "nys_ws_train_step")
        return loss.value

    def close(self):
        if self.h is not None and self.h.value:
            lib().nys_ws_destroy(self.h)
            self.h = C.c_void_p()
