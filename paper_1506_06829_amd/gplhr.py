"""Python binding of the GPLHR HIP library (argument marshalling only).

Every computation runs inside ``libgplhr.so`` (hand-written HIP for gfx950 plus
host C++ for the small projected step); this module only passes device
pointers of torch tensors and the current HIP stream across the C ABI declared
in ``include/gplhr.h``.  If the library has not been built, importing works but
every call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from pathlib import Path
from typing import Optional

import numpy as np
import torch

_LIB_PATH = Path(__file__).resolve().parent / "libgplhr.so"
_lib = None

OK, NOT_CONVERGED = 0, 1
_STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_ALLOC", -3: "ERR_HIP",
           -4: "ERR_BREAKDOWN", -5: "ERR_SINGULAR_SHIFT", -6: "ERR_NUMERIC",
           -7: "ERR_NOT_SIMPLE", -8: "ERR_STATE"}
PRECOND = {"none": 0, "diag": 1, "jacobi": 2, "gmres": 3}


class GplhrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Precond(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("sweeps", ctypes.c_int), ("omega", ctypes.c_double),
                ("steps", ctypes.c_int), ("inner", ctypes.c_int)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("arnoldi_m", ctypes.c_int), ("p_mode", ctypes.c_int), ("V0", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
                ("switch_tol", ctypes.c_double), ("stall_window", ctypes.c_int),
                ("timing", ctypes.c_int), ("proj_before_T", ctypes.c_int),
                ("locking", ctypes.c_int), ("m_max", ctypes.c_int),
                ("algorithm", ctypes.c_int), ("defl_V", ctypes.c_void_p),
                ("defl_Q", ctypes.c_void_p), ("defl_k", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("fp64_iterations", ctypes.c_int64),
                ("spmm_calls", ctypes.c_int64), ("precond_calls", ctypes.c_int64),
                ("breakdowns", ctypes.c_int64), ("spmm_ms", ctypes.c_double),
                ("spmm_bytes", ctypes.c_double), ("gram_ms", ctypes.c_double),
                ("update_ms", ctypes.c_double), ("small_host_ms", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double),
                ("max_rel_resid", ctypes.c_double), ("n_converged", ctypes.c_int),
                ("phase", ctypes.c_int), ("locked", ctypes.c_int),
                ("arnoldi_m", ctypes.c_int)]


EXPORTS = ["gplhr_default_options", "gplhr_create", "gplhr_iterate", "gplhr_get_schur",
           "gplhr_get_eigvecs", "gplhr_get_eig", "gplhr_eig_backward", "gplhr_get_stats",
           "gplhr_destroy",
           "gplhr_last_error", "gplhr_spmm", "gplhr_csr_plane", "gplhr_gram", "gplhr_jacobi",
           "gplhr_block_update", "gplhr_gram_noalloc", "gplhr_get_residual_norms",
           "gplhr_block_copy", "gplhr_proj_orth"]


def lib():
    """Load ``libgplhr.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1506_06829_amd.build`")
    L = ctypes.CDLL(str(_LIB_PATH))
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.gplhr_default_options.argtypes = [ctypes.POINTER(_Options)]
    L.gplhr_default_options.restype = None
    L.gplhr_create.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_Csr), dbl, dbl, i32, i32,
                               ctypes.POINTER(_Precond), ctypes.POINTER(_Options), ctypes.POINTER(vp)]
    L.gplhr_create.restype = i32
    L.gplhr_iterate.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.gplhr_iterate.restype = i32
    L.gplhr_get_schur.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.gplhr_get_schur.restype = i32
    L.gplhr_get_residual_norms.argtypes = [vp, vp]
    L.gplhr_get_residual_norms.restype = i32
    L.gplhr_get_eigvecs.argtypes = [vp, vp]
    L.gplhr_get_eigvecs.restype = i32
    L.gplhr_get_eig.argtypes = [vp, vp, vp, vp, vp]
    L.gplhr_get_eig.restype = i32
    L.gplhr_eig_backward.argtypes = [vp, vp, vp, vp]
    L.gplhr_eig_backward.restype = i32
    L.gplhr_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
    L.gplhr_get_stats.restype = i32
    L.gplhr_destroy.argtypes = [vp]
    L.gplhr_destroy.restype = None
    L.gplhr_last_error.argtypes = [vp]
    L.gplhr_last_error.restype = ctypes.c_char_p
    L.gplhr_spmm.argtypes = [i32, i64, i64, vp, vp, vp, vp, i32, vp, i32, i32, i32, vp]
    L.gplhr_spmm.restype = i32
    L.gplhr_jacobi.argtypes = [i32, i64, i64, vp, vp, vp, ctypes.c_double, i32, vp, i32, vp, i32,
                               i32, i32, vp]
    L.gplhr_jacobi.restype = i32
    L.gplhr_csr_plane.argtypes = [i64, vp, vp, ctypes.POINTER(i32), vp]
    L.gplhr_csr_plane.restype = i32
    L.gplhr_gram.argtypes = [i32, i64, vp, i32, i32, vp, i32, i32, vp, vp]
    L.gplhr_gram.restype = i32
    L.gplhr_block_copy.argtypes = [i32, i64, vp, i32, vp, i32, i32, vp]
    L.gplhr_block_copy.restype = i32
    L.gplhr_gram_noalloc.argtypes = [i32, i64, vp, i32, i32, vp, i32, i32, vp, vp]
    L.gplhr_gram_noalloc.restype = i32
    L.gplhr_block_update.argtypes = [i32, i64, vp, i32, i32, vp, i32, vp, i32, i32,
                                     ctypes.c_double, ctypes.c_double, vp]
    L.gplhr_block_update.restype = i32
    L.gplhr_proj_orth.argtypes = [i32, i64, vp, i32, i32, i32, i32, vp]
    L.gplhr_proj_orth.restype = i32
    _lib = L
    return L


def _check(status: int, handle=None) -> int:
    if status < 0:
        msg = lib().gplhr_last_error(handle)
        raise GplhrError(status, msg.decode() if msg else "")
    return status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceCsr:
    """CSR matrix whose arrays live on the GPU (int32 indices, complex128 values)."""
    n: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @staticmethod
    def from_host(csr, device="cuda") -> "DeviceCsr":
        """From any object with n / indptr / indices / data (e.g. problems.Csr)."""
        return DeviceCsr(int(csr.n),
                         torch.as_tensor(np.asarray(csr.indptr, dtype=np.int32)).to(device),
                         torch.as_tensor(np.asarray(csr.indices, dtype=np.int32)).to(device),
                         torch.as_tensor(np.asarray(csr.data, dtype=np.complex128)).to(device))

    def _c(self) -> _Csr:
        assert self.row_ptr.dtype == torch.int32 and self.col_idx.dtype == torch.int32
        assert self.val.dtype == torch.complex128 and self.val.is_contiguous()
        return _Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                    self.val.data_ptr())


class Solver:
    """One GPLHR solve (a handle of the C library)."""

    def __init__(self, A: DeviceCsr, B: Optional[DeviceCsr], sigma: complex, k: int,
                 block: Optional[int] = None, precond: str = "diag", sweeps: int = 3,
                 omega: float = 0.7, precision: str = "fp64", tol: float = 1e-10,
                 max_iter: int = 500, m: int = 1, p_mode: str = "thick",
                 V0: Optional[torch.Tensor] = None, seed: int = 1, timing: bool = False,
                 switch_tol: float = 1e-8, stall_window: int = 3, stream=None,
                 proj_before_T: bool = True, locking: bool = False, m_max: int = 20,
                 steps: int = 2, inner: str = "jacobi", algorithm: str = "schur",
                 deflate: Optional[tuple] = None):
        L = lib()
        self.n, self.k = A.n, k
        self.block = block or k
        self._keep = (A, B, V0, deflate)
        opt = _Options()
        L.gplhr_default_options(ctypes.byref(opt))
        opt.precision = {"fp64": 0, "mixed": 1}[precision]
        opt.tol = tol
        opt.max_iter = max_iter
        opt.arnoldi_m = m
        opt.p_mode = {"thick": 0, "lobpcg": 1, "none": 2}[p_mode]
        if V0 is not None:
            assert V0.dtype == torch.complex128 and V0.is_contiguous()
            assert tuple(V0.shape) == (A.n, self.block)
            opt.V0 = V0.data_ptr()
        opt.seed = seed
        self._stream = torch.cuda.current_stream() if stream is None else stream
        opt.hip_stream = self._stream.cuda_stream
        opt.switch_tol = switch_tol
        opt.stall_window = stall_window
        opt.timing = 1 if timing else 0
        opt.proj_before_T = 1 if proj_before_T else 0
        opt.locking = 1 if locking else 0
        opt.m_max = m_max
        opt.algorithm = {"schur": 0, "eig": 1}[algorithm]
        if deflate is not None:
            # (V1, Q1): converged Schur bases to deflate (Q1 may be None for B = I)
            V1, Q1 = deflate
            for t in (V1, Q1):
                if t is not None:
                    assert t.dtype == torch.complex128 and t.is_contiguous() and t.shape[0] == A.n
            opt.defl_V = V1.data_ptr()
            opt.defl_Q = Q1.data_ptr() if Q1 is not None else None
            opt.defl_k = V1.shape[1]
        self.algorithm = algorithm
        # precond "gmres": `steps` block GMRES steps right-preconditioned by `inner`
        pre = _Precond(PRECOND[precond], sweeps, omega, steps, PRECOND[inner])
        a = A._c()
        b = B._c() if B is not None else None
        h = ctypes.c_void_p()
        st = L.gplhr_create(ctypes.byref(a), ctypes.byref(b) if b is not None else None,
                            float(complex(sigma).real), float(complex(sigma).imag), k,
                            self.block, ctypes.byref(pre), ctypes.byref(opt), ctypes.byref(h))
        _check(st, None)
        self.h = h

    def iterate(self, max_iter: int = 0):
        nc = ctypes.c_int()
        mr = ctypes.c_double()
        st = _check(lib().gplhr_iterate(self.h, max_iter, ctypes.byref(nc), ctypes.byref(mr)), self.h)
        return st, nc.value, mr.value

    def schur(self, want_vectors: bool = True):
        n, k = self.n, self.k
        V = torch.empty((n, k), dtype=torch.complex128, device="cuda") if want_vectors else None
        Q = torch.empty((n, k), dtype=torch.complex128, device="cuda") if want_vectors else None
        RA = np.zeros((k, k), dtype=np.complex128, order="F")
        RB = np.zeros((k, k), dtype=np.complex128, order="F")
        lam = np.zeros(k, dtype=np.complex128)
        rho = np.zeros(k, dtype=np.float64)
        _check(lib().gplhr_get_schur(self.h, _ptr(V), _ptr(Q), RA.ctypes.data, RB.ctypes.data,
                                     lam.ctypes.data, rho.ctypes.data), self.h)
        return dict(V=V, Q=Q, RA=RA, RB=RB, lam=lam, rho=rho)

    def eig(self, want_vectors: bool = True):
        """GPLHR-EIG output: X, Lambda_A, Lambda_B (diagonals), lam = LA / LB, rho."""
        n, k = self.n, self.k
        X = torch.empty((n, k), dtype=torch.complex128, device="cuda") if want_vectors else None
        LA = np.zeros(k, dtype=np.complex128)
        LB = np.zeros(k, dtype=np.complex128)
        rho = np.zeros(k, dtype=np.float64)
        _check(lib().gplhr_get_eig(self.h, _ptr(X), LA.ctypes.data, LB.ctypes.data,
                                   rho.ctypes.data), self.h)
        return dict(X=X, LA=LA, LB=LB, lam=LA / LB, rho=rho)

    def lam(self) -> np.ndarray:
        """Current eigenvalue approximations of the k leading columns."""
        if self.algorithm == "eig":
            return self.eig(want_vectors=False)["lam"]
        return self.schur(want_vectors=False)["lam"]

    def residual_norms(self) -> np.ndarray:
        """||A x_j - lambda_j B x_j|| / ||x_j|| of the k leading pairs (unit x_j)."""
        out = np.zeros(self.k, dtype=np.float64)
        _check(lib().gplhr_get_residual_norms(self.h, out.ctypes.data), self.h)
        return out

    def eigvecs(self) -> torch.Tensor:
        X = torch.empty((self.n, self.k), dtype=torch.complex128, device="cuda")
        _check(lib().gplhr_get_eigvecs(self.h, _ptr(X)), self.h)
        return X

    def backward(self, grad_lambda: np.ndarray, nnzA: int, nnzB: Optional[int]):
        g = np.ascontiguousarray(np.asarray(grad_lambda, dtype=np.complex128))
        gA = torch.empty(nnzA, dtype=torch.complex128, device="cuda")
        gB = torch.empty(nnzB, dtype=torch.complex128, device="cuda") if nnzB else None
        _check(lib().gplhr_eig_backward(self.h, g.ctypes.data, _ptr(gA), _ptr(gB)), self.h)
        return gA, gB

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().gplhr_get_stats(self.h, ctypes.byref(s)), self.h)
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().gplhr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmm(A: DeviceCsr, X: torch.Tensor, Y: Optional[torch.Tensor] = None,
         val: Optional[torch.Tensor] = None, plane: int = 0) -> torch.Tensor:
    """Y = A X with the library's CSR kernel; complex128 or complex64 blocks
    (``val`` overrides A's values, e.g. a complex64 copy).  ``plane`` selects
    the row schedule (0: natural order; see csr_plane)."""
    v = A.val if val is None else val
    dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
    assert v.dtype == X.dtype and X.dim() == 2 and X.stride(1) == 1
    b = X.shape[1]
    if Y is None:
        Y = torch.empty((A.n, b), dtype=X.dtype, device=X.device)
    _check(lib().gplhr_spmm(dtype, A.n, A.nnz, _ptr(A.row_ptr), _ptr(A.col_idx), _ptr(v), _ptr(X),
                            X.stride(0), _ptr(Y), Y.stride(0), b, int(plane), _stream_ptr()))
    return Y


def jacobi(A: DeviceCsr, R: torch.Tensor, omega: float = 0.7, sweeps: int = 3,
           plane: int = 0) -> torch.Tensor:
    """Y = T R for ``sweeps`` damped Jacobi steps on A (complex128 values)
    from zero, with the library's kernels; R complex128 or complex64."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[R.dtype]
    assert R.dim() == 2 and R.stride(1) == 1 and A.val.dtype == torch.complex128
    b = R.shape[1]
    Y = torch.empty((A.n, b), dtype=R.dtype, device=R.device)
    _check(lib().gplhr_jacobi(dtype, A.n, A.nnz, _ptr(A.row_ptr), _ptr(A.col_idx), _ptr(A.val),
                              float(omega), int(sweeps), _ptr(R), R.stride(0), _ptr(Y), b, b,
                              int(plane), _stream_ptr()))
    return Y


def csr_plane(A: DeviceCsr) -> int:
    """The plane-slab row schedule the solver uses for A's pattern (0: none)."""
    out = ctypes.c_int(0)
    _check(lib().gplhr_csr_plane(A.n, _ptr(A.row_ptr), _ptr(A.col_idx), ctypes.byref(out),
                                 _stream_ptr()))
    return int(out.value)


def block_update(X: torch.Tensor, M: torch.Tensor, Y: Optional[torch.Tensor] = None,
                 beta: complex = 0.0) -> torch.Tensor:
    """Y = beta Y + X M with the library's row-local update (X, Y complex128 or
    complex64 row-major with unit column stride, M complex128 wx-by-wy); Y may
    be X itself."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
    wx, wy = X.shape[1], M.shape[1]
    assert X.dim() == 2 and X.stride(1) == 1 and M.shape[0] == wx
    assert M.dtype == torch.complex128
    Mc = M.t().contiguous()                       # column-major wx x wy
    if Y is None:
        Y = torch.zeros((X.shape[0], wy), dtype=X.dtype, device=X.device)
    assert Y.dtype == X.dtype and Y.stride(1) == 1 and Y.shape == (X.shape[0], wy)
    beta = complex(beta)
    _check(lib().gplhr_block_update(dtype, X.shape[0], _ptr(X), X.stride(0), wx, _ptr(Mc), wx,
                                    _ptr(Y), Y.stride(0), wy, beta.real, beta.imag,
                                    _stream_ptr()))
    return Y


def proj_orth(Z: torch.Tensor, wy: int, w: int, passes: int = 2) -> torch.Tensor:
    """Z[:, wy:wy+w] <- orth((I - Y Y^H) Z[:, wy:wy+w]) for the orthonormal
    Y = Z[:, :wy], in place, with the library's Gram, Cholesky and update
    kernels (Z complex128 or complex64, row-major with unit column stride)."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[Z.dtype]
    assert Z.dim() == 2 and Z.stride(1) == 1 and Z.shape[1] >= wy + w
    _check(lib().gplhr_proj_orth(dtype, Z.shape[0], _ptr(Z), Z.stride(0), wy, w, passes,
                                 _stream_ptr()))
    return Z


def gram(X: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
    """G = X^H Y (complex128, FP64 accumulation) with the library's kernel."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
    assert X.dtype == Y.dtype and X.stride(1) == 1 and Y.stride(1) == 1
    bx, by = X.shape[1], Y.shape[1]
    G = torch.empty((by, bx), dtype=torch.complex128, device=X.device)   # column-major bx x by
    _check(lib().gplhr_gram(dtype, X.shape[0], _ptr(X), X.stride(0), bx, _ptr(Y), Y.stride(0),
                            by, _ptr(G), _stream_ptr()))
    return G.t()


def block_copy(X: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
    """Y = X with the library's streaming block-copy kernel (row-major,
    complex128 or complex64)."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
    assert X.dtype == Y.dtype and X.shape == Y.shape and X.stride(1) == 1 and Y.stride(1) == 1
    _check(lib().gplhr_block_copy(dtype, X.shape[0], _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
                                  X.shape[1], _stream_ptr()))
    return Y


def gram_noalloc(X: torch.Tensor, Y: torch.Tensor, G: torch.Tensor) -> torch.Tensor:
    """G = X^H Y through the allocation-free entry point; the output G is
    the caller's (by-by-bx complex128 storage, i.e. bx-by-by column-major),
    returned as the bx-by-by view."""
    dtype = {torch.complex128: 0, torch.complex64: 1}[X.dtype]
    assert X.dtype == Y.dtype and X.stride(1) == 1 and Y.stride(1) == 1
    bx, by = X.shape[1], Y.shape[1]
    assert G.dtype == torch.complex128 and G.is_contiguous() and tuple(G.shape) == (by, bx)
    _check(lib().gplhr_gram_noalloc(dtype, X.shape[0], _ptr(X), X.stride(0), bx, _ptr(Y),
                                    Y.stride(0), by, _ptr(G), _stream_ptr()))
    return G.t()


class GPLHREig(torch.autograd.Function):
    """k eigenvalues of (A, B) nearest sigma as a differentiable function of
    the stored values of A and B (hand-written backward through the adjoint
    pencil and a sampled dense-dense product; see gplhr_eig_backward)."""

    @staticmethod
    def forward(ctx, valA, valB, A: DeviceCsr, B: Optional[DeviceCsr], sigma, k, opts):
        A2 = DeviceCsr(A.n, A.row_ptr, A.col_idx, valA.detach().contiguous())
        B2 = None if B is None else DeviceCsr(B.n, B.row_ptr, B.col_idx, valB.detach().contiguous())
        s = Solver(A2, B2, sigma, k, **(opts or {}))
        st, _, res = s.iterate()
        if st != OK:
            raise GplhrError(NOT_CONVERGED, f"forward solve did not converge (residual {res:.3e})")
        lam = s.lam()
        ctx.solver = s
        ctx.nnzA = A.nnz
        ctx.nnzB = None if B is None else B.nnz
        return torch.as_tensor(lam, dtype=torch.complex128, device=valA.device)

    @staticmethod
    def backward(ctx, grad_lam):
        g = grad_lam.detach().to("cpu", torch.complex128).numpy()
        gA, gB = ctx.solver.backward(g, ctx.nnzA, ctx.nnzB)
        ctx.solver.close()
        return gA, gB, None, None, None, None, None
