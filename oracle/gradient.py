"""Dense FP64 reference for eigenvalue derivatives -- TEST INFRASTRUCTURE ONLY.

For a simple eigenvalue lambda of the pencil (A, B) with right eigenvector x
(A x = lambda B x) and left eigenvector y (y^H A = lambda y^H B), first-order
perturbation theory gives

    d lambda = (y^H dA x - lambda y^H dB x) / (y^H B x).

For a real loss L(lambda_1..lambda_k) with g_e = dL/dRe(lambda_e) +
i dL/dIm(lambda_e), the gradient with respect to a stored complex entry (i, j)
of A (same convention, dL/dRe + i dL/dIm) is

    sum_e g_e y_e[i] conj(x_e[j]) / conj(y_e^H B x_e),

and for an entry of B the same with an extra factor -conj(lambda_e).  The left
and right eigenvectors come from LAPACK (scipy.linalg.eig with left=True) on
the dense pencil, so this reference is independent of GPLHR.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def nearest_eigs_dense(A: np.ndarray, B: np.ndarray, sigma: complex, k: int):
    """k eigenvalues of (A, B) nearest sigma with left/right eigenvectors."""
    w, vl, vr = sla.eig(A, B, left=True, right=True)
    order = np.argsort(np.abs(w - sigma), kind="stable")[:k]
    return w[order], vl[:, order], vr[:, order]


def eig_grad_dense(A: np.ndarray, B: np.ndarray, sigma: complex, k: int,
                   grad_lambda: np.ndarray, rows_a, cols_a, rows_b=None, cols_b=None):
    """Gradients on the listed entries of A (and B) of a loss whose gradient
    with respect to the k eigenvalues nearest sigma is grad_lambda (ordered
    like the returned eigenvalues)."""
    lam, Y, X = nearest_eigs_dense(A, B, sigma, k)
    denom = np.einsum("ie,ij,je->e", Y.conj(), B, X)
    c = grad_lambda / np.conj(denom)
    gA = np.einsum("e,ie,ie->i", c, Y[rows_a, :], X[cols_a, :].conj())
    gB = None
    if rows_b is not None:
        gB = np.einsum("e,ie,ie->i", -c * np.conj(lam), Y[rows_b, :], X[cols_b, :].conj())
    return lam, gA, gB


def nearest_eigs_sparse(A, B, sigma: complex, k: int, extra: int = 6, tol: float = 1e-14):
    """The same eigentriplets as ``nearest_eigs_dense`` for sparse A, B, by
    ARPACK shift-and-invert (scipy.sparse.linalg.eigs with the given sigma,
    which factors A - sigma B): k + extra eigenpairs of (A, B) nearest sigma,
    and of the adjoint pair (A^H, B^H) nearest conj(sigma) for the left
    eigenvectors (y^H A = lambda y^H B).  The k nearest are kept, each left
    vector paired with the adjoint eigenvalue nearest conj(lambda).  Both
    solves go through LAPACK's LU of the shifted matrix and ARPACK's
    Arnoldi iteration, independent of GPLHR."""
    A = sp.csc_matrix(A, dtype=complex)
    B = sp.csc_matrix(B, dtype=complex)
    m = k + extra

    def shifted_inverse(M, N, s):
        # (M - s N)^{-1} from a dense LU (a random sparse matrix fills in)
        lu = sla.lu_factor((M - s * N).toarray())
        return spla.LinearOperator(M.shape, matvec=lambda x: sla.lu_solve(lu, x), dtype=complex)

    ncv = min(A.shape[0], max(2 * m + 1, 80))
    w, X = spla.eigs(A, k=m, M=B, sigma=sigma, tol=tol, ncv=ncv, OPinv=shifted_inverse(A, B, sigma))
    order = np.argsort(np.abs(w - sigma), kind="stable")[:k]
    lam, X = w[order], X[:, order]
    AH, BH = A.conj().T.tocsc(), B.conj().T.tocsc()
    wl, Yl = spla.eigs(AH, k=m, M=BH, sigma=np.conj(sigma), tol=tol, ncv=ncv,
                       OPinv=shifted_inverse(AH, BH, np.conj(sigma)))
    Y = np.empty_like(X)
    for e in range(k):
        j = int(np.argmin(np.abs(wl - np.conj(lam[e]))))
        Y[:, e] = Yl[:, j]
    return lam, Y, X


def eig_grad(A, B, sigma: complex, k: int, grad_lambda: np.ndarray, rows_a, cols_a,
             rows_b=None, cols_b=None, sparse: bool = False):
    """``eig_grad_dense`` with the eigentriplets from ``nearest_eigs_sparse``
    (sparse=True; A, B sparse) or from LAPACK on the dense pencil."""
    if not sparse:
        return eig_grad_dense(A, B, sigma, k, grad_lambda, rows_a, cols_a, rows_b, cols_b)
    lam, Y, X = nearest_eigs_sparse(A, B, sigma, k)
    Bs = sp.csr_matrix(B)
    denom = np.einsum("ie,ie->e", Y.conj(), Bs @ X)
    c = grad_lambda / np.conj(denom)
    gA = np.einsum("e,ie,ie->i", c, Y[rows_a, :], X[cols_a, :].conj())
    gB = None
    if rows_b is not None:
        gB = np.einsum("e,ie,ie->i", -c * np.conj(lam), Y[rows_b, :], X[cols_b, :].conj())
    return lam, gA, gB
