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
