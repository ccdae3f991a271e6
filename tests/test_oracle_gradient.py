"""Pins of the dense eigenvalue-derivative reference (oracle/gradient.py):
central finite differences and a closed-form special case."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gradient as OG


def loss_and_lam(A, B, sigma, k):
    w = sla.eigvals(A, B)
    lam = w[np.argsort(np.abs(w - sigma), kind="stable")[:k]]
    return float(np.sum(np.abs(lam - sigma) ** 2)), lam


def test_diagonal_matrix_unit_derivatives():
    # A diagonal, B = I: d lambda_i / d a_ii = 1 and every other entry gives 0
    n, sigma, k = 8, 2.1, 3
    A = np.diag(np.arange(n, dtype=complex))
    B = np.eye(n, dtype=complex)
    rows, cols = np.nonzero(np.ones((n, n)))
    lam, Y, X = OG.nearest_eigs_dense(A, B, sigma, k)
    for e in range(k):
        g = np.zeros(k, dtype=complex)
        g[e] = 1.0
        _, gA, _ = OG.eig_grad_dense(A, B, sigma, k, g, rows, cols)
        G = gA.reshape(n, n)
        i = int(round(lam[e].real))
        expect = np.zeros((n, n))
        expect[i, i] = 1.0
        np.testing.assert_allclose(G, expect, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    n, k = 20, 3
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2) + 3 * np.eye(n)
    B = (np.eye(n) + 0.1 * rng.standard_normal((n, n))).astype(complex)
    sigma = 2.5 + 0.5j
    L0, lam = loss_and_lam(A, B, sigma, k)
    g = 2 * (lam - sigma)            # dL/dRe + i dL/dIm of sum |lambda - sigma|^2
    ent = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(6)]
    ra, ca = zip(*ent)
    _, gA, gB = OG.eig_grad_dense(A, B, sigma, k, g, np.array(ra), np.array(ca),
                                  np.array(ra), np.array(ca))
    h = 1e-6
    for t, (i, j) in enumerate(ent):
        for which, M, G in (("A", A, gA), ("B", B, gB)):
            fd = 0j
            for unit in (1.0, 1j):
                Mp, Mm = M.copy(), M.copy()
                Mp[i, j] += h * unit
                Mm[i, j] -= h * unit
                if which == "A":
                    lp, _ = loss_and_lam(Mp, B, sigma, k)
                    lm, _ = loss_and_lam(Mm, B, sigma, k)
                else:
                    lp, _ = loss_and_lam(A, Mp, sigma, k)
                    lm, _ = loss_and_lam(A, Mm, sigma, k)
                fd += unit * (lp - lm) / (2 * h)
            assert abs(G[t] - fd) <= 1e-6 * max(1.0, abs(fd)), (which, i, j, G[t], fd)


@pytest.mark.parametrize("seed", [0, 3])
def test_sparse_reference_matches_dense(seed):
    # the ARPACK shift-and-invert triplets give the same eigenvalues and the
    # same gradients as LAPACK on the dense pencil (random sparse pencil of
    # the gradient workload's family, n = 400)
    import scipy.sparse as sp
    from paper_1506_06829_amd import problems
    Acsr, Bcsr = problems.random_pencil(400, seed=seed)
    A, B = Acsr.to_scipy(), Bcsr.to_scipy()
    sigma, k = 0.0 + 0.0j, 6
    lam_d, _, _ = OG.nearest_eigs_dense(A.toarray(), B.toarray(), sigma, k)
    lam_s, Y, X = OG.nearest_eigs_sparse(A, B, sigma, k)
    np.testing.assert_allclose(lam_s, lam_d, rtol=1e-11)
    # left and right eigenvectors satisfy their equations
    for e in range(k):
        np.testing.assert_allclose(A @ X[:, e], lam_s[e] * (B @ X[:, e]), atol=1e-10 * np.abs(lam_s[e]))
        np.testing.assert_allclose(Y[:, e].conj() @ A, lam_s[e] * (Y[:, e].conj() @ B),
                                   atol=1e-10 * np.abs(lam_s[e]))
    g = 2 * (lam_d - sigma)
    ra = np.repeat(np.arange(400), np.diff(A.indptr))
    rb = np.repeat(np.arange(400), np.diff(B.indptr))
    _, gA_d, gB_d = OG.eig_grad_dense(A.toarray(), B.toarray(), sigma, k, g, ra, A.indices, rb, B.indices)
    _, gA_s, gB_s = OG.eig_grad(A, B, sigma, k, g, ra, A.indices, rb, B.indices, sparse=True)
    assert np.max(np.abs(gA_s - gA_d)) <= 1e-10 * np.max(np.abs(gA_d))
    assert np.max(np.abs(gB_s - gB_d)) <= 1e-10 * np.max(np.abs(gB_d))
