"""Seeded synthetic pencils (A, B, sigma, V0) shaped like the paper's workloads.

This module only *builds inputs*.  It holds none of the eigensolver's arithmetic
(no shifted operator, no preconditioner, no projection), so that both the HIP
path and the CPU oracle can consume exactly the same arrays without sharing
any of the method's code.

The paper's own test matrices (Table 1 of Section 5: Matrix Market, IFISS and a
quantum-chemistry resonance problem) are not available; these generators are
synthetic stand-ins of the same character: non-Hermitian convection-diffusion
operators (one of the paper's problems, PDE2961, is a 2-D variable-coefficient
elliptic PDE), interior targets and a shift inside the spectrum.

Conventions
-----------
* CSR with int32 ``indptr``/``indices`` sorted within each row, complex128
  values.  A ``Csr`` is a plain named tuple of numpy arrays.
* Stencils: unit square/cube, homogeneous Dirichlet boundary, N interior
  points per axis, h = 1/(N+1), operator  -Laplace(u) + c . grad(u)  scaled by
  1/h^2 (diffusion) and 1/h (convection), first-order upwind differences
  (backward difference for a positive velocity component), lexicographic
  ordering with x fastest.
* Diagonal B: ``numpy.random.default_rng(seed).uniform(1, 2, n)``.
* Starting block V0: complex normal, real and imaginary parts N(0, 1/2), drawn
  from ``default_rng(seed)`` as the real n-by-b array followed by the
  imaginary one.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import NamedTuple, Optional

import numpy as np
import scipy.sparse as sp


class Csr(NamedTuple):
    n: int
    indptr: np.ndarray   # int32, n+1
    indices: np.ndarray  # int32, nnz, sorted within rows
    data: np.ndarray     # complex128, nnz

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def csr_from_scipy(M) -> Csr:
    M = sp.csr_matrix(M, dtype=np.complex128)
    M.sum_duplicates()
    M.sort_indices()
    return Csr(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32),
               np.ascontiguousarray(M.data, dtype=np.complex128))


def _upwind_1d(N: int, c: float) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """1-D pieces on N interior points: second difference (scaled 1/h^2) and
    upwind first difference (scaled 1/h) times velocity c."""
    h = 1.0 / (N + 1)
    e = np.ones(N)
    lap = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr") / h**2
    if c >= 0:   # backward difference
        conv = sp.diags([-e[:-1], e], [-1, 0], format="csr") * (c / h)
    else:        # forward difference
        conv = sp.diags([-e, e[:-1]], [0, 1], format="csr") * (c / h)
    return lap, conv


def convection_diffusion(N: int, c: tuple[float, ...]) -> Csr:
    """2-D (len(c) == 2) or 3-D (len(c) == 3) upwind convection-diffusion."""
    d = len(c)
    I = sp.identity(N, format="csr")
    parts = [_upwind_1d(N, ci) for ci in c]
    A = None
    for axis in range(d):
        one = parts[axis][0] + parts[axis][1]
        # x is the fastest index: axis 0 is the innermost Kronecker factor.
        term = None
        for ax in reversed(range(d)):
            f = one if ax == axis else I
            term = f if term is None else sp.kron(term, f, format="csr")
        A = term if A is None else A + term
    return csr_from_scipy(A)


def diagonal_b(n: int, seed: int = 0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(1.0, 2.0, n)


def diag_csr(d: np.ndarray) -> Csr:
    n = d.shape[0]
    return Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               d.astype(np.complex128))


def random_pencil(n: int, seed: int = 0, offdiag_per_row: int = 16,
                  diag_shift: float = 8.0, b_pairs_per_row: float = 2.5,
                  b_scale: float = 0.1) -> tuple[Csr, Csr]:
    """Random sparse non-Hermitian pencil.

    A: per row ``offdiag_per_row`` distinct off-diagonal columns drawn uniformly
    without replacement, values (N(0,1) + i N(0,1))/sqrt(2); diagonal
    ``diag_shift`` + complex normal.
    B = I + b_scale * S with S real symmetric: round(b_pairs_per_row * n)
    uniformly drawn off-diagonal pairs (i != j) with N(0,1) values, mirrored,
    duplicates summed.
    """
    rng = np.random.default_rng(seed)
    q = offdiag_per_row
    cols = np.empty((n, q), dtype=np.int64)
    for i in range(n):
        c = rng.choice(n - 1, size=q, replace=False)
        c[c >= i] += 1
        cols[i] = c
    rows = np.repeat(np.arange(n), q)
    vals = (rng.standard_normal(n * q) + 1j * rng.standard_normal(n * q)) / np.sqrt(2)
    dvals = diag_shift + (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    A = sp.coo_matrix((np.concatenate([vals, dvals]),
                       (np.concatenate([rows, np.arange(n)]),
                        np.concatenate([cols.ravel(), np.arange(n)]))), shape=(n, n))
    npairs = int(round(b_pairs_per_row * n))
    i = rng.integers(0, n, npairs)
    j = rng.integers(0, n - 1, npairs)
    j[j >= i] += 1
    v = rng.standard_normal(npairs)
    S = sp.coo_matrix((np.concatenate([v, v]), (np.concatenate([i, j]), np.concatenate([j, i]))),
                      shape=(n, n))
    B = sp.identity(n, format="csr") + b_scale * S.tocsr()
    return csr_from_scipy(A), csr_from_scipy(B)


def diag_dominant_pencil(n: int, seed: int = 0, offdiag_per_row: int = 16,
                         coupling: float = 0.5, with_b: bool = True) -> tuple[Csr, Optional[Csr]]:
    """Diagonally dominant sparse non-Hermitian pencil (the situation of
    Section 1 where the diagonal makes an effective preconditioner).

    A = D + E: D(i,i) uniform in [0, n) plus 0.1 i N(0,1); E has
    ``offdiag_per_row`` uniformly drawn off-diagonal columns per row (drawn
    with replacement, duplicates summed) with values coupling * CN(0,1).
    B = diag U[1,2] from ``default_rng(0)`` (or None).
    """
    rng = np.random.default_rng(seed)
    q = offdiag_per_row
    d = rng.uniform(0.0, float(n), n) + 0.1j * rng.standard_normal(n)
    rows = np.repeat(np.arange(n), q)
    cols = rng.integers(0, n - 1, n * q)
    cols[cols >= rows] += 1
    vals = coupling * (rng.standard_normal(n * q) + 1j * rng.standard_normal(n * q)) / np.sqrt(2)
    A = sp.coo_matrix((np.concatenate([vals, d]),
                       (np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]))),
                      shape=(n, n))
    B = diag_csr(diagonal_b(n, 0)) if with_b else None
    return csr_from_scipy(A), B


def start_block(n: int, b: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n, b))
    im = rng.standard_normal((n, b))
    return np.ascontiguousarray((re + 1j * im) / np.sqrt(2.0))


@dataclass
class Problem:
    """One synthetic workload.  ``B is None`` means the standard problem."""
    name: str
    A: Csr
    B: Optional[Csr]
    sigma: complex
    k: int
    block: int
    precond: str            # "diag", "jacobi" or "gmres"
    sweeps: int = 0
    omega: float = 0.0
    precision: str = "fp64"  # "fp64" or "mixed"
    tol: float = 1e-10
    V0: np.ndarray = field(default=None, repr=False)
    steps: int = 0           # "gmres": block steps
    inner: str = "jacobi"    # "gmres": inner right preconditioner

    @property
    def n(self) -> int:
        return self.A.n


def _with_v0(p: Problem) -> Problem:
    p.V0 = start_block(p.n, p.block, seed=1)
    return p


def config(name: str, scale: Optional[int] = None) -> Problem:
    """The five workloads, by name.

    c1  2-D upwind, N=32 (n=1024), c=(10,10), B=I, sigma=200, k=b=4, T=diag(C)^-1
    c2  3-D upwind, N=64 (n=262144), c=(20,10,5), B=diag U[1,2], sigma=500+50i,
        k=b=10, 3 weighted-Jacobi sweeps (omega=0.7) on C, complex128
    c3  c2 in mixed precision
    c4  random pencil n=131072, sigma=0, k=b=8, T=diag(C)^-1
    c5  3-D upwind, N=160 (n=4096000), c=(20,10,5), B=diag U[1,2],
        sigma=1000+100i, k=b=16, Jacobi-3, mixed precision
    d1  diagonally dominant pencil (see diag_dominant_pencil), n=262144,
        B=diag U[1,2], sigma=n/2+0.3i, k=b=10, T=diag(C)^-1, complex128
    d1m d1 in mixed precision
    d2  diagonally dominant pencil with coupling 4 (diagonal T alone converges
        slowly), n=262144, B=diag U[1,2], sigma=n/2+0.3i, k=b=10, T = 2 block
        GMRES steps right-preconditioned by 3 Jacobi sweeps (omega=0.7), complex128
    d2m d2 in mixed precision
    c1g c1 with the stronger preconditioner of Section 4 -- T = 8 block GMRES
        steps right-preconditioned by 3 Jacobi sweeps (omega=0.7) -- and a
        block of 8 columns for the k=4 wanted pairs (diag(C) is constant on
        c1, so its diagonal preconditioner is a scalar)

    ``scale`` overrides the grid size N (stencils) or n (random pencil) to give
    a smaller instance of the same family.
    """
    if name == "c1":
        N = scale or 32
        return _with_v0(Problem("c1", convection_diffusion(N, (10.0, 10.0)), None, 200.0 + 0j,
                                4, 4, "diag"))
    if name == "c1g":
        N = scale or 32
        return _with_v0(Problem("c1g", convection_diffusion(N, (10.0, 10.0)), None, 200.0 + 0j,
                                4, 8, "gmres", 3, 0.7, steps=8, inner="jacobi"))
    if name in ("c2", "c3"):
        N = scale or 64
        A = convection_diffusion(N, (20.0, 10.0, 5.0))
        B = diag_csr(diagonal_b(A.n, 0))
        return _with_v0(Problem(name, A, B, 500.0 + 50.0j, 10, 10, "jacobi", 3, 0.7,
                                "fp64" if name == "c2" else "mixed"))
    if name == "c4":
        n = scale or 131072
        A, B = random_pencil(n, 0)
        return _with_v0(Problem("c4", A, B, 0j, 8, 8, "diag"))
    if name == "c5":
        N = scale or 160
        A = convection_diffusion(N, (20.0, 10.0, 5.0))
        B = diag_csr(diagonal_b(A.n, 0))
        return _with_v0(Problem("c5", A, B, 1000.0 + 100.0j, 16, 16, "jacobi", 3, 0.7, "mixed"))
    if name in ("d1", "d1m"):
        n = scale or 262144
        A, B = diag_dominant_pencil(n, 0)
        return _with_v0(Problem(name, A, B, n / 2 + 0.3j, 10, 10, "diag",
                                precision="fp64" if name == "d1" else "mixed"))
    if name in ("d2", "d2m"):
        n = scale or 262144
        A, B = diag_dominant_pencil(n, 0, coupling=4.0)
        return _with_v0(Problem(name, A, B, n / 2 + 0.3j, 10, 10, "gmres", 3, 0.7,
                                precision="fp64" if name == "d2" else "mixed",
                                steps=2, inner="jacobi"))
    raise ValueError(f"unknown workload {name!r}")
