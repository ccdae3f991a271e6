"""Convergence study of the named stencil and random-pencil workloads with the
CPU oracle -- TEST INFRASTRUCTURE ONLY (calls nothing but oracle/ and the
input generators).

Question: can Algorithm 2 reach a 1e-10 relative eigen-residual on the
workloads as specified (k wanted pairs, block b = k, the configured T), and
which of the levers the paper offers changes that: a wider block (b > k),
a deeper Krylov-Arnoldi sequence (larger m, Section 5's remedy for a weak T),
or a stronger T (block GMRES, Section 4)?  An exact shift-and-invert T
separates the method from its preconditioner.

Every case runs Algorithm 2 from the seeded start block for a fixed
iteration budget and reports the iterations to 1e-10 (or that it did not
converge), the smallest and the last residual.  For each pencil the script
also reports the distances of the eigenvalues nearest sigma from dense LAPACK
(zggev) and the ratio d_k / d_{k+1}.

Usage:
    python -m oracle.convergence_study c2 12 [maxit]    # 3-D stencil pencil, N = 12
    python -m oracle.convergence_study c1               # 2-D stencil, N = 32
    python -m oracle.convergence_study c4 2048          # random pencil, n = 2048
Cases run in parallel worker processes, one BLAS thread each; STUDY_ONLY
(a substring of the case labels) restricts the run to matching cases.
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

# one BLAS thread per worker process (set before numpy's BLAS starts)
os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np                            # noqa: E402
import scipy.linalg as sla                    # noqa: E402
import scipy.sparse as sp                     # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import gplhr_oracle as O          # noqa: E402
from paper_1506_06829_amd import problems     # noqa: E402

# (label, T kind, block, m, extra); T kinds: "config" (the workload's own),
# "exact", "jacobi", "gmres<s>" (s block GMRES steps over 3 Jacobi sweeps),
# "exact-real" (exact T and extraction at the real part of sigma)
CASES = {
    "c2": [("configured: Jacobi-3, b = k", "config", 10, 1),
           ("Jacobi-3, b = k, m = 4", "config", 10, 4),
           ("Jacobi-3, b = k + 6", "config", 16, 1),
           ("GMRES(4) over Jacobi-3, b = k", "gmres4", 10, 1),
           ("GMRES(4) over Jacobi-3, b = k + 6", "gmres4", 16, 1),
           ("exact T, b = k", "exact", 10, 1),
           ("exact T, b = k, m = 4", "exact", 10, 4),
           ("exact T, b = k + 2", "exact", 12, 1),
           ("exact T, b = k + 4", "exact", 14, 1),
           ("exact T, b = k + 6", "exact", 16, 1),
           ("exact T, b = k + 6, m = 4", "exact", 16, 4),
           ("Jacobi-3, b = k + 6, m = 4", "config", 16, 4),
           ("GMRES(4) over Jacobi-3, b = k + 6, m = 4", "gmres4", 16, 4),
           ("exact T, real shift Re(sigma), b = k", "exact-real", 10, 1)],
    "c1": [("configured: diag(C)^-1 (a scalar here), b = k", "config", 4, 1),
           ("diag(C)^-1, b = 2k", "config", 8, 1),
           ("GMRES(16) over diag, b = k", "gmres16d", 4, 1),
           ("GMRES(16) over Jacobi-3, b = k", "gmres16", 4, 1),
           ("GMRES(8) over Jacobi-3, b = 2k", "gmres8", 8, 1),
           ("exact T, b = k", "exact", 4, 1)],
    "c4": [("configured: diag(C)^-1, b = k", "config", 8, 1),
           ("diag(C)^-1, b = k, m = 4", "config", 8, 4),
           ("diag(C)^-1, b = k + 4", "config", 12, 1),
           ("GMRES(4) over diag, b = k", "gmres4d", 8, 1),
           ("GMRES(8) over diag, b = k", "gmres8d", 8, 1),
           ("GMRES(4) over diag, b = k + 2", "gmres4d", 10, 1),
           ("GMRES(6) over diag, b = k + 2", "gmres6d", 10, 1),
           ("exact T, b = k", "exact", 8, 1)],
}


def _pencil(name: str, scale):
    p = problems.config(name, scale)
    A = p.A.to_scipy()
    B = None if p.B is None else p.B.to_scipy()
    return p, A, B


def _run(args):
    name, scale, label, kind, b, m, maxit = args
    p, A, B = _pencil(name, scale)
    n = A.shape[0]
    Bm = sp.identity(n, format="csr") if B is None else B
    sigma = p.sigma
    if kind == "exact-real":
        sigma = complex(sigma.real, 0.0)
    C = (A - sigma * Bm).tocsr()
    if kind == "config":
        T = O.make_preconditioner(C, p.precond, p.sweeps, p.omega, p.steps, p.inner)
    elif kind in ("exact", "exact-real"):
        T = O.make_preconditioner(C, "exact")
    elif kind.startswith("gmres"):
        spec = kind[5:]
        inner = "diag" if spec.endswith("d") else "jacobi"
        T = O.make_preconditioner(C, "gmres", 3, 0.7, steps=int(spec.rstrip("d")), inner=inner)
    else:
        raise ValueError(kind)
    t0 = time.perf_counter()
    r = O.gplhr(A, B, sigma, p.k, problems.start_block(n, b), T, m=m, tol=1e-10, maxit=maxit)
    h = np.asarray(r.history)
    return dict(label=label, converged=r.converged, iterations=r.iterations,
                min_rho=float(h.min()), last_rho=float(h[-1]),
                rho_10=float(h[min(10, len(h) - 1)]), seconds=time.perf_counter() - t0,
                lam=np.sort_complex(r.lam[:p.k]))


def spectrum_summary(name: str, scale) -> str:
    p, A, B = _pencil(name, scale)
    Bd = np.eye(A.shape[0]) if B is None else B.toarray()
    ev = sla.eigvals(A.toarray(), Bd)
    d = np.sort(np.abs(ev - p.sigma))
    k = p.k
    return (f"{name} n={A.shape[0]} sigma={p.sigma} k={k}: distances of the nearest "
            f"eigenvalues {np.array2string(d[:k + 7], precision=4, max_line_width=200)}; "
            f"d_k/d_(k+1) = {d[k - 1] / d[k]:.5f}, d_k/d_(k+7) = {d[k - 1] / d[k + 6]:.5f}")


def main(argv):
    name = argv[1] if len(argv) > 1 else "c2"
    scale = int(argv[2]) if len(argv) > 2 and argv[2] != "-" else {"c2": 12, "c4": 2048}.get(name)
    maxit = int(argv[3]) if len(argv) > 3 else 300
    workers = int(os.environ.get("STUDY_WORKERS", "6"))
    print(spectrum_summary(name, scale), flush=True)
    only = os.environ.get("STUDY_ONLY")
    jobs = [(name, scale, lab, kind, b, m, maxit) for lab, kind, b, m in CASES[name]
            if not only or only in lab]
    print(f"| case | converged to 1e-10 | iterations | min residual | last residual |")
    print(f"|---|---|---|---|---|")
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for res in ex.map(_run, jobs):
            it = str(res["iterations"]) if res["converged"] else f"no ({res['iterations']})"
            print(f"| {res['label']} | {'yes' if res['converged'] else 'no'} | {it} | "
                  f"{res['min_rho']:.1e} | {res['last_rho']:.1e} |", flush=True)


if __name__ == "__main__":
    main(sys.argv)
