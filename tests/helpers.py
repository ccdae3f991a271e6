"""Shared helpers of the test-suite (no solver arithmetic)."""
import numpy as np
from scipy.optimize import linear_sum_assignment


def match_err(a, b):
    """Max relative distance between two eigenvalue multisets after optimal
    pairing (eigenvalues are never compared by index)."""
    a, b = np.asarray(a), np.asarray(b)
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return float(np.max(C[r, c] / np.abs(b[c])))


def nearest(vals, sigma, k):
    vals = np.asarray(vals)
    return vals[np.argsort(np.abs(vals - sigma), kind="stable")[:k]]


def gpu_solver(p, precision=None, V0=True, **kw):
    """Solver handle for a problems.Problem (inputs only)."""
    import torch
    from paper_1506_06829_amd import gplhr as G
    A = G.DeviceCsr.from_host(p.A)
    B = None if p.B is None else G.DeviceCsr.from_host(p.B)
    v0 = torch.as_tensor(p.V0).to("cuda") if V0 else None
    opts = dict(precond=p.precond, sweeps=p.sweeps or 3, omega=p.omega or 0.7,
                precision=precision or p.precision, V0=v0)
    if p.precond == "gmres":
        opts.update(steps=p.steps, inner=p.inner)
    opts.update(kw)
    return G.Solver(A, B, p.sigma, p.k, p.block, **opts), A, B


def gpu_trajectory(p, its, precision=None, **kw):
    """Rayleigh-Ritz eigenvalues after 0..its iterations on the GPU."""
    s, _, _ = gpu_solver(p, precision=precision, tol=0.0, **kw)
    lams = [s.lam()]
    for _ in range(its):
        s.iterate(1)
        lams.append(s.lam())
    s.close()
    return lams
