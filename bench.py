"""Benchmark of the GPLHR hot path on one MI355X: time per iteration and time
to k eigenpairs at a 1e-10 relative residual (mixed vs FP64), and SpMM HBM
bandwidth.  Prints ONE JSON line.

Headline workload: the 160^3 pencil (n = 4096000, 3-D upwind convection-
diffusion, B = diag U[1,2], sigma = 1000 + 100i, k = b = 16, three damped
Jacobi sweeps), the largest configuration that fits one GPU.  It does not
reach 1e-10 with any preconditioner and block width the GPU path supports
(the wanted eigenvalues lie at nearly equal distance from sigma; the oracle
convergence study shows the same on scaled instances), so one step is one
complete GPLHR iteration -- every part of the hot path once: sparse products,
preconditioner, projections, Cholesky-QR of the trial and test bases, the
projected pencil, the host Schur step, the basis update and the convergence
check -- timed in the complex64 phase (mixed) and in FP64.  `value` is the
mixed time per iteration; the residual history over a longer run is reported
as iterations-to-stagnation.  Inputs are resident in HBM before the timed
region.

Time to solution (complete create -> iterate to 1e-10 -> output -> destroy)
is reported on the workloads that converge: the 32x32 stencil with the
stronger preconditioner of Section 4 (c1 with block GMRES over Jacobi, block
8), and the diagonally dominant pencils at n = 262144 and 4096000.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The kernel behind the largest share of a 160^3 mixed iteration: the
# LDS-staged Gram of the projected pencil, complex64 64 x 64 over 4096000 rows
# on the FP64 MFMA, timed on its own at the solver's shape.
DOMINANT_KERNEL_PROBE = "Gram c64 64x64"
# HBM-side bytes per launch of that probe from rocprofv3 (FETCH_SIZE scaled
# by 2.000 and WRITE_SIZE by 1.000, the factors being what the same counters
# read for a 256 MiB device copy), valid only for the kernels.hip whose
# SHA-256 prefix is recorded with it; any later change to that file makes the
# reported traffic null until the counters are taken again.
DOMINANT_KERNEL_TRAFFIC = 4261221332          # bytes per launch
DOMINANT_KERNEL_TRAFFIC_SRC = "32cf1a236323714d"   # sha256 prefix of kernels.hip


def kernels_source_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_1506_06829_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


METRIC = "time to k eigenpairs @1e-10 rel. residual, mixed vs FP64; SpMM HBM GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve_once(G, A, B, p, precision, V0, timing):
    s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, sweeps=p.sweeps or 3,
                 omega=p.omega or 0.7, precision=precision, V0=V0, tol=1e-10, max_iter=400,
                 timing=timing)
    st, nconv, res = s.iterate()
    out = s.schur(want_vectors=False)
    stats = s.stats()
    s.close()
    return st, res, out, stats


def time_solves(G, torch, A, B, p, precision, V0, steps, warmup, timing):
    for _ in range(warmup):
        solve_once(G, A, B, p, precision, V0, timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(steps):
        runs.append(solve_once(G, A, B, p, precision, V0, timing))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, runs


def spmm_hbm(G, torch, csr, b, dtype, reps=20, plane=None):
    """Event-timed CSR SpMM (library kernel) on torch's current stream, in the
    row schedule the solver uses for this pattern (plane=None) or a given one."""
    A = G.DeviceCsr.from_host(csr)
    if plane is None:
        plane = G.csr_plane(A)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    val = A.val.to(tdt)
    X = torch.randn(csr.n, b, dtype=tdt, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(3):
        G.spmm(A, X, Y, val=val, plane=plane)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        G.spmm(A, X, Y, val=val, plane=plane)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    e = 8 if dtype == "c64" else 16
    nbytes = csr.nnz * (e + 4) + 4 * (csr.n + 1) + 2 * csr.n * b * e
    del A, val, X, Y
    torch.cuda.empty_cache()
    return dict(ms=ms, bytes=nbytes, gbs=nbytes / ms / 1e6, plane=plane)


def stream_copy_gbs(G, torch, reps=20):
    """Bandwidth of the library's streaming block-copy kernel (each byte read
    once and written once), event-timed on torch's current stream: a 16-wide
    complex64 block of 4096000 rows (the 160^3 block, 524 MB each way) and a
    2 GiB block.  What a kernel that reads and writes HBM attains here."""
    out = {}
    for name, n, w in (("c64_4096000x16", 4096000, 16), ("c64_2GiB", 2**27, 2)):
        X = torch.randn(n, w, dtype=torch.complex64, device="cuda")
        Y = torch.empty_like(X)
        for _ in range(3):
            G.block_copy(X, Y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            G.block_copy(X, Y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        assert torch.equal(X, Y)
        nbytes = 2 * X.numel() * 8
        out[name] = dict(ms=ms, bytes=nbytes, gbs=nbytes / ms / 1e6, frac=nbytes / ms / 1e6 / HBM_PEAK_GBS)
        del X, Y
    torch.cuda.empty_cache()
    return out


FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector (MFMA FP32 rate of the complex64 updates)


def kernel_rooflines(G, torch):
    """Event-timed block updates and Grams at the 160^3 and d1 sizes, each
    against the roofline that bounds it: bytes / 8 TB/s for the HBM-bound
    shapes, flops / the FP64 (or FP32) peak for the wide ones, whichever
    takes longer at peak."""
    def timed(fn, reps=10):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    # the C ABI is called with its arguments marshalled once, so the loop
    # times the kernels rather than the binding's per-call Python work
    L = G.lib()
    sp = G._stream_ptr()

    def checked(call):
        # the status of the first (warm-up) call is checked
        first = [True]

        def f():
            st = call()
            if first[0]:
                first[0] = False
                if st != 0:
                    raise RuntimeError(f"probe call failed with status {st}")
        return f

    out = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for n, dt, wx, wy, beta in ((4096000, "c64", 16, 16, 1.0), (4096000, "c128", 16, 16, 1.0),
                                (4096000, "c128", 64, 32, 0.0), (4096000, "c64", 64, 32, 0.0),
                                (262144, "c128", 10, 10, 1.0)):
        tdt = torch.complex128 if dt == "c128" else torch.complex64
        e = 16 if dt == "c128" else 8
        X = torch.randn(n, wx, dtype=tdt, device="cuda", generator=gen)
        Y = torch.randn(n, wy, dtype=tdt, device="cuda", generator=gen)
        # wx-by-wy coefficients, column-major
        Mc = torch.randn(wy, wx, dtype=torch.complex128, device="cuda", generator=gen)
        args = (0 if dt == "c128" else 1, n, G._ptr(X), X.stride(0), wx, G._ptr(Mc), wx, G._ptr(Y),
                Y.stride(0), wy, float(beta), 0.0, sp)
        ms = timed(checked(lambda: L.gplhr_block_update(*args)))
        nbytes = n * (wx + wy * (2 if beta else 1)) * e
        flops = 8.0 * n * wx * wy
        peak_tf = FP64_PEAK_TFLOPS if dt == "c128" else FP32_PEAK_TFLOPS
        t_mem, t_fl = nbytes / (HBM_PEAK_GBS * 1e6), flops / (peak_tf * 1e9)
        if t_mem >= t_fl:
            rf = {"bound": "hbm", "achieved": nbytes / ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            rf = {"bound": "mfma", "achieved": flops / ms / 1e9, "peak": peak_tf, "unit": "TFLOP/s"}
        rf["frac"] = rf["achieved"] / rf["peak"]
        name = f"block update {dt} {wx}->{wy}" + (" (beta=1)" if beta else "")
        if name.startswith(DOMINANT_KERNEL_PROBE) and DOMINANT_KERNEL_TRAFFIC_SRC == kernels_source_sha():
            rf["traffic"] = DOMINANT_KERNEL_TRAFFIC
        out.append(dict(kernel=name, n=n, ms=ms, bytes=nbytes, flops=flops, **rf))
        del X, Y, Mc
    # (a 10 x 10 Gram at 262144 rows runs shorter than one call's host work,
    # so a loop of calls would time the host; its kernel time is in the
    # rocprofv3 summary of the d1 solve)
    for n, dt, bx, by in ((4096000, "c64", 64, 64), (4096000, "c128", 64, 64),
                          (4096000, "c128", 16, 16), (262144, "c128", 40, 40)):
        tdt = torch.complex128 if dt == "c128" else torch.complex64
        X = torch.randn(n, bx, dtype=tdt, device="cuda", generator=gen)
        Y = torch.randn(n, by, dtype=tdt, device="cuda", generator=gen)
        Gout = torch.empty((by, bx), dtype=torch.complex128, device="cuda")
        args = (0 if dt == "c128" else 1, n, G._ptr(X), X.stride(0), bx, G._ptr(Y), Y.stride(0), by,
                G._ptr(Gout), sp)
        ms = timed(checked(lambda: L.gplhr_gram(*args)))
        nbytes = n * (bx + by) * (16 if dt == "c128" else 8)
        flops = 8.0 * n * bx * by
        t_mem, t_fl = nbytes / (HBM_PEAK_GBS * 1e6), flops / (FP64_PEAK_TFLOPS * 1e9)
        if t_mem >= t_fl:
            rf = {"bound": "hbm", "achieved": nbytes / ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            rf = {"bound": "mfma", "achieved": flops / ms / 1e9, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
        rf["frac"] = rf["achieved"] / rf["peak"]
        name = f"Gram {dt} {bx}x{by} (FP64 MFMA, incl. the partial reduction)"
        if name.startswith(DOMINANT_KERNEL_PROBE) and DOMINANT_KERNEL_TRAFFIC_SRC == kernels_source_sha():
            rf["traffic"] = DOMINANT_KERNEL_TRAFFIC
        out.append(dict(kernel=name, n=n, ms=ms, bytes=nbytes, flops=flops, **rf))
        del X, Y, Gout
    torch.cuda.empty_cache()
    return out


def named_iteration_times(G, torch, name, scale, its, precisions):
    from paper_1506_06829_amd import problems
    p = problems.config(name, scale)
    A = G.DeviceCsr.from_host(p.A)
    B = None if p.B is None else G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(p.V0).to("cuda")
    out = dict(n=p.n, nnz=p.A.nnz, k=p.k, sigma=str(p.sigma), precond=f"{p.precond}{p.sweeps or ''}")
    for prec in precisions:
        s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, sweeps=p.sweeps or 3,
                     omega=p.omega or 0.7, precision=prec, V0=V0, tol=1e-10,
                     switch_tol=0.0, stall_window=10**6)
        s.iterate(2)                      # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _, res = s.iterate(its)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / its
        out[prec] = dict(ms_per_iteration=dt * 1e3, max_rel_resid_after=res,
                         iterations=s.stats()["iterations"], converged=(st == 0))
        s.close()
        log(f"[bench] {name}{'' if scale is None else scale} {prec}: {dt*1e3:.2f} ms/iteration, residual {res:.2e}")
    del A, B, V0
    torch.cuda.empty_cache()
    return out


def timed_solve(G, torch, p, precision, reps=2, **kw):
    """Complete solves (create + iterate to 1e-10 + output) of a workload with
    the given options: one untimed warm-up, then `reps` timed."""
    A = G.DeviceCsr.from_host(p.A)
    B = None if p.B is None else G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(p.V0).to("cuda")
    opts = dict(precond=p.precond, sweeps=p.sweeps or 3, omega=p.omega or 0.7, precision=precision,
                V0=V0, tol=1e-10, max_iter=kw.pop("max_iter", 200))
    if p.precond == "gmres":
        opts.update(steps=p.steps, inner=p.inner)
    opts.update(kw)

    def once():
        s = G.Solver(A, B, p.sigma, p.k, p.block, **opts)
        st, _, res = s.iterate()
        lam = s.lam()
        stats = s.stats()
        s.close()
        return st, res, lam, stats

    try:
        once()
    except G.GplhrError as e:
        # a variant that breaks down (e.g. the LOBPCG-style P of Table 2)
        del A, B, V0
        return dict(converged=False, error=str(e)), None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st, res, lam, stats = once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del A, B, V0
    return dict(s_per_solve=dt, iterations=stats["iterations"],
                fp64_iterations=stats["fp64_iterations"], converged=(st == 0),
                max_rel_resid=res), lam


def deflation_5_plus_5(G, torch, p, reps=2):
    """5 pairs, then 5 more on the deflated pair (two complete solves)."""
    import numpy as np
    A = G.DeviceCsr.from_host(p.A)
    B = G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(np.ascontiguousarray(p.V0[:, :5])).to("cuda")
    opts = dict(precond=p.precond, V0=V0, tol=1e-10, max_iter=200)

    def once():
        s1 = G.Solver(A, B, p.sigma, 5, 5, **opts)
        st1, _, _ = s1.iterate()
        o1 = s1.schur()
        s1.close()
        s2 = G.Solver(A, B, p.sigma, 5, 5, deflate=(o1["V"], o1["Q"]), **opts)
        st2, _, res = s2.iterate()
        lam2 = s2.lam()
        its = s2.stats()["iterations"]
        s2.close()
        return st1 == 0 and st2 == 0, res, np.concatenate([o1["lam"], lam2]), its

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ok, res, lam, its2 = once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del A, B, V0
    return dict(s_per_solve=dt, converged=ok, max_rel_resid=res, second_run_iterations=its2), lam


def eig_diff(a, b):
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    C = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    ri, ci = linear_sum_assignment(C)
    return float(np.max(C[ri, ci] / np.abs(np.asarray(b)[ci])))


def next_rows(G, torch, problems, lam_ref):
    """The extensions of the method on the n = 262144 pencils, each a complete
    solve to 1e-10; eigenvalues compared with the FP64 Schur-form solve."""
    out = {}
    d1 = problems.config("d1")
    for key, prec, kw in [("locking", "fp64", dict(locking=True)),
                          ("locking", "mixed", dict(locking=True)),
                          ("eig_form", "fp64", dict(algorithm="eig")),
                          ("eig_form", "mixed", dict(algorithm="eig")),
                          ("p_lobpcg", "fp64", dict(p_mode="lobpcg", max_iter=60)),
                          ("p_none", "fp64", dict(p_mode="none", max_iter=60)),
                          ("eig_form_p_lobpcg", "fp64", dict(algorithm="eig", p_mode="lobpcg", max_iter=60))]:
        r, lam = timed_solve(G, torch, d1, prec, **kw)
        r["eig_rel_diff_vs_fp64_schur"] = eig_diff(lam, lam_ref) if r["converged"] else None
        out.setdefault(key, {})[prec] = r
        log(f"[bench] d1 {key} {prec}: {r}")
    r, lam = deflation_5_plus_5(G, torch, d1)
    r["eig_rel_diff_vs_fp64_schur"] = eig_diff(lam, lam_ref) if r["converged"] else None
    out["deflation_5_plus_5"] = {"fp64": r}
    log(f"[bench] d1 deflation 5+5: {r['s_per_solve']*1e3:.1f} ms, converged {r['converged']}")
    d2 = problems.config("d2")
    out["gmres_T_d2"] = {"workload": "diagonally dominant pencil with coupling 4, n=262144, k=b=10, "
                                     "T = 2 block GMRES steps over 3 Jacobi sweeps"}
    for prec in ("fp64", "mixed"):
        r, _ = timed_solve(G, torch, d2, prec)
        out["gmres_T_d2"][prec] = r
        log(f"[bench] d2 GMRES T {prec}: {r['s_per_solve']*1e3:.1f} ms, {r['iterations']} its")
    d2.precond = "jacobi"
    r, _ = timed_solve(G, torch, d2, "fp64")
    out["gmres_T_d2"]["jacobi3_only_fp64"] = r
    log(f"[bench] d2 Jacobi-3 T fp64: {r['s_per_solve']*1e3:.1f} ms, {r['iterations']} its")
    return out


def large_time_to_solution(G, torch, problems, n=4096000):
    """The same diagonally dominant family at the 160^3 size: complete solves
    to 1e-10, mixed vs FP64 (one warm-up and one timed solve each)."""
    p = problems.config("d1m", n)
    out = {"workload": f"diagonally dominant generalized pencil n={p.n}, nnz={p.A.nnz}, "
                       f"B=diag U[1,2], sigma=n/2+0.3i, k=b=10, T=diag(A-sigma B)^-1"}
    lams = {}
    for prec in ("mixed", "fp64"):
        r, lam = timed_solve(G, torch, p, prec, reps=1)
        out[prec] = r
        lams[prec] = lam
        log(f"[bench] d1 n={p.n} {prec}: {r.get('s_per_solve', float('nan'))*1e3:.1f} ms, "
            f"{r.get('iterations')} its, converged {r['converged']}")
    if out["mixed"]["converged"] and out["fp64"]["converged"]:
        out["speedup_mixed_vs_fp64"] = out["fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
        out["eig_rel_diff_mixed_vs_fp64"] = eig_diff(lams["mixed"], lams["fp64"])
    return out


def slow_time_to_solution(G, torch, problems, n=4096000):
    """A slowly converging member of the family (coupling 4, diagonal T: about
    25 iterations): complete solves to 1e-10, FP64 vs mixed (default switch,
    and an early switch at 1e-5 with a 20-iteration stall window)."""
    p = problems.config("d2", n)
    p.precond, p.sweeps, p.steps, p.inner = "diag", None, None, None
    out = {"workload": f"diagonally dominant generalized pencil with coupling 4, n={p.n}, nnz={p.A.nnz}, "
                       f"B=diag U[1,2], sigma=n/2+0.3i, k=b=10, T=diag(A-sigma B)^-1"}
    for key, prec, kw in (("fp64", "fp64", {}), ("mixed", "mixed", {}),
                          ("mixed_switch_1e-5", "mixed", {"switch_tol": 1e-5, "stall_window": 20})):
        r, _ = timed_solve(G, torch, p, prec, reps=1, max_iter=300, **kw)
        out[key] = r
        log(f"[bench] d2/diag n={p.n} {key}: {r.get('s_per_solve', float('nan'))*1e3:.1f} ms, "
            f"{r.get('iterations')} its ({r.get('fp64_iterations')} FP64), converged {r['converged']}")
    if all(out[k]["converged"] for k in ("fp64", "mixed", "mixed_switch_1e-5")):
        out["speedup_mixed_vs_fp64"] = out["fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
        out["speedup_mixed_switch_1e-5_vs_fp64"] = out["fp64"]["s_per_solve"] / out["mixed_switch_1e-5"]["s_per_solve"]
    return out


def host_cpu_info():
    """Host CPU model, logical CPUs and the BLAS threads numpy uses."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [dict(api=i.get("internal_api"), threads=i.get("num_threads")) for i in threadpool_info()]
    except Exception:
        pass
    return dict(model=model, logical_cpus=os.cpu_count(), blas=blas)


def c5_iterations(G, torch, p, A, B, V0, steps, warmup, hist_its):
    """Per-iteration time of the 160^3 pencil in the complex64 phase (mixed)
    and in FP64 (`steps` timed iterations after `warmup`), then the residual
    after every further iteration up to `hist_its` in total."""
    out = {}
    for prec in ("mixed", "fp64"):
        s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, sweeps=p.sweeps,
                     omega=p.omega, precision=prec, V0=V0, tol=1e-10,
                     switch_tol=0.0, stall_window=10**6)
        hist = [s.stats()["max_rel_resid"]]
        if warmup:
            s.iterate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _, res = s.iterate(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        done = warmup + steps
        hist.extend([None] * (done - 1) + [res])
        while done < hist_its:
            st, _, res = s.iterate(1)
            done += 1
            hist.append(res)
        lam = s.lam()
        resid_x = s.residual_norms()
        stats = s.stats()
        s.close()
        valid = [(i, h) for i, h in enumerate(hist) if h is not None]
        best_i, best = min(valid, key=lambda t: t[1])
        out[prec] = dict(s_per_iteration=dt, timed_iterations=steps, warmup_iterations=warmup,
                         iterations_run=stats["iterations"], converged=(st == 0),
                         min_rel_resid=best, min_at_iteration=best_i, last_rel_resid=res,
                         rel_resid_at={str(i): h for i, h in valid if i in (0, 10, 20, 30, 40, 60, 80)},
                         max_resid_over_norm_x=float(max(resid_x)), lam=lam)
        log(f"[bench] c5 {prec}: {dt*1e3:.2f} ms/iteration; residual {hist[0]:.2e} -> min {best:.2e} "
            f"at iteration {best_i}, last {res:.2e} after {stats['iterations']}")
    return out


def cpu_baseline_c5(p, gpu_lam):
    """The FP64 oracle on the same 160^3 workload, on the host: set-up (steps
    1-4 of Algorithm 2 and the first convergence check) and one iteration,
    timed separately; the per-eigenvalue difference of the GPU's Rayleigh-Ritz
    values after one iteration (both precisions) from the oracle's."""
    from oracle import gplhr_oracle as O
    t0 = time.perf_counter()
    r0 = O.solve_problem(p, tol=0.0, maxit=0)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    r1 = O.solve_problem(p, tol=0.0, maxit=1)
    t_one = time.perf_counter() - t0 - t_setup
    errs = {}
    for prec, lam in gpu_lam.items():
        errs[prec] = per_eig_err(lam, r1.lam_history[1][:p.k])
    return t_setup, t_one, r0, r1, errs


def per_eig_err(lam, ref):
    """Relative difference of each eigenvalue from its optimally paired reference."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    C = np.abs(np.asarray(lam)[:, None] - np.asarray(ref)[None, :])
    ri, ci = linear_sum_assignment(C)
    return [float(x) for x in C[ri, ci] / np.abs(np.asarray(ref)[ci])]


def c1g_time_to_solution(G, torch, problems):
    """c1 with block GMRES(8) over Jacobi-3 as T and an 8-column block:
    complete solves to 1e-10, mixed vs FP64; eigenvalues against the closed
    form of the 2-D upwind operator."""
    import numpy as np
    p = problems.config("c1g")
    N, c = 32, 10.0
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)
    mu = (2 + c * h) / h**2 - (2 / h**2) * np.sqrt(1 + c * h) * np.cos(j * np.pi * h)
    lam_cf = (mu[:, None] + mu[None, :]).ravel()
    lam_cf = lam_cf[np.argsort(np.abs(lam_cf - 200.0), kind="stable")[:4]]
    out = {"workload": "c1: 2-D upwind stencil N=32 (n=1024), B=I, sigma=200, k=4; block 8, "
                       "T = 8 block GMRES steps over 3 Jacobi sweeps (omega 0.7) (Section 4)"}
    lams = {}
    for prec in ("mixed", "fp64"):
        r, lam = timed_solve(G, torch, p, prec, reps=3, max_iter=1500)
        out[prec] = r
        lams[prec] = lam
        if r["converged"]:
            r["eig_rel_err_vs_closed_form"] = per_eig_err(lam[:4], lam_cf)
        log(f"[bench] c1g {prec}: {r.get('s_per_solve', float('nan'))*1e3:.1f} ms, "
            f"{r.get('iterations')} its, converged {r['converged']}")
    if out["mixed"]["converged"] and out["fp64"]["converged"]:
        out["speedup_mixed_vs_fp64"] = out["fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
    return out


def d1_time_to_solution(G, torch, problems, steps, warmup):
    """The diagonally dominant pencil at n = 262144 (diag T): complete solves
    to 1e-10, mixed vs FP64, with the orthogonality of the output bases."""
    import numpy as np
    p = problems.config("d1m")
    A = G.DeviceCsr.from_host(p.A)
    B = G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(p.V0).to("cuda")
    res = {"workload": f"diagonally dominant generalized pencil n={p.n}, 17 nnz/row, "
                       f"B=diag U[1,2], sigma=n/2+0.3i, k=b=10, T=diag(A-sigma B)^-1"}
    outs = {}
    for prec in ("mixed", "fp64"):
        dt, runs = time_solves(G, torch, A, B, p, prec, V0, steps, warmup, False)
        st, r, out, stats = runs[-1]
        outs[prec] = out
        res[prec] = dict(s_per_solve=dt, converged=(st == 0), max_rel_resid=r,
                         iterations=stats["iterations"], fp64_iterations=stats["fp64_iterations"])
        log(f"[bench] d1 {prec}: {dt*1e3:.2f} ms/solve, {stats['iterations']} its")
    res["speedup_mixed_vs_fp64"] = res["fp64"]["s_per_solve"] / res["mixed"]["s_per_solve"]
    res["eig_rel_diff_mixed_vs_fp64"] = max(per_eig_err(outs["mixed"]["lam"], outs["fp64"]["lam"]))

    def orth_loss(precision):
        s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, precision=precision, V0=V0,
                     tol=1e-10, max_iter=400)
        s.iterate()
        o = s.schur()
        s.close()
        eye = torch.eye(p.k, dtype=torch.complex128, device="cuda")
        V, Q = o["V"], o["Q"]
        return {"V": float((V.conj().T @ V - eye).abs().max()), "Q": float((Q.conj().T @ Q - eye).abs().max())}
    res["orthogonality_loss"] = {"mixed": orth_loss("mixed"), "fp64": orth_loss("fp64")}
    del A, B, V0
    torch.cuda.empty_cache()
    return res, outs["fp64"]["lam"]


def c4_gradient(G, torch, problems, reps=2):
    """The gradient workload's generator at n = 2048 (sigma = 0, k = 8; block
    10, T = 6 block GMRES steps over diag(C)^-1, tol 1e-12): forward solve +
    backward (adjoint solve and SDDMM) through GPLHREig, timed end to end."""
    p = problems.config("c4", 2048)
    dA, dB = G.DeviceCsr.from_host(p.A), G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(problems.start_block(p.n, 10)).to("cuda")
    opts = dict(precond="gmres", steps=6, inner="diag", block=10, tol=1e-12, max_iter=3000, V0=V0)

    def once():
        valA = dA.val.clone().requires_grad_(True)
        valB = dB.val.clone().requires_grad_(True)
        lam = G.GPLHREig.apply(valA, valB, dA, dB, p.sigma, p.k, opts)
        loss = torch.sum(torch.abs(lam - p.sigma) ** 2)
        loss.backward()
        return float(loss), float(valA.grad.abs().max())

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss, gmax = once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    log(f"[bench] c4 n=2048 forward+backward: {dt*1e3:.1f} ms")
    return {"workload": "c4 generator at n=2048 (A 17 nnz/row, B = I + 0.1 S), sigma=0, k=8, block 10, "
                        "T = 6 block GMRES steps over diag(C)^-1, tol 1e-12; loss sum |lambda - sigma|^2",
            "s_forward_backward": dt, "loss": loss, "max_abs_grad_A": gmax}


def c4_full_size_convergence(G, torch, problems, its=1000):
    """The gradient workload at its configured size (n = 131072): the largest
    relative residual every 250 iterations with the strongest T and widest
    block the GPU path allows for k = 8 (6 block GMRES steps over diag(C)^-1,
    block 10).  It does not converge: the 8 wanted eigenvalues are not
    separated from the rest at this density."""
    p = problems.config("c4")
    A, B = G.DeviceCsr.from_host(p.A), G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(problems.start_block(p.n, 10)).to("cuda")
    s = G.Solver(A, B, p.sigma, p.k, 10, precond="gmres", steps=6, inner="diag", V0=V0, tol=1e-10)
    hist = {}
    done = 0
    t0 = time.perf_counter()
    st = 1
    while done < its:
        st, _, res = s.iterate(250)
        done += 250
        hist[str(done)] = res
        if st == 0:
            break
    dt = time.perf_counter() - t0
    s.close()
    log(f"[bench] c4 n=131072: residual after {done} iterations {res:.2e} ({dt:.1f} s)")
    return {"n": p.n, "block": 10, "precond": "6 block GMRES steps over diag(C)^-1",
            "rel_resid_after": hist, "converged": st == 0, "s_per_iteration": dt / done}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed GPLHR iterations of the 160^3 pencil")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--history", type=int, default=40,
                    help="iterations of the 160^3 pencil for the residual history")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline, SpMM and roofline measurements")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the block-update and Gram probes (for profiling)")
    ap.add_argument("--spmm-only", action="store_true",
                    help="only the SpMM bandwidth measurement on the 160^3 operator (for profiling)")
    ap.add_argument("--named-only", action="store_true",
                    help="only the per-iteration timing of the named stencil workloads (for profiling)")
    ap.add_argument("--d1-only", action="store_true",
                    help="only the complete n = 262144 diagonally dominant solves (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the GPLHR hot path here runs on one GPU; --gpus must be 1 "
                                   "(the row-sharded multi-GPU design is not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1506_06829_amd import gplhr as G
    from paper_1506_06829_amd import problems

    if args.spmm_only:
        stream = stream_copy_gbs(G, torch)
        c5A = problems.convection_diffusion(160, (20.0, 10.0, 5.0))
        # the solver's schedule (plane = 160^2 rows) for both precisions, then
        # the natural row order for comparison (dispatches in this order)
        res = {dt: spmm_hbm(G, torch, c5A, 16, dt) for dt in ("c64", "c128")}
        res["c64_natural_order"] = spmm_hbm(G, torch, c5A, 16, "c64", plane=0)
        # a plain device copy of known size, for scaling hardware byte counters
        x = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"spmm_160cube_b16": res, "stream_copy": stream,
                          "copy_bytes_each_way": x.numel() * 8}), flush=True)
        return

    if args.kernels_only:
        out = kernel_rooflines(G, torch)
        x = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"other_kernel_rooflines": out, "copy_bytes_each_way": x.numel() * 8}), flush=True)
        return

    if args.d1_only:
        d1, _ = d1_time_to_solution(G, torch, problems, 1, 1)
        print(json.dumps({"d1_time_to_solution": d1}), flush=True)
        return

    if args.named_only:
        named = {"c2_64cube_fp64_vs_c3_mixed": named_iteration_times(G, torch, "c2", None, 10, ["fp64", "mixed"]),
                 "c5_160cube": named_iteration_times(G, torch, "c5", None, 3, ["mixed", "fp64"])}
        print(json.dumps({"named_workloads": named}), flush=True)
        return

    # ---- headline: the 160^3 pencil, time per iteration, mixed vs FP64 ----
    p = problems.config("c5")
    log(f"[bench] workload c5 n={p.n} nnz={p.A.nnz} k=b={p.k} sigma={p.sigma}")
    A = G.DeviceCsr.from_host(p.A)
    B = G.DeviceCsr.from_host(p.B)
    V0 = torch.as_tensor(p.V0).to("cuda")
    torch.cuda.synchronize()
    c5 = c5_iterations(G, torch, p, A, B, V0, args.steps, args.warmup, args.history)
    t_mixed, t_fp64 = c5["mixed"]["s_per_iteration"], c5["fp64"]["s_per_iteration"]
    # the eigenvalues after exactly one iteration, for the comparison with the oracle
    lam1 = {}
    for prec in ("mixed", "fp64"):
        s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, sweeps=p.sweeps,
                     omega=p.omega, precision=prec, V0=V0, tol=0.0, switch_tol=0.0,
                     stall_window=10**6)
        s.iterate(1)
        lam1[prec] = s.lam()
        s.close()
    # per-class kernel times of two more mixed iterations with the timers on
    s = G.Solver(A, B, p.sigma, p.k, p.block, precond=p.precond, sweeps=p.sweeps, omega=p.omega,
                 precision="mixed", V0=V0, tol=0.0, switch_tol=0.0, stall_window=10**6, timing=True)
    s.iterate(2)
    stats_t = s.stats()
    s.close()
    del A, B, V0
    torch.cuda.empty_cache()

    # ---- SpMM HBM bandwidth on the 160^3 operator, 16-wide block ----
    c5A = p.A
    sp64 = spmm_hbm(G, torch, c5A, 16, "c64")
    sp128 = spmm_hbm(G, torch, c5A, 16, "c128")
    log(f"[bench] SpMM 160^3 b=16: c64 {sp64['gbs']:.0f} GB/s ({sp64['ms']:.3f} ms), "
        f"c128 {sp128['gbs']:.0f} GB/s ({sp128['ms']:.3f} ms)")
    stream = stream_copy_gbs(G, torch)
    for k, v in stream.items():
        log(f"[bench] streaming copy {k}: {v['gbs']:.0f} GB/s ({v['frac']:.2f} of HBM peak)")
    rooflines = kernel_rooflines(G, torch)
    for r in rooflines:
        log(f"[bench] {r['kernel']} n={r['n']}: {r['ms']*1e3:.0f} us, {r['achieved']:.0f} {r['unit']} "
            f"({r['frac']:.2f} of {r['bound']} peak)")
    dom = next(r for r in rooflines if r["kernel"].startswith(DOMINANT_KERNEL_PROBE))

    extra = {}
    if not args.no_extra:
        extra["c1g_time_to_solution"] = c1g_time_to_solution(G, torch, problems)
        d1, lam_ref = d1_time_to_solution(G, torch, problems, 3, 1)
        extra["d1_time_to_solution"] = d1
        extra["next_rows"] = next_rows(G, torch, problems, lam_ref)
        log("[bench] building the n = 4096000 diagonally dominant pencil")
        extra["d1_time_to_solution_4096000"] = large_time_to_solution(G, torch, problems)
        torch.cuda.empty_cache()
        extra["named_workloads"] = {
            "c2_64cube_fp64_vs_c3_mixed": named_iteration_times(G, torch, "c2", None, 10, ["fp64", "mixed"])}
        extra["c4_gradient"] = c4_gradient(G, torch, problems)
        extra["c4_131072_convergence"] = c4_full_size_convergence(G, torch, problems)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        log("[bench] oracle CPU baseline on the same 160^3 workload (set-up + 1 iteration)")
        t_setup, t_one, r0, r1, errs = cpu_baseline_c5(p, lam1)
        info = host_cpu_info()
        threads = max([b["threads"] for b in (info["blas"] or []) if b.get("threads")] or [1])
        cpu = {"value": t_one, "unit": "s/iteration", "cores": threads, "kind": "oracle",
               "sample": f"the FP64 oracle (numpy/scipy) on the same 160^3 workload: set-up "
                         f"(the initialisation of Algorithm 2, {t_setup:.1f} s) and one GPLHR iteration "
                         f"({t_one:.1f} s); scipy.sparse products single-threaded, dense BLAS "
                         f"on {threads} threads",
               "setup_s": t_setup, "host": info,
               "gpu_vs_oracle_after_one_iteration": {
                   "eig_rel_err": errs, "max": {k: max(v) for k, v in errs.items()}},
               "gpu_speedup_per_iteration": {"mixed": t_one / t_mixed, "fp64": t_one / t_fp64}}
        log(f"[bench] oracle: set-up {t_setup:.1f} s, one iteration {t_one:.1f} s; GPU-vs-oracle "
            f"eigenvalue rel. difference after one iteration: mixed {max(errs['mixed']):.1e}, "
            f"fp64 {max(errs['fp64']):.1e}")

    for prec in ("mixed", "fp64"):
        c5[prec]["lam"] = [str(z) for z in c5[prec]["lam"]]
    line = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s/iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": "c5: 3-D upwind convection-diffusion 160^3 (n=4096000, 28.5M nnz), "
                               "B=diag U[1,2], sigma=1000+100i, k=b=16, m=1, 3 damped Jacobi sweeps "
                               "(omega 0.7); one step = one GPLHR iteration, complex64 phase of the "
                               "mixed mode (FP64 Grams, projected step and residuals); the pencil "
                               "does not reach 1e-10 (see iterations-to-stagnation)",
                   "n": p.n, "nnz": p.A.nnz, "k": p.k, "block": p.block, "trial_width": 4 * p.block},
        "fp64": {"value": t_fp64, "unit": "s/iteration"},
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
        "c5": c5,
        "roofline": {"bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                     "unit": dom["unit"], "frac": dom["frac"], "traffic": dom.get("traffic"),
                     "kernel": dom["kernel"], "n": dom["n"], "ms_per_launch": dom["ms"],
                     "bytes_per_launch": dom.get("bytes"), "flops_per_launch": dom.get("flops")},
        "spmm": {"c64": dict(sp64, frac=sp64["gbs"] / HBM_PEAK_GBS),
                 "c128": dict(sp128, frac=sp128["gbs"] / HBM_PEAK_GBS),
                 "in_solve_ms_per_launch": stats_t["spmm_ms"] / max(1, stats_t["spmm_calls"]),
                 "in_solve_bytes_per_launch": stats_t["spmm_bytes"] / max(1, stats_t["spmm_calls"])},
        "stream_copy": stream,
        "other_kernel_rooflines": rooflines,
        "c5_mixed_kernel_class_ms_per_iteration": {
            "spmm": stats_t["spmm_ms"] / 2, "gram": stats_t["gram_ms"] / 2,
            "update": stats_t["update_ms"] / 2, "host_small_step": stats_t["small_host_ms"] / 2},
        **extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
