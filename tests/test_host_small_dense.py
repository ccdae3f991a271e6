"""CPU tests of the library's host-side dense step (small_dense.cpp): the
complex Schur form and its reordering, thin QR, the harmonic Schur-Rayleigh-
Ritz step of Algorithm 2 (ordered generalized Schur form of the projected
pencil, Section 3.3), the ordered eigenvectors of Algorithm 3, and the Q-free
factors of Theorem 2.2.  The C++ source is compiled with a small harness and
checked against LAPACK (scipy) and the defining identities; the Q-free
factors are also compared with the CPU oracle."""
import os
import subprocess
from pathlib import Path

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gplhr_oracle as O

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1506_06829_amd" / "csrc"


# Host-only sanitizer build of small_dense.cpp (g++, no device code):
# AddressSanitizer and UndefinedBehaviorSanitizer, any report fatal.
SANITIZERS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-g"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def harness(request, tmp_path_factory):
    """The harness built as the library builds small_dense.cpp, and again
    with the host sanitizers: every check below runs on both builds."""
    exe = tmp_path_factory.mktemp("host") / f"harness_{request.param}"
    flags = ["-O2", "-std=c++17", "-fcx-limited-range", f"-I{CSRC}"]
    if request.param == "sanitized":
        flags += SANITIZERS
    subprocess.run(["g++", *flags, str(ROOT / "tests" / "host_small_dense_harness.cpp"),
                    str(CSRC / "small_dense.cpp"), "-o", str(exe)], check=True)
    return exe


def fmt(M):
    return "\n".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in np.asarray(M, complex).ravel(order="F"))


def run(exe, text):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], input=text, capture_output=True, text=True, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    out = p.stdout
    lines = out.splitlines()
    ok = lines[0].split()[1] == "1"
    res, i = {}, 1
    while i < len(lines):
        name, r, c = lines[i].split()
        r, c = int(r), int(c)
        vals = np.array([[float(x) for x in l.split()] for l in lines[i + 1:i + 1 + r * c]])
        res[name] = (vals[:, 0] + 1j * vals[:, 1]).reshape((r, c), order="F") if r * c else np.zeros((r, c), complex)
        i += 1 + r * c
    return ok, res


def rand_c(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("s,nsel", [(12, 0), (40, 20), (64, 32)])
def test_schur_and_reordering(harness, s, nsel):
    rng = np.random.default_rng(s)
    M = rand_c(rng, s, s)
    ok, r = run(harness, f"schur {s} {nsel}\n{fmt(M)}\n")
    assert ok
    T, Y = r["T"], r["Y"]
    assert np.abs(Y.conj().T @ Y - np.eye(s)).max() < 1e-12
    assert np.abs(np.tril(T, -1)).max() < 1e-12 * np.abs(T).max()
    assert np.abs(Y @ T @ Y.conj().T - M).max() < 1e-12 * np.abs(M).max() * s
    ev = np.diag(T)
    ref = np.linalg.eigvals(M)
    assert np.abs(np.sort_complex(ev) - np.sort_complex(ref)).max() < 1e-10 * np.abs(ref).max()
    if nsel:
        a = np.abs(ev[:nsel])
        assert np.all(a[:-1] >= a[1:] * (1 - 1e-12))
        # the selected ones are the nsel largest in modulus
        assert np.min(a) >= np.sort(np.abs(ref))[-nsel] * (1 - 1e-10)


@pytest.mark.parametrize("r_,c", [(30, 10), (64, 48), (16, 16)])
def test_qr_thin(harness, r_, c):
    rng = np.random.default_rng(r_ + c)
    X = rand_c(rng, r_, c)
    ok, r = run(harness, f"qr {r_} {c}\n{fmt(X)}\n")
    Q, R = r["Q"], r["R"]
    assert np.abs(Q.conj().T @ Q - np.eye(c)).max() < 1e-13
    assert np.abs(np.tril(R, -1)).max() == 0 or np.abs(np.tril(R, -1)).max() < 1e-14
    d = np.diag(R)
    assert np.all(np.abs(d.imag) < 1e-14 * np.abs(d)) and np.all(d.real > 0)
    assert np.abs(Q @ R - X).max() < 1e-13 * np.abs(X).max() * r_


def _pencil(seed, s):
    rng = np.random.default_rng(seed)
    F = rand_c(rng, s, s) + 2 * np.eye(s)
    G = np.eye(s) + 0.3 * rand_c(rng, s, s)
    sigma = complex(rng.normal(), rng.normal()) * 0.5
    return F, G, sigma


@pytest.mark.parametrize("s,b,nkeep", [(40, 10, 20), (30, 10, 10), (64, 16, 32)])
def test_harmonic_srr(harness, s, b, nkeep):
    F, G, sigma = _pencil(s + b, s)
    K = F - sigma * G
    ok, r = run(harness, f"srr {s} {b} {nkeep} {float(sigma.real)!r} {float(sigma.imag)!r}\n{fmt(K)}\n{fmt(G)}\n")
    assert ok
    YR, YL, RA, RB = r["YR"], r["YL"], r["RA"], r["RB"]
    assert YR.shape == (s, nkeep) and YL.shape == (s, b)
    assert np.abs(YR.conj().T @ YR - np.eye(nkeep)).max() < 1e-12
    assert np.abs(YL.conj().T @ YL - np.eye(b)).max() < 1e-12
    # partial generalized Schur form of (F, G): F Y_R = Y_L R_A, G Y_R = Y_L R_B
    Y1 = YR[:, :b]
    assert np.abs(F @ Y1 - YL @ RA).max() < 1e-10 * np.abs(F).max()
    assert np.abs(G @ Y1 - YL @ RB).max() < 1e-10 * np.abs(G).max()
    assert np.abs(np.tril(RA, -1)).max() < 1e-12 and np.abs(np.tril(RB, -1)).max() < 1e-12
    # normalisation: R_B has a real non-negative diagonal
    dB = np.diag(RB)
    assert np.all(np.abs(dB.imag) < 1e-12 * np.abs(dB)) and np.all(dB.real >= 0)
    # the b eigenvalues of (F, G) nearest sigma, in order of distance
    lam = np.diag(RA) / dB
    ev = sla.eigvals(F, G)
    ref = ev[np.argsort(np.abs(ev - sigma))[:b]]
    assert np.abs(lam - ref).max() < 1e-9 * np.abs(ref).max()
    # Q-free factors (Theorem 2.2): equal to the oracle's for the same R_A, R_B
    MA, MB, _ = O.q_free_factors(RA, RB)
    assert np.abs(r["MA"] - MA).max() < 1e-11 * max(1.0, np.abs(MA).max())
    assert np.abs(r["MB"] - MB).max() < 1e-11 * max(1.0, np.abs(MB).max())


@pytest.mark.parametrize("s,nkeep", [(40, 20), (24, 24)])
def test_harmonic_eig(harness, s, nkeep):
    F, G, sigma = _pencil(7 * s, s)
    K = F - sigma * G
    ok, r = run(harness, f"eig {s} 0 {nkeep} {float(sigma.real)!r} {float(sigma.imag)!r}\n{fmt(K)}\n{fmt(G)}\n")
    assert ok
    Yb = r["Ybar"]
    assert Yb.shape == (s, nkeep)
    assert np.abs(np.linalg.norm(Yb, axis=0) - 1).max() < 1e-12
    # each column is an eigenvector of (F, G); eigenvalues nearest sigma first
    lam = np.array([(y.conj() @ F @ y) / (y.conj() @ G @ y) for y in Yb.T])
    res = np.linalg.norm(F @ Yb - (G @ Yb) * lam[None, :], axis=0)
    assert res.max() < 1e-9 * np.abs(F).max()
    ev = sla.eigvals(F, G)
    ref = ev[np.argsort(np.abs(ev - sigma))[:nkeep]]
    assert np.abs(lam - ref).max() < 1e-9 * np.abs(ref).max()


def test_q_free_factors_match_oracle(harness):
    rng = np.random.default_rng(5)
    b = 8
    RA = np.triu(rand_c(rng, b, b)) + 2 * np.eye(b)
    RB = np.triu(rand_c(rng, b, b))
    RB[np.diag_indices(b)] = np.abs(np.diag(RB)) + 0.5
    ok, r = run(harness, f"qfree {b}\n{fmt(RA)}\n{fmt(RB)}\n")
    MA, MB, _ = O.q_free_factors(RA, RB)
    assert np.abs(r["MA"] - MA).max() < 1e-12 * np.abs(MA).max()
    assert np.abs(r["MB"] - MB).max() < 1e-12 * np.abs(MB).max()
