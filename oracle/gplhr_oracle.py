"""Plain FP64 CPU reference implementation of GPLHR -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The product path (the HIP library and its Python binding) never
calls it, and shares no code with it.

It implements the Schur-vector form of the Generalized Preconditioned Locally
Harmonic Residual method (Vecharynski, Yang, Xue; Section 3, "The GPLHR
algorithm" of Section 3.5) from the equations that define each part, with
numpy/scipy primitives:

* the trial subspace of Section 3.1: the generalized Sylvester correction
  operator L and right-hand side F (eq. operator), the projected
  preconditioner T_L (eq. prec_gen / eq. prec) and the Krylov-Arnoldi
  sequence of T_L L (Algorithm 1, eq. krylov_sep_block), augmented by P
  (eq. trial_partial1, eq. P1);
* the test subspace and the harmonic Schur-Rayleigh-Ritz step of Section 3.3
  (eq. proj_schur, Proposition 3.2);
* the Q-free factors of Theorem 2.2 (eq. M, eqs. G1_fix / G2_fix).

Primitives:

* sparse products:  scipy.sparse CSR times a dense block,
* ``orth``:         Householder QR (scipy.linalg.qr, economic),
* ``ordqz``:        complex QZ (scipy.linalg.qz) reordered by adjacent swaps
                    (LAPACK ztgexc) so that |alpha/beta - sigma| ascends,
* small matrices:   numpy dense FP64 complex.

Readings taken where the paper is silent or inconsistent:

* ``orth`` (footnote of Algorithm 1) is any orthonormalisation of the span; we
  use Householder QR and normalise to the Q factor whose triangular factor has
  a positive real diagonal (unique for full rank).
* ordqz factors are unique only up to unimodular column scalings of Y_L, Y_R,
  and the Q-free factors M_A, M_B depend on that scaling through the
  1 - R_B(j,j) term of eq. G1_fix.  We scale so that R_B has a real
  non-negative diagonal (the choice under which M_B tends to I for B = I, as
  Section 3.3 remarks).  With both conventions fixed, every iterate is a
  well-defined function of the inputs (up to rounding).
* Test-basis step of Algorithm 2: the paper orthonormalises and then subtracts
  Q (Q^* Qhat), which would leave U non-orthonormal although Section 3.3
  requires orthonormal U.  We project first and orthonormalise afterwards.
* Ordering ties in ordqz are broken by QZ position (stable); beta = 0 sorts as
  +infinity.
* Convergence: relative eigen-residual ||A x - lambda B x|| / ||A x|| of the
  Rayleigh-Ritz eigenpairs of (V^* A V, V^* B V) (Section 5.1 uses this
  measure, with eigenvectors obtained from V by Rayleigh-Ritz, Section 2.1).
* First iteration: P is empty, so the trial space has (m+2)b columns.
* Block width b may exceed k; the k leading pairs decide convergence.

Parity pins: see tests/test_oracle.py (closed-form spectra of the 2-D and
3-D upwind stencils, dense QZ eigenvalues of small pencils, the Schur-form and
Q-free-form invariants of Section 2, Propositions 3.1 and 3.2, the residual
identity that follows Algorithm 2, the Krylov-Arnoldi sequence against the
correction operator and T_L assembled densely in Kronecker form,
exact-preconditioner and full-space special cases).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg.lapack import ztgexc


# --------------------------------------------------------------------------
# small dense building blocks
# --------------------------------------------------------------------------

def _unit_phase(z: np.ndarray) -> np.ndarray:
    a = np.abs(z)
    out = np.ones_like(z)
    nz = a > 0
    out[nz] = z[nz] / a[nz]
    return out


def orth(X: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of X (footnote of Algorithm 1 leaves
    the procedure open).  Householder QR, with the columns of the Q factor
    rescaled so that the triangular factor has a positive real diagonal: the
    unique 'Q' of X = QR for full-rank X."""
    Qx, Rx = sla.qr(X, mode="economic")
    return Qx * _unit_phase(np.diag(Rx))[None, :]


def _dist(a: complex, b: complex, sigma: complex) -> float:
    if b == 0:
        return np.inf
    return abs(a / b - sigma)


def ordqz(F: np.ndarray, G: np.ndarray, sigma: complex):
    """Full generalized Schur form of (F, G), ordered so that
    |R_A(i,i)/R_B(i,i) - sigma| is non-decreasing (the ordering footnote of
    Algorithm 2).  Returns (R_A, R_B, Y_L, Y_R) with F Y_R = Y_L R_A and
    G Y_R = Y_L R_B."""
    RA, RB, YL, YR = sla.qz(F, G, output="complex")
    s = F.shape[0]
    for pos in range(s):
        d = [_dist(RA[j, j], RB[j, j], sigma) for j in range(pos, s)]
        j = pos + int(np.argmin(d))          # first minimum: ties keep QZ order
        if j != pos:
            # ztgexc moves the diagonal entry at (1-based) ifst to ilst.
            RA, RB, YL, YR, info = ztgexc(RA, RB, YL, YR, j + 1, pos + 1)
            if info != 0:
                raise RuntimeError(f"ztgexc failed (info={info})")
    # The factors are unique only up to unimodular column scalings of Y_L and
    # Y_R; M_A, M_B (through G1 of eq. G1_fix) depend on that choice.  Fix it:
    # scale Y_L so that R_B has a real non-negative diagonal (R_A's diagonal
    # real positive where R_B(j,j) = 0).  With this choice M_B tends to I for
    # B = I, as Section 3.3 states.
    dB, dA = np.diag(RB), np.diag(RA)
    th = np.where(np.abs(dB) > 0, _unit_phase(dB), _unit_phase(dA))
    YL = YL * th[None, :]
    RA = th.conj()[:, None] * RA
    RB = th.conj()[:, None] * RB
    return RA, RB, YL, YR


def q_free_factors(RA: np.ndarray, RB: np.ndarray):
    """M_A, M_B of the 'Q-free' Schur form (Theorem 2.2, eq. M) with the
    diagonal G1, G2 of eqs. G1_fix and G2_fix (Section 2.2).  Also returns
    G = R_A G1 + R_B G2 (unit upper triangular by Lemma 2.1)."""
    k = RA.shape[0]
    g1 = np.zeros(k, dtype=complex)
    g2 = np.zeros(k, dtype=complex)
    for j in range(k):
        a, b = RA[j, j], RB[j, j]
        if abs(a) < abs(b):
            g1[j] = 0.0
            g2[j] = 1.0 / b
        else:
            g1[j] = (1.0 - b) / a
            g2[j] = 1.0
    G = RA @ np.diag(g1) + RB @ np.diag(g2)
    Ginv_RA = sla.solve_triangular(G, RA, lower=False)
    MA = np.diag(g2) @ Ginv_RA
    MB = np.eye(k) - np.diag(g1) @ Ginv_RA
    return MA, MB, G


# --------------------------------------------------------------------------
# preconditioners T ~ (A - sigma B)^{-1}  (Section 4)
# --------------------------------------------------------------------------

def block_gmres(C: sp.csr_matrix, R: np.ndarray, M: Callable[[np.ndarray], np.ndarray],
                steps: int) -> np.ndarray:
    """``steps`` block GMRES steps on C W = R from W_0 = 0 with the right
    preconditioner M (the inner solve that Section 4 suggests as a stronger T;
    block form as recommended there).

    Definition: with K = span{R, (C M) R, ..., (C M)^{s-1} R} (block Krylov
    space), W = M X where X in K minimises ||R - C M X||_F.  Computed by block
    Arnoldi (block modified Gram-Schmidt, Householder QR of each new block) and
    the small least-squares problem min_Y ||E_1 beta - Hbar Y||_F.
    """
    a = R.shape[1]
    s = steps
    V0, beta = _qr_pos(R)
    basis = [V0]
    H = np.zeros(((s + 1) * a, s * a), dtype=complex)
    for j in range(s):
        Wn = C @ M(basis[j])
        for i in range(j + 1):
            Hij = basis[i].conj().T @ Wn
            Wn = Wn - basis[i] @ Hij
            H[i * a:(i + 1) * a, j * a:(j + 1) * a] = Hij
        Vn, Hn = _qr_pos(Wn)
        H[(j + 1) * a:(j + 2) * a, j * a:(j + 1) * a] = Hn
        basis.append(Vn)
    E = np.zeros(((s + 1) * a, a), dtype=complex)
    E[:a] = beta
    Y = np.linalg.lstsq(H, E, rcond=None)[0]
    return M(np.hstack(basis[:s]) @ Y)


def _qr_pos(X: np.ndarray):
    """X = Q R, Householder QR with R's diagonal made real non-negative (the Q
    of ``orth`` together with its triangular factor)."""
    Qx, Rx = sla.qr(X, mode="economic")
    ph = _unit_phase(np.diag(Rx))
    return Qx * ph[None, :], Rx * ph.conj()[:, None]


def make_preconditioner(C: sp.csr_matrix, kind: str, sweeps: int = 3, omega: float = 0.7,
                        steps: int = 2, inner: str = "jacobi"
                        ) -> Callable[[np.ndarray], np.ndarray]:
    """T applied to a block.

    kind = "identity": T = I.
    kind = "diag":     T = diag(C)^{-1}.
    kind = "jacobi":   ``sweeps`` damped Jacobi steps on C w = r from w_0 = 0:
                       w_{t+1} = w_t + omega diag(C)^{-1} (r - C w_t).
    kind = "gmres":    ``steps`` block GMRES steps on C w = r (``block_gmres``)
                       right-preconditioned by the ``inner`` kind
                       ("identity", "diag" or "jacobi" with sweeps, omega).
    kind = "exact":    T = C^{-1} by sparse LU.
    """
    if kind == "identity":
        return lambda R: R.copy()
    d = C.diagonal()
    if kind == "diag":
        return lambda R: R / d[:, None]
    if kind == "jacobi":
        def apply(R):
            Wb = np.zeros_like(R)
            for _ in range(sweeps):
                Wb = Wb + omega * (R - C @ Wb) / d[:, None]
            return Wb
        return apply
    if kind == "gmres":
        M = make_preconditioner(C, inner, sweeps, omega)
        return lambda R: block_gmres(C, R, M, steps)
    if kind == "exact":
        lu = spla.splu(sp.csc_matrix(C))
        return lambda R: lu.solve(np.ascontiguousarray(R))
    raise ValueError(kind)


# --------------------------------------------------------------------------
# convergence measure
# --------------------------------------------------------------------------

def ritz_pairs(A, B, V: np.ndarray, sigma: complex):
    """Rayleigh-Ritz eigenpairs of (A, B) on span(V) (Section 2.1), ordered by
    |lambda - sigma|, with relative eigen-residuals ||A x - lambda B x||/||A x||
    (Section 5.1)."""
    AV = A @ V
    BV = V if B is None else B @ V
    lam, Zr = sla.eig(V.conj().T @ AV, V.conj().T @ BV)
    order = np.argsort(np.abs(lam - sigma), kind="stable")
    lam = lam[order]
    Zr = Zr[:, order]
    Zr = Zr / np.linalg.norm(Zr, axis=0)
    Ax = AV @ Zr
    Bx = BV @ Zr
    res = np.linalg.norm(Ax - Bx * lam[None, :], axis=0)
    rho = res / np.linalg.norm(Ax, axis=0)
    return lam, V @ Zr, rho, res


# --------------------------------------------------------------------------
# Section 3.1: the correction equation and its preconditioned Krylov space
# --------------------------------------------------------------------------

def projector(Y: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """X -> (I - Y Y^*) X: the orthogonal projector onto the complement of
    col{Y} (Y with orthonormal columns)."""
    return lambda X: X - Y @ (Y.conj().T @ X)


def left_basis(V: np.ndarray, Q: np.ndarray, standard: bool) -> np.ndarray:
    """The basis whose complement is the range of the correction operator:
    the left Schur basis Q of the generalized problem (eq. sylvester), the
    right basis V itself when B = I (eq. sylvester_st)."""
    return V if standard else Q


def correction_rhs(A, Bmul, X: np.ndarray, L: np.ndarray, MA: np.ndarray,
                   MB: np.ndarray, project_left: bool = True) -> np.ndarray:
    """F of eq. operator: minus the projected residual of the Q-free Schur
    form (eq. gschur2), -(I - L L^*)(A X M_B - B X M_A).  With locking, M_A and
    M_B are the columns of the active (trailing) pairs.  project_left=False
    leaves (I - L L^*) out, for the variant of Table 3 that omits the
    projection performed before T."""
    R = A @ X @ MB - Bmul(X) @ MA
    return -(projector(L)(R) if project_left else R)


def sylvester_operator(A, Bmul, V: np.ndarray, L: np.ndarray, MA: np.ndarray,
                       MB: np.ndarray, project_left: bool = True
                       ) -> Callable[[np.ndarray], np.ndarray]:
    """The generalized Sylvester operator of eq. operator,
    C -> (P_L A P_V) C M_B - (P_L B P_V) C M_A, with P_Y = I - Y Y^*
    (eq. sylvester for B != I, eq. sylvester_st with L = V for B = I).
    project_left=False leaves P_L out (the variant of Table 3)."""
    PV, PL = projector(V), projector(L)

    def apply(C: np.ndarray) -> np.ndarray:
        Cp = PV(C)
        Y = A @ Cp @ MB - Bmul(Cp) @ MA
        return PL(Y) if project_left else Y
    return apply


def projected_preconditioner(T: Callable, V: np.ndarray, L: np.ndarray,
                             right_projector: bool = True) -> Callable:
    """T_L of eq. prec_gen (eq. prec for B = I): (I - V V^*) T (I - L L^*).
    Without the right projector it is (I - V V^*) T: the variant of Table 3,
    which together with project_left=False in the operator and right-hand
    side applies T to the unprojected residual blocks."""
    PV, PL = projector(V), projector(L)
    if right_projector:
        return lambda X: PV(T(PL(X)))
    return lambda X: PV(T(X))


def krylov_arnoldi(TL: Callable, Lop: Callable, F: np.ndarray, m: int):
    """Algorithm 1: the Krylov-Arnoldi sequence K = [W, S_1, ..., S_m] of the
    operator T_L L started at T_L F (eq. krylov_sep_block).  W = orth(T_L F);
    each S_l is T_L L(S_{l-1}) (S_0 = W) made orthogonal to W and to the
    earlier S_j, then orthonormalised."""
    W = orth(TL(F))
    S: list = []
    prev = W
    for _ in range(m):
        Sl = TL(Lop(prev))
        Sl = Sl - W @ (W.conj().T @ Sl)
        for Sj in S:
            Sl = Sl - Sj @ (Sj.conj().T @ Sl)
        Sl = orth(Sl)
        S.append(Sl)
        prev = Sl
    return W, S


def augment(P: np.ndarray, blocks) -> np.ndarray:
    """The extra block of eq. trial_partial1 made orthonormal against the
    rest of the trial basis: P minus its components along each block, then
    orthonormalised."""
    for Y in blocks:
        P = P - Y @ (Y.conj().T @ P)
    return orth(P)


def harmonic_test_basis(C, Q: np.ndarray, Z_new: np.ndarray) -> np.ndarray:
    """U = [Q, Qhat], an orthonormal basis of (A - sigma B) Z whose leading
    block is Q (Proposition 3.2: C V lies in col{Q}); Qhat spans the part of
    C Z_new orthogonal to Q, Z_new being the trial blocks after V."""
    return np.hstack([Q, orth(projector(Q)(C @ Z_new))])


# --------------------------------------------------------------------------
# Algorithm 2
# --------------------------------------------------------------------------

@dataclass
class GplhrResult:
    V: np.ndarray
    Q: np.ndarray
    RA: np.ndarray
    RB: np.ndarray
    MA: np.ndarray
    MB: np.ndarray
    lam: np.ndarray          # Rayleigh-Ritz eigenvalues on span(V), nearest sigma first
    X: np.ndarray            # matching unit eigenvectors
    rho: np.ndarray          # relative eigen-residuals
    iterations: int
    converged: bool
    history: list = field(default_factory=list)   # max rho over the k leading pairs, per check
    lam_history: list = field(default_factory=list)
    lock_history: list = field(default_factory=list)  # (q, m) used by each iteration
    trace: list = field(default_factory=list)     # optional per-iteration internals

    @property
    def R(self) -> np.ndarray:
        """Standard problem output R = M_B^{-1} M_A (last line of Algorithm 2)."""
        return np.linalg.solve(self.MB, self.MA)


def gplhr(A, B, sigma: complex, k: int, V0: np.ndarray, precond: Callable,
          m: int = 1, tol: float = 1e-10, maxit: int = 500, p_mode: str = "thick",
          proj_before_T: bool = True, locking: bool = False, m_max: int = 20,
          keep_trace: bool = False, callback: Optional[Callable] = None) -> GplhrResult:
    """Algorithm 2 (GPLHR, Schur-vector form).

    A, B     scipy sparse n-by-n (B None: standard problem, B = I).
    sigma    target shift, not an eigenvalue.
    k        number of wanted eigenpairs; the block width b = V0.shape[1] >= k.
    precond  callable applying T ~ (A - sigma B)^{-1} to a block.
    m        Krylov-Arnoldi depth (number of S blocks).
    p_mode   "thick":  P = Z Ybar_R(:, b+1:2b) (eq. P1);
             "lobpcg": P = the previous V (eq. P_lobpcg: V^(i) - V^(i-1) C_V spans,
                       together with V^(i), the same space; the projections of
                       P against V, W and S then turn it into that direction);
             "none":   no P block (trial space of eq. trial_partial).
    proj_before_T  apply (I - QQ^*) (B = I: (I - VV^*)) before T, as in eqs.
             prec_gen / prec; False gives the variant of Table 3 without it.
    locking  soft locking (the remarks after Algorithm 2): once the q leading
             Rayleigh-Ritz pairs have converged (contiguously; q never decreases
             and stays below b), V and Q keep all b columns but W, S_l and P
             are built for the a = b - q trailing columns only (the S recursion
             uses the trailing a-by-a blocks of M_A, M_B; P keeps its first a
             columns), and m <- min(floor(m0 b / (b - q)), m_max).
    """
    A = sp.csr_matrix(A)
    std = B is None
    Bm = sp.identity(A.shape[0], format="csr", dtype=complex) if std else sp.csr_matrix(B)
    C = (A - sigma * Bm).tocsr()
    b = V0.shape[1]
    if k > b:
        raise ValueError("k must not exceed the block width")

    def Bx(X):
        return X if std else Bm @ X

    # initial bases: V = orth(V0), Q = orth((A - sigma B) V), then their
    # ordered Schur form and the Q-free factors (Theorem 2.2)
    V = orth(V0)
    Q = orth(C @ V)
    P = None
    RA, RB, YL, YR = ordqz(Q.conj().T @ (A @ V), Q.conj().T @ Bx(V), sigma)
    V = V @ YR
    Q = Q @ YL
    MA, MB, _ = q_free_factors(RA, RB)

    history, lam_history, lock_history, trace = [], [], [], []
    m0 = m
    q = 0
    it = 0
    while True:
        lam, X, rho, _ = ritz_pairs(A, None if std else Bm, V, sigma)
        history.append(float(np.max(rho[:k])))
        lam_history.append(lam[:k].copy())
        if callback is not None:
            callback(it, lam, rho)
        if np.max(rho[:k]) <= tol or it >= maxit:
            break
        it += 1
        if locking:
            nconv = 0
            while nconv < b and rho[nconv] <= tol:
                nconv += 1
            q = max(q, min(nconv, b - 1))
            m = min((m0 * b) // (b - q), m_max)
        a = b - q
        lock_history.append((q, m))
        if P is not None:
            P = P[:, :a]
        # trial subspace (Section 3.1): the correction equation of the a
        # active pairs, L(C) = F with V^* C = 0 (eq. operator), and the
        # Krylov-Arnoldi sequence of T_L L from T_L F (Algorithm 1)
        L = left_basis(V, Q, std)
        Lop = sylvester_operator(A, Bx, V, L, MA[q:, q:], MB[q:, q:], proj_before_T)
        F = correction_rhs(A, Bx, V, L, MA[:, q:], MB[:, q:], proj_before_T)
        TL = projected_preconditioner(precond, V, L, proj_before_T)
        W, S_list = krylov_arnoldi(TL, Lop, F, m)
        S = np.hstack(S_list)
        # the extra search directions of eq. trial_partial1 (Section 3.4)
        if P is not None:
            P = augment(P, [V, W, S])
        Z = np.hstack([V, W, S] + ([P] if P is not None else []))
        # test subspace (Section 3.3, Proposition 3.2)
        U = harmonic_test_basis(C, Q, Z[:, b:])
        # harmonic Schur-Rayleigh-Ritz (Section 3.3, eq. proj_schur): ordered
        # generalized Schur form of the projected pencil (U^* A Z, U^* B Z)
        Fp = U.conj().T @ (A @ Z)
        Gm = U.conj().T @ Bx(Z)
        RAb, RBb, YLb, YRb = ordqz(Fp, Gm, sigma)
        RA = RAb[:b, :b]
        RB = RBb[:b, :b]
        state_in = dict(V_in=V, Q_in=Q, MA_in=MA, MB_in=MB, W=W, S=S_list, q=q)
        # new approximate Schur bases V = Z Y_R, Q = U Y_L
        V_old = V
        V = Z @ YRb[:, :b]
        Q = U @ YLb[:, :b]
        # P: thick restart (eq. P1), the previous V (eq. P_lobpcg), or none
        if p_mode == "thick":
            P = Z @ YRb[:, b:b + a]
        elif p_mode == "lobpcg":
            P = V_old[:, q:]
        else:
            P = None
        # Q-free factors of the new Schur form (Theorem 2.2, eq. M)
        MA, MB, _ = q_free_factors(RA, RB)
        if keep_trace:
            trace.append(dict(Z=Z, U=U, F=Fp, G=Gm, RAb=RAb, RBb=RBb, YLb=YLb, YRb=YRb,
                              V=V, Q=Q, RA=RA, RB=RB, MA=MA, MB=MB, **state_in))

    return GplhrResult(V=V, Q=Q, RA=RA, RB=RB, MA=MA, MB=MB, lam=lam, X=X, rho=rho,
                       iterations=it, converged=bool(np.max(rho[:k]) <= tol),
                       history=history, lam_history=lam_history,
                       lock_history=lock_history, trace=trace)


@dataclass
class GplhrEigResult:
    X: np.ndarray            # unit-norm approximate eigenvectors (n x b)
    alpha: np.ndarray        # diag(X^* A X)  (Lambda_A)
    beta: np.ndarray         # diag(X^* B X)  (Lambda_B)
    lam: np.ndarray          # alpha / beta, in the column order of X
    rho: np.ndarray          # ||A x - lam B x|| / ||A x||
    iterations: int
    converged: bool
    history: list = field(default_factory=list)
    lam_history: list = field(default_factory=list)


def _unit_columns_and_forms(A, Bm, X):
    X = X / np.linalg.norm(X, axis=0)[None, :]
    AX = A @ X
    BX = Bm @ X
    alpha = np.einsum("ij,ij->j", X.conj(), AX)
    beta = np.einsum("ij,ij->j", X.conj(), BX)
    return X, AX, BX, alpha, beta


def gplhr_eig(A, B, sigma: complex, k: int, X0: np.ndarray, precond: Callable,
              m: int = 1, tol: float = 1e-10, maxit: int = 500, p_mode: str = "thick",
              callback: Optional[Callable] = None) -> GplhrEigResult:
    """Algorithm 3 (GPLHR-EIG, Appendix A): the eigenvector form.

    The iterate is a block X of unit-norm approximate eigenvectors with the
    diagonal bilinear forms Lambda_A = diag(X^* A X), Lambda_B = diag(X^* B X);
    the eigenvalue approximations are their ratios (Rayleigh quotients).  The
    residual block is A X Lambda_B - B X Lambda_A, the S recursion applies the
    same diagonal forms, and the projected pencil (U^* A Z, U^* B Z) is solved
    by a full eigendecomposition ordered by closeness to sigma.  b = X0.shape[1]
    columns are iterated; the k leading ones decide convergence, measured by
    ||A x_j - lambda_j B x_j|| / ||A x_j|| at the Rayleigh quotient lambda_j.

    p_mode  "thick":  P = Z Ybar(:, b+1:2b) (the thick restart of Algorithm 3);
            "lobpcg": P = W Y_W + S Y_S + P Y_P (Algorithm 3's LOBPCG-style
                      direction, without the thick restart);
            "none":   no P block.
    Reading: the test-basis step projects against Q before orthonormalising
    (as for Algorithm 2).
    """
    A = sp.csr_matrix(A)
    std = B is None
    Bm = sp.identity(A.shape[0], format="csr", dtype=complex) if std else sp.csr_matrix(B)
    C = (A - sigma * Bm).tocsr()
    b = X0.shape[1]
    X, AX, BX, alpha, beta = _unit_columns_and_forms(A, Bm, X0.astype(complex))
    Q = C @ X
    P = None
    history, lam_history = [], []
    it = 0
    while True:
        lam = alpha / beta
        rho = np.linalg.norm(AX - BX * lam[None, :], axis=0) / np.linalg.norm(AX, axis=0)
        history.append(float(np.max(rho[:k])))
        lam_history.append(lam[:k].copy())
        if callback is not None:
            callback(it, lam, rho)
        if np.max(rho[:k]) <= tol or it >= maxit:
            break
        it += 1
        # orthonormal bases of the current X and of (A - sigma B) X
        V = orth(X)
        Q = orth(Q)
        # the correction equation with the diagonal forms Lambda_A, Lambda_B in
        # place of M_A, M_B, and its Krylov-Arnoldi sequence (Algorithm 1)
        L = left_basis(V, Q, std)
        LA, LB = np.diag(alpha), np.diag(beta)
        Lop = sylvester_operator(A, lambda Y: Bm @ Y, V, L, LA, LB)
        F = correction_rhs(A, lambda Y: Bm @ Y, X, L, LA, LB)
        W, S_list = krylov_arnoldi(projected_preconditioner(precond, V, L), Lop, F, m)
        S = np.hstack(S_list)
        if P is not None:
            P = augment(P, [V, W, S])
        Z = np.hstack([V, W, S] + ([P] if P is not None else []))
        U = harmonic_test_basis(C, Q, Z[:, b:])
        # eigenvectors of the projected pencil (U^* A Z, U^* B Z), nearest sigma first
        ev, Yb = sla.eig(U.conj().T @ (A @ Z), U.conj().T @ (Bm @ Z), homogeneous_eigvals=True)
        d = np.array([_dist(ev[0][j], ev[1][j], sigma) for j in range(ev.shape[1])])
        Yb = Yb[:, np.argsort(d, kind="stable")]
        Y = Yb[:, :b]
        # new X from the leading eigenvectors; P from the next ones (thick
        # restart) or from the non-V part of X (LOBPCG-style direction)
        Pn = Z[:, b:] @ Y[b:, :]
        X = V @ Y[:b, :] + Pn
        Q = C @ X
        if p_mode == "thick":
            P = Z @ Yb[:, b:2 * b] if Z.shape[1] >= 2 * b else None
        elif p_mode == "lobpcg":
            P = Pn
        else:
            P = None
        # unit columns and the diagonal forms diag(X^* A X), diag(X^* B X)
        X, AX, BX, alpha, beta = _unit_columns_and_forms(A, Bm, X)
    return GplhrEigResult(X=X, alpha=alpha, beta=beta, lam=lam, rho=rho, iterations=it,
                          converged=bool(np.max(rho[:k]) <= tol), history=history,
                          lam_history=lam_history)


def deflated_pair(A, B, V1: np.ndarray, Q1: Optional[np.ndarray]):
    """The deflated pair of the remarks after Algorithm 2, formed explicitly
    (dense, small n only): ((I - Q1 Q1^*) A (I - V1 V1^*), (I - Q1 Q1^*) B (I - V1 V1^*)),
    or ((I - V1 V1^*) A (I - V1 V1^*), None) for B = I."""
    L = V1 if B is None else Q1

    def both(M):
        M = M - L @ (L.conj().T @ M)
        return M - (M @ V1) @ V1.conj().T

    Ad = both(sp.csr_matrix(A).toarray().astype(complex))
    Bd = None if B is None else both(sp.csr_matrix(B).toarray().astype(complex))
    return sp.csr_matrix(Ad), None if Bd is None else sp.csr_matrix(Bd)


def gplhr_deflated(A, B, sigma: complex, k: int, V0: np.ndarray, precond: Callable,
                   V1: np.ndarray, Q1: Optional[np.ndarray], **kw) -> GplhrResult:
    """Further Schur vectors by deflation: Algorithm 2 on ``deflated_pair``.

    Reading (the paper names the deflated pair only): the iteration starts
    from (I - V1 V1^*) V0 and the preconditioner is followed by
    (I - V1 V1^*), so that the trial subspace stays orthogonal to the deflated
    vectors (on span(V1) the deflated pair vanishes identically)."""
    Ad, Bd = deflated_pair(A, B, V1, Q1)

    def pv(X):
        return X - V1 @ (V1.conj().T @ X)

    return gplhr(Ad, Bd, sigma, k, pv(V0), lambda R: pv(precond(R)), **kw)


def solve_problem(problem, tol: Optional[float] = None, maxit: int = 500, **kw) -> GplhrResult:
    """Run the oracle on a ``problems.Problem`` (inputs only; no method code
    lives there)."""
    A = problem.A.to_scipy()
    B = None if problem.B is None else problem.B.to_scipy()
    Bm = sp.identity(A.shape[0], format="csr") if B is None else B
    C = (A - problem.sigma * Bm).tocsr()
    T = make_preconditioner(C, problem.precond, problem.sweeps, problem.omega,
                            problem.steps, problem.inner)
    solver = gplhr_eig if kw.pop("algorithm", "schur") == "eig" else gplhr
    return solver(A, B, problem.sigma, problem.k, problem.V0, T,
                  tol=problem.tol if tol is None else tol, maxit=maxit, **kw)
