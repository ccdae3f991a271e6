// GPLHR driver: Algorithm 2 ("The GPLHR algorithm", Section 3.5) on one HIP
// stream, with the block work in kernels.hip and the small projected step in
// small_dense.cpp.  Exposed through the C ABI in capi.cpp.
//
// Trial basis layout (n-by-smax, row-major, ld = smax, smax = (m+3) b):
//   Z = [ V | W | S_1 .. S_mc | P ]   with V at column 0 (b columns) and, for
//   the a = b - q active columns (q locked, 0 without locking), W at b, S_l at
//   b + l a and P at pos = b + (mc+1) a, mc the depth of the iteration.  Since
//   mc a <= m b, everything fits in smax columns.  Between iterations P is kept
//   at smax - b (= pos when q = 0) and moved to pos when the layout shrinks.
//   CZ = C Z with C = A - sigma B is kept alongside Z (fresh sparse products for
//   W and S_l, the same linear combinations as Z for V and P), BZ likewise when
//   B is a general sparse matrix.  U = [ Q | Qhat ].
#include "driver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace gplhr {

using small::Mat;

static double2 to_d2(cd z) { return make_double2(z.real(), z.imag()); }

// ---------------------------------------------------------------------------
// allocation helpers
// ---------------------------------------------------------------------------
template <typename P>
static void dalloc(P **p, size_t count, hipStream_t st) {
    *p = static_cast<P *>(dev_alloc((count ? count : 1) * sizeof(P), st));
}
template <typename P>
static void dfree(P *&p, hipStream_t st) {
    dev_free((void *)p, st);
    p = nullptr;
}

Ctx::~Ctx() {
    for (auto &pr : timers) {
        for (auto &ev : pr.second.pool) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    }
    dfree(c_rp, st); dfree(c_ci, st); dfree(c_val, st); dfree(c_val32, st);
    dfree(a_rp, st); dfree(a_ci, st); dfree(a_val, st);
    dfree(b_rp, st); dfree(b_ci, st); dfree(b_val, st); dfree(b_val32, st);
    dfree(bd, st); dfree(bd32, st); dfree(dinv, st); dfree(dinv32, st); dfree(dw, st); dfree(dw32, st);
    dfree(cvdw, st); dfree(cvdw32, st);
    for (Work<double2> *w : {&wd}) { dfree(w->Z, st); dfree(w->CZ, st); dfree(w->BZ, st); dfree(w->U, st); dfree(w->R, st); dfree(w->J1, st); dfree(w->J2, st); dfree(w->G, st); dfree(w->Gz, st); dfree(w->Gx, st); dfree(w->Vd, st); dfree(w->Qd, st); }
    for (Work<float2> *w : {&wf}) { dfree(w->Z, st); dfree(w->CZ, st); dfree(w->BZ, st); dfree(w->U, st); dfree(w->R, st); dfree(w->J1, st); dfree(w->J2, st); dfree(w->G, st); dfree(w->Gz, st); dfree(w->Gx, st); dfree(w->Vd, st); dfree(w->Qd, st); }
    dfree(part, st); dfree(g0, st); dfree(g1, st); dfree(rinv, st); dfree(coefY, st); dfree(cpack, st);
    dfree(mbase, st); dfree(fbase, st); dfree(dZr, st); dfree(rnorm, st);
    dfree(gmH, st); dfree(gmY, st);
    // the staging buffers go back to the free list only once the stream has
    // finished with them (dev_free above waited for it)
    (void)hipStreamSynchronize(st);
    pinned_free(hpin, hpin_bytes);
    pinned_free(hgm, hgm_bytes);
}

// ---------------------------------------------------------------------------
// timing of kernel classes with HIP events on the solver stream
// ---------------------------------------------------------------------------
void Ctx::tbegin(int cls) {
    if (!opt.timing) return;
    Timer &t = timers[cls];
    if (t.used == (int)t.pool.size()) {
        hipEvent_t a, b;
        GPLHR_HIP_CHECK(hipEventCreate(&a));
        GPLHR_HIP_CHECK(hipEventCreate(&b));
        t.pool.push_back({a, b});
    }
    GPLHR_HIP_CHECK(hipEventRecord(t.pool[t.used].first, st));
}
void Ctx::tend(int cls) {
    if (!opt.timing) return;
    Timer &t = timers[cls];
    GPLHR_HIP_CHECK(hipEventRecord(t.pool[t.used].second, st));
    ++t.used;
}
void Ctx::tflush() {
    if (!opt.timing) return;
    for (auto &pr : timers) {
        Timer &t = pr.second;
        for (int i = 0; i < t.used; ++i) {
            float ms = 0.f;
            GPLHR_HIP_CHECK(hipEventSynchronize(t.pool[i].second));
            GPLHR_HIP_CHECK(hipEventElapsedTime(&ms, t.pool[i].first, t.pool[i].second));
            t.ms += ms;
            t.count += 1;
        }
        t.used = 0;
    }
}

// Vanishing Cholesky pivots counted on the device so far (waits for the stream).
int Ctx::read_breakdowns() {
    int *hs = reinterpret_cast<int *>(hpin);
    GPLHR_HIP_CHECK(hipMemcpyAsync(hs, dstatus, sizeof(int), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    return *hs;
}

template <> Work<double2> &Ctx::W<double2>() { return wd; }
template <> Work<float2> &Ctx::W<float2>() { return wf; }

// ---------------------------------------------------------------------------
// block primitives
// ---------------------------------------------------------------------------
template <typename T>
void Ctx::gram(const T *X, int ldx, int bx, const T *Y, int ldy, int by, const T *yscale,
               double2 *out) {
    tbegin(T_GRAM);
    launch_gram<T>(st, n, X, ldx, bx, Y, ldy, by, yscale, part, PART_CAP, out, bx);
    tend(T_GRAM);
}

template <typename T>
void Ctx::update(T *out, int ldo, int wout, int ocol, int split, int ocol2, bool beta1,
                 int nterms, const UpdTerm<T> *terms, const T *add, int ldadd) {
    tbegin(T_UPDATE);
    launch_update<T>(st, n, out, ldo, wout, ocol, split, ocol2,
                     beta1 ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0), nterms, terms,
                     add, ldadd);
    tend(T_UPDATE);
}

// X(:, xcol:xcol+wx) -= Y(:, ycol:ycol+wy) (Y^H X)   [mirrors receive the same
// coefficients applied to their own columns]
template <typename T>
void Ctx::project(T *X, int ldx, int xcol, int wx, const T *Y, int ldy, int ycol, int wy,
                  T *mir1, const T *ymir1, T *mir2, const T *ymir2) {
    gram<T>(Y + ycol, ldy, wy, X + xcol, ldx, wx, nullptr, g0);
    UpdTerm<T> t;
    t.in = Y; t.ld = ldy; t.col = ycol; t.w = wy; t.M = g0; t.ldm = wy;
    t.alpha = make_double2(-1.0, 0.0);
    update<T>(X, ldx, wx, xcol, wx, 0, true, 1, &t);
    if (mir1) {
        t.in = ymir1;
        update<T>(mir1, ldx, wx, xcol, wx, 0, true, 1, &t);
    }
    if (mir2) {
        t.in = ymir2;
        update<T>(mir2, ldx, wx, xcol, wx, 0, true, 1, &t);
    }
}

// Cholesky-QR, `passes` times: X <- X R^{-1} with X^H X = R^H R (FP64 Gram);
// mirrors are multiplied by the same R^{-1}.
template <typename T>
void Ctx::cholqr(T *X, int ld, int col, int w, int passes, T *mir1, T *mir2) {
    for (int p = 0; p < passes; ++p) {
        gram<T>(X + col, ld, w, X + col, ld, w, nullptr, g0);
        launch_chol_rinv(st, w, g0, rinv, dstatus);
        UpdTerm<T> t;
        t.in = X; t.ld = ld; t.col = col; t.w = w; t.M = rinv; t.ldm = w; t.upper = true;
        update<T>(X, ld, w, col, w, 0, false, 1, &t);
        if (mir1) {
            t.in = mir1;
            update<T>(mir1, ld, w, col, w, 0, false, 1, &t);
        }
        if (mir2) {
            t.in = mir2;
            update<T>(mir2, ld, w, col, w, 0, false, 1, &t);
        }
    }
}

// X(:, xcol:xcol+w) <- orth((I - Y Y^H) X) for Y = X(:, ycol:ycol+wy), the
// orthonormal columns just before the block (ycol + wy = xcol; wy may be 0).
// Each pass is one Gram [Y X]^H X, the Cholesky factor of the projected
// block's Gram X^H X - (Y^H X)^H (Y^H X), and one row-local update
// X <- X Rinv + Y Cy with Cy = -(Y^H X) Rinv; a second pass restores what
// the first loses to cancellation (two passes equal block Gram-Schmidt twice
// followed by Cholesky-QR twice, to rounding).  A pass whose projection
// cancels almost all of a column only projects (see launch_chol_proj).
template <typename T>
void Ctx::proj_orth(T *X, int ld, int ycol, int wy, int xcol, int w, int passes) {
    for (int p = 0; p < passes; ++p) {
        gram<T>(X + ycol, ld, wy + w, X + xcol, ld, w, nullptr, g0);
        launch_chol_proj(st, wy, w, g0, rinv, g1, dstatus, p + 1 < passes);
        UpdTerm<T> t[2];
        t[0].in = X; t[0].ld = ld; t[0].col = xcol; t[0].w = w; t[0].M = rinv; t[0].ldm = w;
        t[0].upper = true;
        t[1].in = X; t[1].ld = ld; t[1].col = ycol; t[1].w = wy; t[1].M = g1; t[1].ldm = wy;
        update<T>(X, ld, w, xcol, w, 0, false, wy > 0 ? 2 : 1, t);
    }
}

template <typename T>
void Ctx::spmm_c(const T *X, int ldx, T *Y, int ldy, int wc, int mode, const T *Rhs, int ldr) {
    Work<T> &w = W<T>();
    tbegin(T_SPMM);
    if (mode == 2 && !w.cvdw) throw Error(-1, "spmm: the two-sweep product needs the values of C diag(dw)");
    launch_spmm<T>(st, n, c_rp, c_ci, mode == 2 ? w.cvdw : w.cval, X, ldx, Y, ldy, wc, mode, Rhs, ldr, w.dw,
                   c_plane, c_nnz);
    tend(T_SPMM);
    ++n_spmm;
    spmm_bytes += (double)c_nnz * (sizeof(T) + 4) + 4.0 * (n + 1) +
                  (double)n * wc * sizeof(T) * (mode == 1 ? 3 : 2);
}

template <typename T>
void Ctx::spmm_b(const T *X, int ldx, T *Y, int ldy, int wc) {
    Work<T> &w = W<T>();
    tbegin(T_SPMM);
    launch_spmm<T>(st, n, b_rp, b_ci, w.bval, X, ldx, Y, ldy, wc, 0, nullptr, 0, nullptr, b_plane, b_nnz);
    tend(T_SPMM);
    ++n_spmm;
    spmm_bytes += (double)b_nnz * (sizeof(T) + 4) + 4.0 * (n + 1) + 2.0 * n * wc * sizeof(T);
}

// Deflation (remarks after Algorithm 2): with converged bases V1, Q1 the
// iteration runs on ((I - Q1 Q1^H) A (I - V1 V1^H), (I - Q1 Q1^H) B (I - V1 V1^H))
// (Q1 = V1 for B = I).  The trial basis is kept orthogonal to V1, so the
// deflated products are the plain ones followed by (I - Q1 Q1^H).
template <typename T>
void Ctx::deflate_left(T *Y, int ldy, int wc) {
    Work<T> &w = W<T>();
    project<T>(Y, ldy, 0, wc, w.Qd, defl_k, 0, defl_k);
}
template <typename T>
void Ctx::deflate_right(T *X, int ldx, int col, int wc) {
    Work<T> &w = W<T>();
    project<T>(X, ldx, col, wc, w.Vd, defl_k, 0, defl_k);
}

// Y = C X (deflated), for blocks of the trial basis
template <typename T>
void Ctx::cprod(const T *X, int ldx, T *Y, int ldy, int wc) {
    spmm_c<T>(X, ldx, Y, ldy, wc, 0, nullptr, 0);
    if (defl_k) deflate_left<T>(Y, ldy, wc);
}

// Y = B X (deflated) when B Z is kept explicitly; nothing otherwise
template <typename T>
void Ctx::bprod(const T *X, int ldx, T *Y, int ldy, int wc) {
    if (!bexp()) return;
    if (bk == B_SPARSE) spmm_b<T>(X, ldx, Y, ldy, wc);
    else launch_scale_rows<T>(st, n, wc, X, ldx, W<T>().bd, Y, ldy);
    if (defl_k) deflate_left<T>(Y, ldy, wc);
}

// dest = M in for a basic preconditioner kind (NONE, DIAG, JACOBI); wc columns.
template <typename T>
void Ctx::apply_inner(int kind, const T *in, int ldi, T *dest, int ldd, int wc) {
    Work<T> &w = W<T>();
    if (kind == GPLHR_PRECOND_NONE) {
        launch_scale_rows<T>(st, n, wc, in, ldi, nullptr, dest, ldd);
    } else if (kind == GPLHR_PRECOND_DIAG) {
        launch_scale_rows<T>(st, n, wc, in, ldi, w.dinv, dest, ldd);
    } else {
        // w_1 = omega D^{-1} r; w_{t+1} = w_t + omega D^{-1} (r - C w_t)
        if (pre.sweeps == 1) {
            launch_scale_rows<T>(st, n, wc, in, ldi, w.dw, dest, ldd);
            return;
        }
        // w_1 and w_2 in one pass (SpMM mode 2: C w_1 = (C diag(dw)) r from
        // the prescaled values), then one pass per further sweep
        T *cur = nullptr;
        for (int t = 1; t < pre.sweeps; ++t) {
            const bool last = (t == pre.sweeps - 1);
            T *o = last ? dest : (cur == w.J1 ? w.J2 : w.J1);
            if (t == 1) spmm_c<T>(in, ldi, o, last ? ldd : b, wc, 2, in, ldi);
            else spmm_c<T>(cur, b, o, last ? ldd : b, wc, 1, in, ldi);
            cur = o;
        }
    }
}

// dest(:, dcol:dcol+wc) = T R  (R = Work.R, ld b, wc <= b columns)
template <typename T>
void Ctx::apply_T(T *dest, int ldd, int dcol, int wc) {
    ++n_prec;
    if (pre.kind == GPLHR_PRECOND_GMRES)
        apply_gmres<T>(dest, ldd, dcol, wc);
    else
        apply_inner<T>(pre.kind, W<T>().R, b, dest + dcol, ldd, wc);
}

// Block GMRES(s) on C X = R from X_0 = 0 with the right preconditioner M:
// block Arnoldi on C M from V_0 beta = R (classical block Gram-Schmidt, two
// passes; Cholesky-QR, two passes), then min ||E_1 beta - Hbar Y||_F on the
// host and dest = M (V_{0..s-1} Y).  One host synchronisation per call.
template <typename T>
void Ctx::apply_gmres(T *dest, int ldd, int dcol, int a) {
    Work<T> &w = W<T>();
    const int s = pre.steps, lg = (s + 1) * b;
    T *G = w.G;
    // small factors: slot(j, 0/1) = Gram-Schmidt coefficients of both passes
    // for step j, slot(j, 2/3) = Cholesky factors of both passes (j = s: beta)
    auto slot = [&](int j, int kind) { return gmH + (size_t)(j * 4 + kind) * GM_SLOT; };
    auto qr2 = [&](int col, int j) {
        for (int p = 0; p < 2; ++p) {
            gram<T>(G + col, lg, a, G + col, lg, a, nullptr, g0);
            launch_chol_rinv(st, a, g0, rinv, dstatus, slot(j, 2 + p));
            UpdTerm<T> t;
            t.in = G; t.ld = lg; t.col = col; t.w = a; t.M = rinv; t.ldm = a; t.upper = true;
            update<T>(G, lg, a, col, a, 0, false, 1, &t);
        }
    };
    launch_scale_rows<T>(st, n, a, w.R, b, nullptr, G, lg);
    qr2(0, s);
    for (int j = 0; j < s; ++j) {
        apply_inner<T>(pre.inner, G + j * a, lg, w.Gz, b, a);          // M V_j
        spmm_c<T>(w.Gz, b, G + (j + 1) * a, lg, a, 0, nullptr, 0);     // C M V_j
        const int wv = (j + 1) * a;
        for (int p = 0; p < 2; ++p) {
            gram<T>(G, lg, wv, G + wv, lg, a, nullptr, slot(j, p));
            UpdTerm<T> t;
            t.in = G; t.ld = lg; t.col = 0; t.w = wv; t.M = slot(j, p); t.ldm = wv;
            t.alpha = make_double2(-1.0, 0.0);
            update<T>(G, lg, a, wv, a, 0, true, 1, &t);
        }
        qr2(wv, j);
    }
    const size_t tot = (size_t)(s + 1) * 4 * GM_SLOT;
    GPLHR_HIP_CHECK(hipMemcpyAsync(hgm, gmH, tot * sizeof(double2), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    tflush();
    const cd *h = reinterpret_cast<const cd *>(hgm);
    auto sl = [&](int j, int kind) { return h + (size_t)(j * 4 + kind) * GM_SLOT; };
    auto tri = [&](int j) {   // R2 R1 of the two Cholesky-QR passes
        Mat r1(a, a), r2(a, a);
        std::memcpy(r1.data(), sl(j, 2), (size_t)a * a * sizeof(cd));
        std::memcpy(r2.data(), sl(j, 3), (size_t)a * a * sizeof(cd));
        return small::matmul(r2, r1);
    };
    Mat Hb((s + 1) * a, s * a), E((s + 1) * a, a);
    const Mat beta = tri(s);
    for (int jj = 0; jj < a; ++jj)
        for (int ii = 0; ii < a; ++ii) E(ii, jj) = beta(ii, jj);
    for (int j = 0; j < s; ++j) {
        const int wv = (j + 1) * a;
        const cd *h1 = sl(j, 0), *h2 = sl(j, 1);
        for (int jj = 0; jj < a; ++jj)
            for (int ii = 0; ii < wv; ++ii)
                Hb(ii, j * a + jj) = h1[ii + (size_t)jj * wv] + h2[ii + (size_t)jj * wv];
        const Mat r = tri(j);
        for (int jj = 0; jj < a; ++jj)
            for (int ii = 0; ii < a; ++ii) Hb(wv + ii, j * a + jj) = r(ii, jj);
    }
    for (const cd &v : Hb.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
            throw Error(-6, "non-finite block GMRES Hessenberg matrix");
    Mat Qh, Rh;
    small::qr_thin(Hb, Qh, Rh);
    const Mat Y = small::tri_solve_upper(Rh, small::matmul_hn(Qh, E));
    std::memcpy(hgm, Y.data(), (size_t)s * a * a * sizeof(cd));
    GPLHR_HIP_CHECK(hipMemcpyAsync(gmY, hgm, (size_t)s * a * a * sizeof(double2), hipMemcpyHostToDevice, st));
    UpdTerm<T> t;
    t.in = G; t.ld = lg; t.col = 0; t.w = s * a; t.M = gmY; t.ldm = s * a;
    update<T>(w.Gx, b, a, 0, a, 0, false, 1, &t);
    apply_inner<T>(pre.inner, w.Gx, b, dest + dcol, ldd, a);
    // hgm is written again only after the next call's synchronisation, which
    // follows this upload on the stream.
}

// ---------------------------------------------------------------------------
// projected pencil -> ordered Schur form -> basis update
// ---------------------------------------------------------------------------
// p_cols: width of the P block the update should produce (0: none).
template <typename T>
void Ctx::srr_and_update(int s_cur, int p_cols) {
    Work<T> &w = W<T>();
    const int ld = smax;
    const T *bsrc = bexp() ? w.BZ : w.Z;
    const T *bsc = bscale<T>();
    // a8: F1 = U^H (A - sigma B) Z, F2 = U^H B Z   (s_cur x s_cur, FP64)
    // F2 follows F1 in one buffer, so both come back in one copy
    const size_t ss = (size_t)s_cur * s_cur;
    double2 *F2 = F1 + ss;
    gram<T>(w.U, ld, s_cur, w.CZ, ld, s_cur, nullptr, F1);
    gram<T>(w.U, ld, s_cur, bsrc, ld, s_cur, bsc, F2);
    GPLHR_HIP_CHECK(hipMemcpyAsync(hpin, fbase, (1 + 2 * ss) * sizeof(double2), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    tflush();
    const int64_t breakdowns_before = n_breakdown;
    {
        int stv = 0;
        std::memcpy(&stv, hpin, sizeof(int));
        n_breakdown = stv;
    }
    // a singular projected pencil after vanishing Cholesky pivots in this
    // iteration comes from a block that lost rank, not from the shift
    auto singular = [&]() {
        if (n_breakdown > breakdowns_before)
            return Error(-4, "orthonormalisation broke down: a block of the trial or test basis "
                             "lost rank and the projected pencil is singular");
        return Error(-5, "projected pencil is singular: sigma is numerically an eigenvalue "
                         "(Proposition 3.1)");
    };
    // a9: ordered generalized Schur form on the host (FP64)
    auto t0 = std::chrono::steady_clock::now();
    Mat K(s_cur, s_cur), Gm(s_cur, s_cur);
    std::memcpy(K.data(), hpin + 1, ss * sizeof(cd));
    std::memcpy(Gm.data(), hpin + 1 + ss, ss * sizeof(cd));
    for (const cd &v : K.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
            throw Error(-6, "non-finite entries in the projected pencil");
    const bool lobpcg = (opt.p_mode == GPLHR_P_LOBPCG);
    const bool thick = (opt.p_mode == GPLHR_P_THICK);
    const int nkeep = std::min(thick ? b + p_cols : b, s_cur);
    const int offP = smax - b;
    if (eig) {
        // Algorithm 3, the harmonic Rayleigh-Ritz step: eigenvectors Ybar of
        // the projected pencil nearest sigma; X = Z Ybar(:, 1:b),
        // P = Z Ybar(:, b+1:b+p) (thick) or P = [W S P] Ybar(b+1:s, 1:b)
        // (LOBPCG-style)
        Mat Yb;
        if (!small::harmonic_eig(K, Gm, nkeep, Yb)) throw singular();
        small_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        int nc = Yb.c;
        cd *hc = reinterpret_cast<cd *>(hpin);
        std::memcpy(hc, Yb.data(), (size_t)s_cur * nc * sizeof(cd));
        if (lobpcg && p_cols > 0 && s_cur > b) {
            cd *ext = hc + (size_t)s_cur * nc;
            for (int j = 0; j < p_cols; ++j)
                for (int i = 0; i < s_cur; ++i)
                    ext[(size_t)j * s_cur + i] = (i < b) ? cd(0.0, 0.0) : Yb(i, (b - p_cols) + j);
            nc += p_cols;
        }
        GPLHR_HIP_CHECK(hipMemcpyAsync(coefY, hpin, (size_t)s_cur * nc * sizeof(double2), hipMemcpyHostToDevice, st));
        UpdTerm<T> t;
        t.ld = ld; t.col = 0; t.w = s_cur; t.M = coefY; t.ldm = s_cur;
        t.in = w.Z;
        update<T>(w.Z, ld, nc, 0, b, offP, false, 1, &t);
        // C V and B V only: C P and B P are formed afresh once P is
        // orthonormalised
        t.in = w.CZ;
        update<T>(w.CZ, ld, b, 0, b, offP, false, 1, &t);
        if (bexp()) {
            t.in = w.BZ;
            update<T>(w.BZ, ld, b, 0, b, offP, false, 1, &t);
        }
        pw = nc - b;
        eig_orthonormalise<T>();
        return;
    }
    small::SrrResult r;
    if (!small::harmonic_srr(K, Gm, sigma, b, nkeep, r)) throw singular();
    small_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    RA = r.RA; RB = r.RB; MA = r.MA; MB = r.MB;
    // coefficients: [Y_R | Y_P] (s_cur x nc), Y_L (s_cur x b), M1 = M_B, M2 = sigma M_B - M_A.
    // Y_P is Ybar_R(:, b+1:b+p) for the thick restart (eq. P1), or, for the
    // LOBPCG-style direction, the unit vectors that pick the active columns of
    // the current V, so that one row-local update produces V_new and P = V_old.
    int nc = r.ncols;
    size_t off = 0;
    std::memcpy(hpin + off, r.YR.data(), (size_t)s_cur * nc * sizeof(cd));
    if (lobpcg && p_cols > 0 && s_cur > b) {
        cd *ext = reinterpret_cast<cd *>(hpin) + (size_t)s_cur * nc;
        std::fill(ext, ext + (size_t)s_cur * p_cols, cd(0.0, 0.0));
        for (int j = 0; j < p_cols; ++j) ext[(size_t)j * s_cur + (b - p_cols) + j] = cd(1.0, 0.0);
        nc += p_cols;
    }
    off += (size_t)s_cur * nc;
    std::memcpy(hpin + off, r.YL.data(), (size_t)s_cur * b * sizeof(cd));
    off += (size_t)s_cur * b;
    Mat m2(b, b);
    for (int j = 0; j < b; ++j)
        for (int i = 0; i < b; ++i) m2(i, j) = sigma * MB(i, j) - MA(i, j);
    std::memcpy(hpin + off, MB.data(), (size_t)b * b * sizeof(cd));
    off += (size_t)b * b;
    std::memcpy(hpin + off, m2.data(), (size_t)b * b * sizeof(cd));
    off += (size_t)b * b;
    // one upload of the packed coefficients; M_B and sigma M_B - M_A stay in
    // cpack for the next iteration's residual blocks (M1c, M2c)
    GPLHR_HIP_CHECK(hipMemcpyAsync(cpack, hpin, off * sizeof(double2), hipMemcpyHostToDevice, st));
    const double2 *cY = cpack, *cL = cpack + (size_t)s_cur * nc;
    M1c = cL + (size_t)s_cur * b;
    M2c = M1c + (size_t)b * b;
    // a10: V = Z Y_R, P = Z Y_P (and the same for CZ, BZ); Q = U Y_L.  P lands
    // at its between-iterations slot smax - b.
    UpdTerm<T> t;
    t.ld = ld; t.col = 0; t.w = s_cur; t.M = cY; t.ldm = s_cur;
    t.in = w.Z;
    update<T>(w.Z, ld, nc, 0, b, offP, false, 1, &t);
    // C V and B V only: C P and B P are formed afresh once P is
    // orthonormalised
    t.in = w.CZ;
    update<T>(w.CZ, ld, b, 0, b, offP, false, 1, &t);
    if (bexp()) {
        t.in = w.BZ;
        update<T>(w.BZ, ld, b, 0, b, offP, false, 1, &t);
    }
    t.in = w.U; t.M = cL;
    update<T>(w.U, ld, b, 0, b, 0, false, 1, &t);
    // The host writes the pinned staging buffer again only after a stream
    // synchronisation, so the uploads above cannot be overtaken.
    pw = nc - b;
}

// The initialisation of Algorithm 2 from Z(:, 0:w0) (V0, or [V P] when restarting in
// another precision): orthonormalise, C Z, U = orth(C Z), ordered QZ, rotate.
// check_rank: reject a numerically rank-deficient V0 (BREAKDOWN).
template <typename T>
void Ctx::init_from_Z(int w0, bool check_rank) {
    Work<T> &w = W<T>();
    const int ld = smax;
    if (defl_k)
        for (int pass = 0; pass < 2; ++pass) deflate_right<T>(w.Z, ld, 0, w0);
    if (check_rank) {
        // The starting block must have numerically full column rank: a
        // vanishing pivot (at most 64 eps after diagonal scaling) in the first
        // Cholesky-QR pass means a column depends on the others to about
        // 1e-7 relative, and the shifted factor would fill it with rounding
        // noise.  The counter is zero before the first pass of a handle.
        cholqr<T>(w.Z, ld, 0, w0, 1, nullptr, nullptr);
        const int pivots = read_breakdowns();
        if (pivots > 0)
            throw Error(-4, "the starting block is rank deficient: its Cholesky-QR met " +
                                std::to_string(pivots) + " vanishing pivot(s)");
        cholqr<T>(w.Z, ld, 0, w0, 1, nullptr, nullptr);
    } else {
        cholqr<T>(w.Z, ld, 0, w0, 2, nullptr, nullptr);
    }
    for (int c = 0; c < w0; c += b) {
        const int wc = std::min(b, w0 - c);
        cprod<T>(w.Z + c, ld, w.CZ + c, ld, wc);
        bprod<T>(w.Z + c, ld, w.BZ + c, ld, wc);
    }
    launch_scale_rows<T>(st, n, w0, w.CZ, ld, nullptr, w.U, ld);
    cholqr<T>(w.U, ld, 0, w0, 2, nullptr, nullptr);
    srr_and_update<T>(w0, (w0 > b && opt.p_mode != GPLHR_P_NONE) ? b - q : 0);
}

// Algorithm 3 bookkeeping on the device: the new X in Z(:, 0:b) becomes
// X = V Rx with V orthonormal (two Cholesky-QR passes, mirrored onto C X and
// B X) and Rx scaled to unit-norm columns of X; Q = orth(C V), whose span is
// that of C X (Algorithm 3).
template <typename T>
void Ctx::eig_orthonormalise() {
    Work<T> &w = W<T>();
    const int ld = smax;
    T *bz = bexp() ? w.BZ : nullptr;
    const size_t bb = (size_t)b * b;
    for (int p = 0; p < 2; ++p) {
        gram<T>(w.Z, ld, b, w.Z, ld, b, nullptr, g0);
        launch_chol_rinv(st, b, g0, rinv, dstatus, g1 + p * bb);
        UpdTerm<T> t;
        t.ld = ld; t.col = 0; t.w = b; t.M = rinv; t.ldm = b; t.upper = true;
        t.in = w.Z;  update<T>(w.Z, ld, b, 0, b, 0, false, 1, &t);
        t.in = w.CZ; update<T>(w.CZ, ld, b, 0, b, 0, false, 1, &t);
        if (bz) { t.in = bz; update<T>(bz, ld, b, 0, b, 0, false, 1, &t); }
    }
    launch_scale_rows<T>(st, n, b, w.CZ, ld, nullptr, w.U, ld);
    cholqr<T>(w.U, ld, 0, b, 2, nullptr, nullptr);
    GPLHR_HIP_CHECK(hipMemcpyAsync(hpin, g1, 2 * bb * sizeof(double2), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    Mat r1(b, b), r2(b, b);
    std::memcpy(r1.data(), hpin, bb * sizeof(cd));
    std::memcpy(r2.data(), hpin + bb, bb * sizeof(cd));
    Rx = small::matmul(r2, r1);
    for (int j = 0; j < b; ++j) {
        double nrm = 0.0;
        for (int i = 0; i <= j; ++i) nrm += std::norm(Rx(i, j));
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) throw Error(-6, "vanishing or non-finite eigenvector approximation");
        for (int i = 0; i <= j; ++i) Rx(i, j) /= nrm;
    }
}

// The initialisation of Algorithm 3 from X = Z(:, 0:b) (X0, or the current X when the
// FP64 phase begins): C X (and B X), X = V Rx, Q = orth(C V); P empty.
template <typename T>
void Ctx::init_eig() {
    Work<T> &w = W<T>();
    if (defl_k)
        for (int pass = 0; pass < 2; ++pass) deflate_right<T>(w.Z, smax, 0, b);
    cprod<T>(w.Z, smax, w.CZ, smax, b);
    bprod<T>(w.Z, smax, w.BZ, smax, b);
    eig_orthonormalise<T>();
    pw = 0;
}

// One GPLHR iteration (one pass of the loop of Algorithm 2), with soft locking of the q
// leading columns when enabled.
template <typename T>
void Ctx::iterate_once() {
    Work<T> &w = W<T>();
    const int ld = smax;
    const int a = b - q;                       // active columns
    const int offW = b;
    const int pos = b + (m_cur + 1) * a;       // P slot of this iteration
    const int offPs = smax - b;                // P slot between iterations
    const int pa = std::min(pw, a);            // P columns used (first ones kept)
    const int s_cur = pos + pa;
    T *Z = w.Z, *CZ = w.CZ, *BZ = w.BZ, *U = w.U;
    // left projector basis: Q when B != I, V when B = I (eqs. prec_gen / prec)
    const T *Lb = (bk == B_IDENT) ? Z : U;
    const T *bsc = bscale<T>();

    // src block (width ws) -> new block of width a at dst:
    //   R = (A - sigma B) X M_B(., q:) + B X (sigma M_B - M_A)(., q:)   (moff selects
    //   the columns q: of M for X = V and the trailing a-by-a block for X = S_l;
    //   Algorithm 3 passes M_B = Rx Lambda_B, M_A = Rx Lambda_A for X = V and the
    //   diagonal Lambda_B, Lambda_A for S_l)
    //   R <- (I - Q Q^H) R;  Y = T R;  Y <- (I - [V W S_<l] [.]^H) Y (two passes)
    //   Y <- orth(Y);  C Y (and B Y)
    auto build = [&](int src, int ws, const double2 *m1, const double2 *m2, int moff, int dst) {
        UpdTerm<T> t[2];
        t[0].in = CZ; t[0].ld = ld; t[0].col = src; t[0].w = ws; t[0].M = m1 + moff; t[0].ldm = b;
        t[1].in = bexp() ? BZ : Z; t[1].ld = ld; t[1].col = src; t[1].w = ws;
        t[1].M = m2 + moff; t[1].ldm = b; t[1].rowscale = bsc;
        update<T>(w.R, b, a, 0, a, 0, false, 2, t);
        // The residual block of the Schur form needs no left projection when
        // B != I: every ordered QZ step leaves Q^H A V = R_A and Q^H B V = R_B,
        // and with G = R_A G1 + R_B G2 (eq. M) Q^H R = R_A M_B - R_B M_A = 0,
        // so (I - Q Q^H) R = R up to rounding of the size R carries anyway.
        // With B = I the left basis is V, for which this does not hold.
        const bool q_orthogonal = src == 0 && !eig && bk != B_IDENT && !defl_k;
        if (opt.proj_before_T && !q_orthogonal) project<T>(w.R, b, 0, a, Lb, ld, 0, b);
        apply_T<T>(Z, ld, dst, a);
        if (defl_k)
            for (int pass = 0; pass < 2; ++pass) deflate_right<T>(Z, ld, dst, a);
        proj_orth<T>(Z, ld, 0, dst, dst, a, 2);
        cprod<T>(Z + dst, ld, CZ + dst, ld, a);
        bprod<T>(Z + dst, ld, BZ + dst, ld, a);
    };
    const double2 *m1 = eig ? M1 : M1c, *m2 = eig ? M2 : M2c;
    build(0, b, m1, m2, q * b, offW);                                // W
    for (int l = 1; l <= m_cur; ++l)                                  // S_1 .. S_m
        build(offW + (l - 1) * a, a, eig ? M1s : m1, eig ? M2s : m2, q + q * b, offW + l * a);

    // P <- orth(P - [V W S][V W S]^H P), then C P (and B P)
    if (pa > 0) {
        T *bz = bexp() ? BZ : nullptr;
        if (pos != offPs) {
            // the layout is narrower than the kept one: move P next to S_mc
            // (row-local, so overlapping column ranges are safe)
            update<T>(Z, ld, pa, pos, pa, 0, false, 0, nullptr, Z + offPs, ld);
        }
        // the LOBPCG-style P (the previous V) lies almost inside span [V W S]
        // once V converges: its first pass is a plain projection, so it takes
        // a third one
        proj_orth<T>(Z, ld, 0, pos, pos, pa, opt.p_mode == GPLHR_P_LOBPCG ? 3 : 2);
        // C P (and B P) by fresh sparse products: one SpMM moves fewer bytes
        // than mirroring the four updates above onto C Z
        cprod<T>(Z + pos, ld, CZ + pos, ld, pa);
        bprod<T>(Z + pos, ld, BZ + pos, ld, pa);
    }
    // test basis U = [Q, orth((I - Q Q^H) C [W S P])].  First pass from
    // X = C [W S P]: the Grams Q^H X and X^H X into one (b + wq)-by-wq array,
    // the projected Cholesky factor, and U(:, b:) = X Rinv + Q Cy; the second
    // pass on U itself.
    const int wq = s_cur - b;
    {
        tbegin(T_GRAM);
        launch_gram<T>(st, n, U, ld, b, CZ + b, ld, wq, nullptr, part, PART_CAP, g0, b + wq);
        launch_gram<T>(st, n, CZ + b, ld, wq, CZ + b, ld, wq, nullptr, part, PART_CAP, g0 + b, b + wq);
        tend(T_GRAM);
        launch_chol_proj(st, b, wq, g0, rinv, g1, dstatus, true);
        UpdTerm<T> t[2];
        t[0].in = CZ; t[0].ld = ld; t[0].col = b; t[0].w = wq; t[0].M = rinv; t[0].ldm = wq;
        t[0].upper = true;
        t[1].in = U; t[1].ld = ld; t[1].col = 0; t[1].w = b; t[1].M = g1; t[1].ldm = b;
        update<T>(U, ld, wq, b, wq, 0, false, 2, t);
    }
    proj_orth<T>(U, ld, 0, b, b, wq, 1);
    // projected pencil, ordered Schur form, new V, Q, P (Section 3.5)
    srr_and_update<T>(s_cur, opt.p_mode == GPLHR_P_NONE ? 0 : a);
    ++n_iter;
    if (sizeof(T) == sizeof(double2)) ++n_iter64;
}

// Exact C V (and B V) by fresh sparse products: removes the drift of the
// mirrored products (C P and B P are always formed afresh once P is
// orthonormalised).
template <typename T>
void Ctx::refresh_products() {
    Work<T> &w = W<T>();
    cprod<T>(w.Z, smax, w.CZ, smax, b);
    bprod<T>(w.Z, smax, w.BZ, smax, b);
}

// Soft locking: q <- max(q, min(leading converged pairs, b - 1)) and the
// Krylov-Arnoldi depth that keeps the trial subspace at its size.
void Ctx::update_locking() {
    if (!opt.locking) { m_cur = m; return; }
    q = std::max(q, std::min(nlead, b - 1));
    m_cur = std::min((m * b) / (b - q), opt.m_max);
}

// Rayleigh-Ritz pairs on span(V) and their relative residuals (FP64).
template <typename T>
void Ctx::check() {
    Work<T> &w = W<T>();
    const int ld = smax;
    const T *bsrc = bexp() ? w.BZ : w.Z;
    const T *bsc = bscale<T>();
    // V^H C V and V^H B V side by side in g0, from one pass over V, so they
    // come back in one copy
    const size_t bb = (size_t)b * b;
    tbegin(T_GRAM);
    launch_gram2<T>(st, n, w.Z, ld, b, w.CZ, ld, b, bsrc, ld, b, bsc, part, PART_CAP, g0, b);
    tend(T_GRAM);
    GPLHR_HIP_CHECK(hipMemcpyAsync(hpin, g0, 2 * bb * sizeof(double2), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    Mat Va(b, b), Vb(b, b);
    std::memcpy(Va.data(), hpin, bb * sizeof(cd));
    std::memcpy(Vb.data(), hpin + bb, bb * sizeof(cd));
    for (size_t e = 0; e < bb; ++e) {
        Va.a[e] += sigma * Vb.a[e];
        if (!std::isfinite(Va.a[e].real()) || !std::isfinite(Va.a[e].imag()) ||
            !std::isfinite(Vb.a[e].real()) || !std::isfinite(Vb.a[e].imag()))
            throw Error(-6, "non-finite Rayleigh quotient matrices");
    }
    std::vector<cd> lam;
    Mat Zr;
    if (eig) {
        // Algorithm 3: x_j = V Rx(:, j); Lambda_A = diag(X^H A X), Lambda_B =
        // diag(X^H B X); lambda_j = Lambda_A(j,j) / Lambda_B(j,j).  The next
        // iteration's coefficients: Rx Lambda_B, Rx (sigma Lambda_B - Lambda_A)
        // for the residual, Lambda_B, sigma Lambda_B - Lambda_A for S.
        Zr = Rx;
        const Mat ax = small::matmul(Va, Rx), bx = small::matmul(Vb, Rx);
        alpha_h.assign(b, cd(0.0, 0.0));
        beta_h.assign(b, cd(0.0, 0.0));
        lam.assign(b, cd(0.0, 0.0));
        for (int j = 0; j < b; ++j) {
            for (int i = 0; i < b; ++i) {
                alpha_h[j] += std::conj(Rx(i, j)) * ax(i, j);
                beta_h[j] += std::conj(Rx(i, j)) * bx(i, j);
            }
            lam[j] = alpha_h[j] / beta_h[j];
            if (!std::isfinite(lam[j].real()) || !std::isfinite(lam[j].imag()))
                throw Error(-6, "Rayleigh quotient with x^H B x = 0");
        }
        cd *mh = reinterpret_cast<cd *>(hpin) + bb + 2 * b;
        std::fill(mh, mh + 4 * bb, cd(0.0, 0.0));
        for (int j = 0; j < b; ++j) {
            const cd m2d = sigma * beta_h[j] - alpha_h[j];
            for (int i = 0; i <= j; ++i) {
                mh[i + (size_t)j * b] = Rx(i, j) * beta_h[j];
                mh[bb + i + (size_t)j * b] = Rx(i, j) * m2d;
            }
            mh[2 * bb + j + (size_t)j * b] = beta_h[j];
            mh[3 * bb + j + (size_t)j * b] = m2d;
        }
        GPLHR_HIP_CHECK(hipMemcpyAsync(M1, mh, 4 * bb * sizeof(double2), hipMemcpyHostToDevice, st));
    } else {
        if (!small::ritz(Va, Vb, sigma, lam, Zr)) throw Error(-6, "Rayleigh-Ritz step failed");
    }
    lam_h = lam;
    Zr_h = Zr;
    // Zr and the eigenvalues in one upload (dZr holds both)
    std::memcpy(hpin, Zr.data(), bb * sizeof(cd));
    std::memcpy(hpin + bb, lam.data(), b * sizeof(cd));
    GPLHR_HIP_CHECK(hipMemcpyAsync(dZr, hpin, (bb + b) * sizeof(double2), hipMemcpyHostToDevice, st));
    const int nblk = launch_resid_partials<T>(st, n, b, w.CZ, ld, w.Z, ld,
                                              bexp() ? w.BZ : nullptr, ld, bsc,
                                              to_d2(sigma), dZr, dZr + bb, part, RESID_BLOCKS);
    launch_reduce_partials(st, part, nblk, b, 1, rnorm, b);
    GPLHR_HIP_CHECK(hipMemcpyAsync(hpin + bb + b, rnorm, b * sizeof(double2), hipMemcpyDeviceToHost, st));
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    rho_h.assign(b, 0.0);
    resid_h.assign(b, 0.0);
    max_rho = 0.0;
    nconv = 0;
    nlead = 0;
    bool lead = true, lead_all = true;
    for (int j = 0; j < b; ++j) {
        const cd v = reinterpret_cast<cd *>(hpin)[bb + b + j];
        resid_h[j] = std::sqrt(v.real());
        rho_h[j] = v.imag() > 0 ? std::sqrt(v.real() / v.imag()) : INFINITY;
        if (!std::isfinite(rho_h[j]) && v.imag() > 0) throw Error(-6, "non-finite residual");
        if (lead_all && rho_h[j] <= opt.tol) ++nlead;
        else lead_all = false;
        if (j < k) {
            max_rho = std::max(max_rho, rho_h[j]);
            if (lead && rho_h[j] <= opt.tol) ++nconv;
            else lead = false;
        }
    }
    history.push_back(max_rho);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
void Ctx::setup(const gplhr_csr *A, const gplhr_csr *B, cd sig, int k_, int b_,
                const gplhr_precond *T, const gplhr_options *o) {
    auto t0 = std::chrono::steady_clock::now();
    if (o) opt = *o; else gplhr_default_options(&opt);
    if (T) pre = *T; else { pre = gplhr_precond{}; pre.kind = GPLHR_PRECOND_NONE; }
    st = static_cast<hipStream_t>(opt.hip_stream);
    sigma = sig;
    if (!A || !A->row_ptr || !A->col_idx || !A->val) throw Error(-1, "A must be a device CSR");
    n = A->n;
    k = k_;
    b = b_;
    m = opt.arnoldi_m;
    m_cur = m;
    if (n < 1 || n > INT32_MAX - 1) throw Error(-1, "n out of range");
    if (A->nnz < 0 || A->nnz > INT32_MAX) throw Error(-1, "nnz(A) out of range");
    if (k < 1 || b < k) throw Error(-1, "need 1 <= k <= block");
    if (m < 1) throw Error(-1, "arnoldi_m must be >= 1");
    if (opt.locking && opt.m_max < m) throw Error(-1, "m_max must be >= arnoldi_m");
    if (opt.algorithm != GPLHR_ALG_SCHUR && opt.algorithm != GPLHR_ALG_EIG)
        throw Error(-1, "unknown algorithm");
    eig = (opt.algorithm == GPLHR_ALG_EIG);
    if (eig && opt.locking) throw Error(-1, "locking is available for the Schur form only");
    if (opt.p_mode != GPLHR_P_THICK && opt.p_mode != GPLHR_P_LOBPCG && opt.p_mode != GPLHR_P_NONE)
        throw Error(-1, "unsupported p_mode");
    if (opt.precision != GPLHR_FP64 && opt.precision != GPLHR_MIXED) throw Error(-1, "bad precision");
    smax = (m + 3) * b;
    if ((m + 2) * b > 48 || smax > 64)
        throw Error(-1, "(m+2)*block must be <= 48 and (m+3)*block <= 64");
    if (smax > n) throw Error(-1, "trial subspace (m+3)*block exceeds n");
    if (!(opt.tol >= 0.0)) throw Error(-1, "tol must be >= 0");
    if (pre.kind < 0 || pre.kind > GPLHR_PRECOND_GMRES) throw Error(-1, "unknown preconditioner");
    if (pre.kind == GPLHR_PRECOND_GMRES) {
        if (pre.inner < 0 || pre.inner >= GPLHR_PRECOND_GMRES)
            throw Error(-1, "GMRES inner preconditioner must be NONE, DIAG or JACOBI");
        if (pre.steps < 1 || pre.steps * b > 64) throw Error(-1, "GMRES needs 1 <= steps and steps * block <= 64");
    }
    // the basic preconditioner applied (T itself, or M inside block GMRES)
    const int ik = (pre.kind == GPLHR_PRECOND_GMRES) ? pre.inner : pre.kind;
    if (ik == GPLHR_PRECOND_JACOBI && (pre.sweeps < 1 || !(pre.omega > 0.0 && pre.omega < 2.0)))
        throw Error(-1, "Jacobi needs sweeps >= 1 and 0 < omega < 2");
    if (!std::isfinite(sigma.real()) || !std::isfinite(sigma.imag())) throw Error(-1, "sigma must be finite");

    // pinned staging for every small host <-> device transfer of the handle
    hpin_bytes = sizeof(double2) * 4 * 64 * 64 + 4096;
    hpin = static_cast<double2 *>(pinned_alloc(hpin_bytes));
    // row_ptr[0] and row_ptr[n] of a CSR, both read with one synchronisation
    auto row_ptr_ends = [&](const int32_t *rp, int32_t *ends) {
        int32_t *he = reinterpret_cast<int32_t *>(hpin);
        GPLHR_HIP_CHECK(hipMemcpyAsync(he, rp, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GPLHR_HIP_CHECK(hipMemcpyAsync(he + 1, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        ends[0] = he[0];
        ends[1] = he[1];
    };

    // A: validate and keep a copy (pattern + values) for the backward pass
    int32_t ends[2];
    row_ptr_ends(A->row_ptr, ends);
    if (ends[0] != 0 || ends[1] != A->nnz) throw Error(-1, "A: row_ptr[0] must be 0 and row_ptr[n] = nnz");
    int64_t bad_rows = 0, bad_vals = 0;
    csr_validate(st, n, A->row_ptr, A->col_idx, static_cast<const double2 *>(A->val), &bad_rows, &bad_vals);
    if (bad_rows) throw Error(-1, "A: " + std::to_string(bad_rows) + " rows with unsorted, duplicate or out-of-range columns");
    if (bad_vals) throw Error(-6, "A: non-finite values");
    a_nnz = A->nnz;
    dalloc(&a_rp, n + 1, st); dalloc(&a_ci, a_nnz, st); dalloc(&a_val, a_nnz, st);
    GPLHR_HIP_CHECK(hipMemcpyAsync(a_rp, A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
    GPLHR_HIP_CHECK(hipMemcpyAsync(a_ci, A->col_idx, sizeof(int32_t) * a_nnz, hipMemcpyDeviceToDevice, st));
    GPLHR_HIP_CHECK(hipMemcpyAsync(a_val, A->val, sizeof(double2) * a_nnz, hipMemcpyDeviceToDevice, st));

    bk = B_IDENT;
    if (B) {
        if (!B->row_ptr || !B->col_idx || !B->val) throw Error(-1, "B must be a device CSR");
        if (B->n != n) throw Error(-1, "A and B must have the same order");
        if (B->nnz < 0 || B->nnz > INT32_MAX) throw Error(-1, "nnz(B) out of range");
        row_ptr_ends(B->row_ptr, ends);
        if (ends[0] != 0 || ends[1] != B->nnz) throw Error(-1, "B: row_ptr[0] must be 0 and row_ptr[n] = nnz");
        csr_validate(st, n, B->row_ptr, B->col_idx, static_cast<const double2 *>(B->val), &bad_rows, &bad_vals);
        if (bad_rows) throw Error(-1, "B: " + std::to_string(bad_rows) + " malformed rows");
        if (bad_vals) throw Error(-6, "B: non-finite values");
        b_nnz = B->nnz;
        dalloc(&b_rp, n + 1, st); dalloc(&b_ci, b_nnz, st); dalloc(&b_val, b_nnz, st);
        GPLHR_HIP_CHECK(hipMemcpyAsync(b_rp, B->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
        GPLHR_HIP_CHECK(hipMemcpyAsync(b_ci, B->col_idx, sizeof(int32_t) * b_nnz, hipMemcpyDeviceToDevice, st));
        GPLHR_HIP_CHECK(hipMemcpyAsync(b_val, B->val, sizeof(double2) * b_nnz, hipMemcpyDeviceToDevice, st));
        const int64_t nondiag = csr_count_nondiag_rows(st, n, b_rp, b_ci);
        if (nondiag == 0) {
            bk = B_DIAG;
            dalloc(&bd, n, st);
            GPLHR_HIP_CHECK(hipMemcpyAsync(bd, b_val, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        } else {
            bk = B_SPARSE;
        }
    }
    // a1: C = A - sigma B on the union pattern, its diagonal, the preconditioner
    c_nnz = build_shifted(st, n, a_nnz, a_rp, a_ci, a_val, bk == B_IDENT ? 0 : 1, bk == B_DIAG,
                          b_rp, b_ci, b_val, to_d2(sigma), &c_rp, &c_ci, &c_val);
    c_plane = spmm_plane(st, n, c_rp, c_ci);
    if (bk == B_SPARSE) b_plane = spmm_plane(st, n, b_rp, b_ci);
    if (ik != GPLHR_PRECOND_NONE) {
        double2 *dg = nullptr;
        dalloc(&dg, n, st);
        const int64_t zeros = extract_diag(st, n, c_rp, c_ci, c_val, dg);
        if (zeros) {
            dfree(dg, st);
            throw Error(-5, "diag(A - sigma B) has " + std::to_string(zeros) + " zero entries");
        }
        dalloc(&dinv, n, st);
        launch_recip_scaled(st, n, dg, make_double2(1.0, 0.0), dinv);
        if (ik == GPLHR_PRECOND_JACOBI) {
            dalloc(&dw, n, st);
            launch_recip_scaled(st, n, dg, make_double2(pre.omega, 0.0), dw);
        }
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        dfree(dg, st);
    }
    mixed = (opt.precision == GPLHR_MIXED);
    phase = mixed ? 0 : 1;

    // workspace
    const size_t blk_s = (size_t)n * smax, blk_b = (size_t)n * b;
    wd.cval = c_val; wd.bval = b_val; wd.bd = bd; wd.dinv = dinv; wd.dw = dw;
    if (dw && pre.sweeps > 1) {
        dalloc(&cvdw, c_nnz, st);
        launch_scale_cols(st, c_nnz, c_ci, c_val, dw, cvdw);
        wd.cvdw = cvdw;
    }
    dalloc(&wd.Z, blk_s, st); dalloc(&wd.CZ, blk_s, st); dalloc(&wd.U, blk_s, st);
    defl_k = opt.defl_k;
    if (defl_k < 0 || defl_k > 64) throw Error(-1, "defl_k must be in [0, 64]");
    if (defl_k) {
        if (!opt.defl_V || (bk != B_IDENT && !opt.defl_Q))
            throw Error(-1, "deflation needs V1 (and Q1 when B != I)");
        if (defl_k + smax > n) throw Error(-1, "defl_k + (m+3)*block exceeds n");
        const void *q1 = (bk == B_IDENT) ? opt.defl_V : opt.defl_Q;
        dalloc(&wd.Vd, (size_t)n * defl_k, st);
        dalloc(&wd.Qd, (size_t)n * defl_k, st);
        GPLHR_HIP_CHECK(hipMemcpyAsync(wd.Vd, opt.defl_V, sizeof(double2) * n * defl_k, hipMemcpyDeviceToDevice, st));
        GPLHR_HIP_CHECK(hipMemcpyAsync(wd.Qd, q1, sizeof(double2) * n * defl_k, hipMemcpyDeviceToDevice, st));
    }
    if (bexp()) dalloc(&wd.BZ, blk_s, st);
    dalloc(&wd.R, blk_b, st);
    const bool jac2 = (ik == GPLHR_PRECOND_JACOBI && pre.sweeps > 1);
    const bool gm = (pre.kind == GPLHR_PRECOND_GMRES);
    const size_t blk_g = gm ? (size_t)n * (pre.steps + 1) * b : 0;
    if (jac2) { dalloc(&wd.J1, blk_b, st); dalloc(&wd.J2, blk_b, st); }
    if (gm) { dalloc(&wd.G, blk_g, st); dalloc(&wd.Gz, blk_b, st); dalloc(&wd.Gx, blk_b, st); }
    if (mixed) {
        dalloc(&c_val32, c_nnz, st);
        launch_c128_to_c64_flat(st, c_nnz, c_val, c_val32);
        wf.cval = c_val32;
        if (bk == B_SPARSE) { dalloc(&b_val32, b_nnz, st); launch_c128_to_c64_flat(st, b_nnz, b_val, b_val32); wf.bval = b_val32; }
        if (bk == B_DIAG) { dalloc(&bd32, n, st); launch_c128_to_c64_flat(st, n, bd, bd32); wf.bd = bd32; }
        if (dinv) { dalloc(&dinv32, n, st); launch_c128_to_c64_flat(st, n, dinv, dinv32); wf.dinv = dinv32; }
        if (dw) { dalloc(&dw32, n, st); launch_c128_to_c64_flat(st, n, dw, dw32); wf.dw = dw32; }
        if (cvdw) { dalloc(&cvdw32, c_nnz, st); launch_c128_to_c64_flat(st, c_nnz, cvdw, cvdw32); wf.cvdw = cvdw32; }
        dalloc(&wf.Z, blk_s, st); dalloc(&wf.CZ, blk_s, st); dalloc(&wf.U, blk_s, st);
        if (bexp()) dalloc(&wf.BZ, blk_s, st);
        if (defl_k) {
            dalloc(&wf.Vd, (size_t)n * defl_k, st);
            dalloc(&wf.Qd, (size_t)n * defl_k, st);
            launch_c128_to_c64_flat(st, (int64_t)n * defl_k, wd.Vd, wf.Vd);
            launch_c128_to_c64_flat(st, (int64_t)n * defl_k, wd.Qd, wf.Qd);
        }
        dalloc(&wf.R, blk_b, st);
        if (jac2) { dalloc(&wf.J1, blk_b, st); dalloc(&wf.J2, blk_b, st); }
        if (gm) { dalloc(&wf.G, blk_g, st); dalloc(&wf.Gz, blk_b, st); dalloc(&wf.Gx, blk_b, st); }
    }
    dalloc(&part, PART_CAP, st);
    dalloc(&g0, 64 * 64, st); dalloc(&g1, 64 * 64, st); dalloc(&rinv, 64 * 64, st);
    dalloc(&coefY, 64 * 64, st); dalloc(&cpack, 4 * 64 * 64, st);
    // M_B-type coefficient blocks of Algorithm 3, side by side (one upload)
    dalloc(&mbase, 4 * 64 * 64, st);
    M1 = mbase; M2 = M1 + (size_t)b * b; M1s = M2 + (size_t)b * b; M2s = M1s + (size_t)b * b;
    // [status | F1 | F2]: the breakdown counter and the projected pencil come
    // back in one copy
    dalloc(&fbase, 1 + 2 * 64 * 64, st);
    dstatus = reinterpret_cast<int *>(fbase);
    F1 = fbase + 1;
    dalloc(&dZr, 64 * 64 + 64, st); dalloc(&rnorm, 64, st);
    if (gm) {
        dalloc(&gmH, (size_t)(pre.steps + 1) * 4 * GM_SLOT, st);
        dalloc(&gmY, 64 * 16, st);
        hgm_bytes = sizeof(double2) * (pre.steps + 1) * 4 * GM_SLOT;
        hgm = static_cast<double2 *>(pinned_alloc(hgm_bytes));
    }
    GPLHR_HIP_CHECK(hipMemsetAsync(dstatus, 0, sizeof(int), st));

    // V0 -> Z(:, 0:b), then the initialisation of Algorithm 2
    if (opt.V0)
        GPLHR_HIP_CHECK(hipMemcpy2DAsync(wd.Z, smax * sizeof(double2), opt.V0, b * sizeof(double2),
                                         b * sizeof(double2), n, hipMemcpyDeviceToDevice, st));
    else
        launch_randn(st, n, b, opt.seed, wd.Z, smax);
    if (mixed) {
        launch_c128_to_c64(st, n, b, wd.Z, smax, wf.Z, smax);
        if (eig) init_eig<float2>(); else init_from_Z<float2>(b, true);
    } else {
        if (eig) init_eig<double2>(); else init_from_Z<double2>(b, true);
    }
    if (phase == 0) check<float2>(); else check<double2>();
    checked = true;
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void Ctx::switch_to_fp64() {
    const int offP = smax - b;
    launch_c64_to_c128(st, n, b, wf.Z, smax, wd.Z, smax);
    if (eig) {
        // restart Algorithm 3 from the current X = V Rx (P starts empty)
        std::memcpy(hpin, Rx.data(), (size_t)b * b * sizeof(cd));
        GPLHR_HIP_CHECK(hipMemcpyAsync(coefY, hpin, (size_t)b * b * sizeof(double2), hipMemcpyHostToDevice, st));
        UpdTerm<double2> t;
        t.in = wd.Z; t.ld = smax; t.col = 0; t.w = b; t.M = coefY; t.ldm = b;
        update<double2>(wd.Z, smax, b, 0, b, 0, false, 1, &t);
        phase = 1;
        init_eig<double2>();
        checked = false;
        return;
    }
    int w0 = b;
    if (pw > 0) {
        launch_c64_to_c128(st, n, pw, wf.Z + offP, smax, wd.Z + b, smax);
        w0 = b + pw;
    }
    phase = 1;
    init_from_Z<double2>(w0, false);
    checked = false;
}

int Ctx::run(int max_it) {
    auto t0 = std::chrono::steady_clock::now();
    if (max_it <= 0) max_it = opt.max_iter;
    int status = 1;
    int done = 0;
    double best = INFINITY;
    int since_best = 0;
    int since_refresh = 0;
    while (true) {
        if (!checked) {
            if (phase == 0) check<float2>(); else check<double2>();
            checked = true;
        }
        if (phase == 1 && max_rho <= opt.tol) {
            // confirm with freshly computed sparse products
            refresh_products<double2>();
            check<double2>();
            since_refresh = 0;
            if (max_rho <= opt.tol) { status = 0; converged = true; break; }
        }
        if (phase == 0) {
            if (max_rho < 0.9 * best) { best = max_rho; since_best = 0; }
            else ++since_best;
            if (max_rho <= opt.switch_tol || since_best >= opt.stall_window) {
                switch_to_fp64();
                continue;
            }
        }
        if (done >= max_it) break;
        update_locking();
        if (phase == 0) iterate_once<float2>(); else iterate_once<double2>();
        checked = false;
        ++done;
        if (phase == 1 && ++since_refresh >= REFRESH_EVERY) {
            refresh_products<double2>();
            since_refresh = 0;
            checked = false;
        }
    }
    tflush();
    iterate_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

// V, Q (n x k, ld k) in complex128
void Ctx::copy_out(void *V, void *Q) {
    if (phase == 0) {
        if (V) launch_c64_to_c128(st, n, k, wf.Z, smax, static_cast<double2 *>(V), k);
        if (Q) launch_c64_to_c128(st, n, k, wf.U, smax, static_cast<double2 *>(Q), k);
    } else {
        if (V) GPLHR_HIP_CHECK(hipMemcpy2DAsync(V, k * sizeof(double2), wd.Z, smax * sizeof(double2), k * sizeof(double2), n, hipMemcpyDeviceToDevice, st));
        if (Q) GPLHR_HIP_CHECK(hipMemcpy2DAsync(Q, k * sizeof(double2), wd.U, smax * sizeof(double2), k * sizeof(double2), n, hipMemcpyDeviceToDevice, st));
    }
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
}

// x_j = V z_j, j < k (n x k, ld k, complex128)
void Ctx::eigvecs(double2 *X) {
    const size_t bb = (size_t)b * b;
    GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    std::memcpy(hpin, Zr_h.data(), bb * sizeof(cd));
    GPLHR_HIP_CHECK(hipMemcpyAsync(dZr, hpin, bb * sizeof(double2), hipMemcpyHostToDevice, st));
    UpdTerm<double2> t;
    t.col = 0; t.w = b; t.M = dZr; t.ldm = b;
    if (phase == 0) {
        double2 *tmp = nullptr;
        dalloc(&tmp, (size_t)n * b, st);
        launch_c64_to_c128(st, n, b, wf.Z, smax, tmp, b);
        t.in = tmp; t.ld = b;
        launch_update<double2>(st, n, X, k, k, 0, k, 0, make_double2(0, 0), 1, &t);
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        dfree(tmp, st);
    } else {
        t.in = wd.Z; t.ld = smax;
        launch_update<double2>(st, n, X, k, k, 0, k, 0, make_double2(0, 0), 1, &t);
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
    }
}

// explicit instantiations
template void Ctx::iterate_once<double2>();
template void Ctx::iterate_once<float2>();
template void Ctx::update<double2>(double2 *, int, int, int, int, int, bool, int,
                                   const UpdTerm<double2> *, const double2 *, int);

}  // namespace gplhr
namespace gplhr {
template void Ctx::gram<double2>(const double2 *, int, int, const double2 *, int, int,
                                 const double2 *, double2 *);
template void Ctx::gram<float2>(const float2 *, int, int, const float2 *, int, int, const float2 *,
                                double2 *);
}  // namespace gplhr
