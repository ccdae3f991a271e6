// Host FP64 complex dense kernels for the projected (s-by-s) and Rayleigh-Ritz
// (k-by-k) steps of GPLHR.  Written from the textbook algorithms: Householder
// Hessenberg reduction, single-shift implicit QR with Wilkinson shifts, Schur
// reordering by adjacent plane-rotation swaps, Householder QR.
#include "small_dense.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>

namespace gplhr {
namespace small {

static inline double abs1(const cd &z) { return std::abs(z.real()) + std::abs(z.imag()); }

static inline cd unit_phase(const cd &z) {
    double a = std::abs(z);
    return a > 0.0 ? z / a : cd(1.0, 0.0);
}

Mat matmul(const Mat &A, const Mat &B) {
    Mat C(A.r, B.c);
    for (int j = 0; j < B.c; ++j)
        for (int l = 0; l < A.c; ++l) {
            const cd blj = B(l, j);
            if (blj == cd(0.0, 0.0)) continue;
            for (int i = 0; i < A.r; ++i) C(i, j) += A(i, l) * blj;
        }
    return C;
}

Mat matmul_hn(const Mat &A, const Mat &B) {
    Mat C(A.c, B.c);
    for (int j = 0; j < B.c; ++j)
        for (int i = 0; i < A.c; ++i) {
            cd acc(0.0, 0.0);
            for (int l = 0; l < A.r; ++l) acc += std::conj(A(l, i)) * B(l, j);
            C(i, j) = acc;
        }
    return C;
}

bool lu_solve(const Mat &Kin, const Mat &N, Mat &X) {
    const int n = Kin.r, nr = N.c;
    Mat K = Kin;
    X = N;
    double kmax2 = 0.0;
    for (const cd &v : K.a) kmax2 = std::max(kmax2, std::norm(v));
    const double kmax = std::sqrt(kmax2);
    if (!(kmax > 0.0) || !std::isfinite(kmax)) return false;
    const double tiny = kmax * n * DBL_EPSILON * 1e-3;
    // right-looking elimination with the multipliers stored in place; every
    // inner loop runs down a column (contiguous)
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = std::norm(K(j, j));
        for (int i = j + 1; i < n; ++i) {
            const double v = std::norm(K(i, j));
            if (v > best) { best = v; p = i; }
        }
        if (!(std::sqrt(best) > tiny)) return false;
        if (p != j) {
            for (int c = 0; c < n; ++c) std::swap(K(j, c), K(p, c));
            for (int c = 0; c < nr; ++c) std::swap(X(j, c), X(p, c));
        }
        const cd inv = 1.0 / K(j, j);
        cd *l = &K(0, j);
        for (int i = j + 1; i < n; ++i) l[i] *= inv;
        for (int c = j + 1; c < n; ++c) {
            const cd u = K(j, c);
            if (u == cd(0.0, 0.0)) continue;
            cd *kc = &K(0, c);
            for (int i = j + 1; i < n; ++i) kc[i] -= l[i] * u;
        }
        for (int c = 0; c < nr; ++c) {
            const cd u = X(j, c);
            if (u == cd(0.0, 0.0)) continue;
            cd *xc = &X(0, c);
            for (int i = j + 1; i < n; ++i) xc[i] -= l[i] * u;
        }
    }
    // back substitution, column by column of U
    for (int c = 0; c < nr; ++c) {
        cd *xc = &X(0, c);
        for (int i = n - 1; i >= 0; --i) {
            const cd v = xc[i] / K(i, i);
            xc[i] = v;
            const cd *ui = &K(0, i);
            for (int r = 0; r < i; ++r) xc[r] -= ui[r] * v;
        }
    }
    return true;
}

// Plane rotation G = [c s; -conj(s) c] (c real) with G [f; g] = [r; 0].
struct Rot {
    double c;
    cd s;
};

static Rot make_rot(const cd &f, const cd &g) {
    Rot R;
    const double sf = abs1(f), sg = abs1(g);
    if (sg == 0.0) {
        R.c = 1.0;
        R.s = 0.0;
        return R;
    }
    const double sc = std::max(sf, sg);
    if (!(sc > 1e-290 && sc < 1e290)) {
        // extreme magnitudes (or NaN): the library moduli, which scale inside
        if (sf == 0.0) {
            R.c = 0.0;
            R.s = std::conj(g) / std::abs(g);
        } else {
            const double af = std::abs(f), nrm = std::hypot(af, std::abs(g));
            R.c = af / nrm;
            R.s = (f / af) * std::conj(g) / nrm;
        }
        return R;
    }
    // scaled by the larger 1-norm, the squares neither overflow nor underflow
    // to zero; |f| and sqrt(|f|^2 + |g|^2) then take two square roots
    const double inv = 1.0 / sc;
    const cd fs = f * inv, gs = g * inv;
    const double f2 = std::norm(fs), g2 = std::norm(gs);
    if (f2 == 0.0) {
        // f = 0, or below 1e-154 |g|: the rotation that swaps up g
        R.c = 0.0;
        R.s = std::conj(gs) / std::sqrt(g2);
        return R;
    }
    const double af = std::sqrt(f2), nrm = std::sqrt(f2 + g2);
    R.c = af / nrm;
    R.s = fs * std::conj(gs) / (af * nrm);
    return R;
}

// rows p, q of M (columns c0..c1-1) <- G * rows
static inline void rot_rows(Mat &M, int p, int q, int c0, int c1, const Rot &G) {
    for (int j = c0; j < c1; ++j) {
        const cd x = M(p, j), y = M(q, j);
        M(p, j) = G.c * x + G.s * y;
        M(q, j) = -std::conj(G.s) * x + G.c * y;
    }
}

// columns p, q of M (rows r0..r1-1) <- cols * G^H
static inline void rot_cols(Mat &M, int p, int q, int r0, int r1, const Rot &G) {
    for (int i = r0; i < r1; ++i) {
        const cd x = M(i, p), y = M(i, q);
        M(i, p) = G.c * x + std::conj(G.s) * y;
        M(i, q) = -G.s * x + G.c * y;
    }
}

static void hessenberg(Mat &H, Mat &Y) {
    const int n = H.r;
    std::vector<cd> v(n), d(n), e(n);
    for (int j = 0; j + 2 < n; ++j) {
        double tail = 0.0;
        for (int i = j + 2; i < n; ++i) tail += std::norm(H(i, j));
        if (tail == 0.0) continue;
        const cd alpha = H(j + 1, j);
        const double xnorm = std::sqrt(std::norm(alpha) + tail);
        const cd beta = -unit_phase(alpha) * xnorm;
        double vn2 = 0.0;
        for (int i = j + 1; i < n; ++i) {
            v[i] = H(i, j);
            if (i == j + 1) v[i] -= beta;
            vn2 += std::norm(v[i]);
        }
        const double tau = 2.0 / vn2;
        // H <- (I - tau v v^H) H on rows j+1..n-1
        for (int c = j; c < n; ++c) {
            cd d(0.0, 0.0);
            for (int i = j + 1; i < n; ++i) d += std::conj(v[i]) * H(i, c);
            d *= tau;
            for (int i = j + 1; i < n; ++i) H(i, c) -= v[i] * d;
        }
        // H <- H (I - tau v v^H), Y <- Y (I - tau v v^H) on columns j+1..n-1
        // (row sums accumulated column by column: contiguous in memory)
        std::fill(d.begin(), d.end(), cd(0.0, 0.0));
        std::fill(e.begin(), e.end(), cd(0.0, 0.0));
        for (int i = j + 1; i < n; ++i) {
            const cd vi = v[i];
            const cd *hc = &H(0, i), *yc = &Y(0, i);
            for (int r = 0; r < n; ++r) {
                d[r] += hc[r] * vi;
                e[r] += yc[r] * vi;
            }
        }
        for (int r = 0; r < n; ++r) {
            d[r] *= tau;
            e[r] *= tau;
        }
        for (int i = j + 1; i < n; ++i) {
            const cd cv = std::conj(v[i]);
            cd *hc = &H(0, i), *yc = &Y(0, i);
            for (int r = 0; r < n; ++r) {
                hc[r] -= d[r] * cv;
                yc[r] -= e[r] * cv;
            }
        }
        H(j + 1, j) = beta;
        for (int i = j + 2; i < n; ++i) H(i, j) = 0.0;
    }
}

bool schur(Mat &T, Mat &Y) {
    const int n = T.r;
    Y = Mat::eye(n);
    if (n == 1) return std::isfinite(std::abs(T(0, 0)));
    hessenberg(T, Y);
    double hnorm = 0.0;
    for (const cd &v : T.a) hnorm = std::max(hnorm, abs1(v));
    if (!std::isfinite(hnorm)) return false;
    if (hnorm == 0.0) return true;
    const double eps = DBL_EPSILON;
    int ihi = n - 1;
    int its = 0, total = 0;
    const int max_total = 40 * n;
    while (ihi > 0) {
        int l = ihi;
        for (; l > 0; --l) {
            double s = abs1(T(l, l)) + abs1(T(l - 1, l - 1));
            if (s == 0.0) s = hnorm;
            if (abs1(T(l, l - 1)) <= eps * s) {
                T(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == ihi) {
            --ihi;
            its = 0;
            continue;
        }
        if (++total > max_total) return false;
        ++its;
        cd mu;
        if (its % 11 == 0) {
            // exceptional shift
            const double h = abs1(T(ihi, ihi - 1)) + (ihi >= 2 ? abs1(T(ihi - 1, ihi - 2)) : 0.0);
            mu = T(ihi, ihi) + cd(0.75 * h, -0.4375 * h);
        } else {
            const cd a = T(ihi - 1, ihi - 1), b = T(ihi - 1, ihi), c = T(ihi, ihi - 1),
                     d = T(ihi, ihi);
            const cd p = 0.5 * (a - d);
            const cd disc = std::sqrt(p * p + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = (std::abs(m1 - d) <= std::abs(m2 - d)) ? m1 : m2;
        }
        // implicit single-shift QR sweep on the active block l..ihi
        Rot G = make_rot(T(l, l) - mu, T(l + 1, l));
        rot_rows(T, l, l + 1, l, n, G);
        rot_cols(T, l, l + 1, 0, std::min(l + 3, ihi + 1), G);
        rot_cols(Y, l, l + 1, 0, n, G);
        for (int j = l; j + 2 <= ihi; ++j) {
            G = make_rot(T(j + 1, j), T(j + 2, j));
            rot_rows(T, j + 1, j + 2, j, n, G);
            T(j + 2, j) = 0.0;
            rot_cols(T, j + 1, j + 2, 0, std::min(j + 4, ihi + 1), G);
            rot_cols(Y, j + 1, j + 2, 0, n, G);
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) T(i, j) = 0.0;
    return true;
}

static void swap_adjacent(Mat &T, Mat &Y, int k) {
    const int n = T.r;
    const cd t11 = T(k, k), t22 = T(k + 1, k + 1);
    const cd f = T(k, k + 1), g = t22 - t11;
    if (f == cd(0.0, 0.0) && g == cd(0.0, 0.0)) return;
    const Rot G = make_rot(f, g);
    rot_rows(T, k, k + 1, k, n, G);
    rot_cols(T, k, k + 1, 0, k + 2, G);
    rot_cols(Y, k, k + 1, 0, n, G);
    T(k, k) = t22;
    T(k + 1, k + 1) = t11;
    T(k + 1, k) = 0.0;
}

void reorder_desc_abs(Mat &T, Mat &Y, int nsel) {
    const int n = T.r;
    nsel = std::min(nsel, n);
    for (int pos = 0; pos < nsel; ++pos) {
        int best = pos;
        double bv = std::abs(T(pos, pos));
        for (int j = pos + 1; j < n; ++j) {
            const double v = std::abs(T(j, j));
            if (v > bv) { bv = v; best = j; }
        }
        for (int j = best - 1; j >= pos; --j) swap_adjacent(T, Y, j);
    }
}

void qr_thin(const Mat &Xin, Mat &Qf, Mat &R) {
    const int m = Xin.r, n = Xin.c;
    Mat X = Xin;
    std::vector<std::vector<cd>> vs(n);
    std::vector<double> taus(n, 0.0);
    R = Mat(n, n);
    for (int j = 0; j < n; ++j) {
        double xn2 = 0.0;
        for (int i = j; i < m; ++i) xn2 += std::norm(X(i, j));
        const cd alpha = X(j, j);
        const double xnorm = std::sqrt(xn2);
        std::vector<cd> v(m, cd(0.0, 0.0));
        cd beta = alpha;
        if (xnorm > 0.0) {
            beta = -unit_phase(alpha) * xnorm;
            double vn2 = 0.0;
            for (int i = j; i < m; ++i) {
                v[i] = X(i, j);
                if (i == j) v[i] -= beta;
                vn2 += std::norm(v[i]);
            }
            if (vn2 > 0.0) {
                const double tau = 2.0 / vn2;
                taus[j] = tau;
                for (int c = j + 1; c < n; ++c) {
                    cd d(0.0, 0.0);
                    for (int i = j; i < m; ++i) d += std::conj(v[i]) * X(i, c);
                    d *= tau;
                    for (int i = j; i < m; ++i) X(i, c) -= v[i] * d;
                }
            }
        }
        X(j, j) = beta;
        for (int i = j + 1; i < m; ++i) X(i, j) = 0.0;
        vs[j] = std::move(v);
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) R(i, j) = X(i, j);
    Qf = Mat(m, n);
    for (int j = 0; j < n; ++j) Qf(j, j) = 1.0;
    for (int j = n - 1; j >= 0; --j) {
        if (taus[j] == 0.0) continue;
        const std::vector<cd> &v = vs[j];
        for (int c = 0; c < n; ++c) {
            cd d(0.0, 0.0);
            for (int i = j; i < m; ++i) d += std::conj(v[i]) * Qf(i, c);
            d *= taus[j];
            for (int i = j; i < m; ++i) Qf(i, c) -= v[i] * d;
        }
    }
    // positive real diagonal of R
    for (int j = 0; j < n; ++j) {
        const cd th = unit_phase(R(j, j));
        for (int i = 0; i < m; ++i) Qf(i, j) *= th;
        for (int c = j; c < n; ++c) R(j, c) *= std::conj(th);
        R(j, j) = cd(R(j, j).real(), 0.0);
    }
}

Mat tri_eigvecs(const Mat &T) {
    const int n = T.r;
    double tmax = 0.0;
    for (const cd &v : T.a) tmax = std::max(tmax, std::abs(v));
    const double smin = std::max(DBL_EPSILON * tmax, 1e-300);
    Mat V(n, n);
    for (int j = 0; j < n; ++j) {
        V(j, j) = 1.0;
        for (int i = j - 1; i >= 0; --i) {
            cd acc(0.0, 0.0);
            for (int l = i + 1; l <= j; ++l) acc += T(i, l) * V(l, j);
            cd d = T(i, i) - T(j, j);
            if (std::abs(d) < smin) d = smin;
            V(i, j) = -acc / d;
        }
        double nrm = 0.0;
        for (int i = 0; i <= j; ++i) nrm += std::norm(V(i, j));
        nrm = std::sqrt(nrm);
        for (int i = 0; i <= j; ++i) V(i, j) /= nrm;
    }
    return V;
}

bool harmonic_eig(const Mat &K, const Mat &Gm, int nkeep, Mat &Ybar) {
    const int s = K.r;
    // eigenvectors of (K + sigma Gm, Gm) are those of M = K^{-1} Gm, with
    // eigenvalues 1/(lambda - sigma): order by |.| descending in the Schur form
    // and take the eigenvectors of its leading triangular block
    Mat M;
    if (!lu_solve(K, Gm, M)) return false;
    Mat Y;
    if (!schur(M, Y)) return false;
    const int nc = std::min(nkeep, s);
    reorder_desc_abs(M, Y, nc);
    Mat Tl(nc, nc);
    for (int j = 0; j < nc; ++j)
        for (int i = 0; i <= j; ++i) Tl(i, j) = M(i, j);
    const Mat E = tri_eigvecs(Tl);
    Ybar = Mat(s, nc);
    for (int j = 0; j < nc; ++j)
        for (int l = 0; l <= j; ++l) {
            const cd e = E(l, j);
            for (int i = 0; i < s; ++i) Ybar(i, j) += Y(i, l) * e;
        }
    for (const cd &v : Ybar.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
    return true;
}

Mat tri_solve_upper(const Mat &U, const Mat &B) {
    const int n = U.r;
    Mat X = B;
    for (int c = 0; c < X.c; ++c)
        for (int i = n - 1; i >= 0; --i) {
            cd acc = X(i, c);
            for (int l = i + 1; l < n; ++l) acc -= U(i, l) * X(l, c);
            X(i, c) = acc / U(i, i);
        }
    return X;
}

void q_free_factors(const Mat &RA, const Mat &RB, Mat &MA, Mat &MB) {
    const int k = RA.r;
    std::vector<cd> g1(k), g2(k);
    for (int j = 0; j < k; ++j) {
        const cd a = RA(j, j), b = RB(j, j);
        if (std::abs(a) < std::abs(b)) {
            g1[j] = 0.0;
            g2[j] = 1.0 / b;
        } else {
            g1[j] = (1.0 - b) / a;
            g2[j] = 1.0;
        }
    }
    Mat G(k, k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i <= j; ++i) G(i, j) = RA(i, j) * g1[j] + RB(i, j) * g2[j];
    const Mat X = tri_solve_upper(G, RA);  // G^{-1} R_A
    MA = Mat(k, k);
    MB = Mat(k, k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) {
            MA(i, j) = g2[i] * X(i, j);
            MB(i, j) = (i == j ? cd(1.0, 0.0) : cd(0.0, 0.0)) - g1[i] * X(i, j);
        }
}

bool harmonic_srr(const Mat &K, const Mat &Gm, std::complex<double> sigma, int b, int nkeep,
                  SrrResult &out) {
    const int s = K.r;
    // Proposition 3.1: K = U^H (A - sigma B) Z is nonsingular, so the ordered
    // generalized Schur form of (K + sigma Gm, Gm) follows from the Schur form
    // of M = K^{-1} Gm, whose eigenvalues are 1/(lambda - sigma).
    Mat M;
    if (!lu_solve(K, Gm, M)) return false;
    Mat Y;
    if (!schur(M, Y)) return false;
    const int ncols = std::min(nkeep, s);
    reorder_desc_abs(M, Y, ncols);
    // K Y(:,1:b) = Y_L R_C  with R_C = R_A - sigma R_B
    Mat KY1(s, b);
    {
        Mat Y1(s, b);
        for (int j = 0; j < b; ++j)
            for (int i = 0; i < s; ++i) Y1(i, j) = Y(i, j);
        KY1 = matmul(K, Y1);
    }
    Mat RC;
    qr_thin(KY1, out.YL, RC);
    Mat Tb(b, b);
    for (int j = 0; j < b; ++j)
        for (int i = 0; i <= j; ++i) Tb(i, j) = M(i, j);
    out.RB = matmul(RC, Tb);
    out.RA = Mat(b, b);
    for (int j = 0; j < b; ++j)
        for (int i = 0; i < b; ++i) out.RA(i, j) = RC(i, j) + sigma * out.RB(i, j);
    // Normalise the unimodular freedom of Y_L: R_B gets a real non-negative
    // diagonal (R_A a positive one where R_B(j,j) = 0), so that M_B -> I for
    // B = I.
    for (int j = 0; j < b; ++j) {
        const cd d = out.RB(j, j);
        const cd th = std::abs(d) > 0.0 ? unit_phase(d) : unit_phase(out.RA(j, j));
        for (int i = 0; i < s; ++i) out.YL(i, j) *= th;
        for (int c = 0; c < b; ++c) {
            out.RA(j, c) *= std::conj(th);
            out.RB(j, c) *= std::conj(th);
        }
    }
    out.YR = Mat(s, ncols);
    for (int j = 0; j < ncols; ++j)
        for (int i = 0; i < s; ++i) out.YR(i, j) = Y(i, j);
    out.ncols = ncols;
    q_free_factors(out.RA, out.RB, out.MA, out.MB);
    for (const cd &v : out.MA.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
    for (const cd &v : out.MB.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
    return true;
}

bool ritz(const Mat &Va, const Mat &Vb, std::complex<double> sigma, std::vector<cd> &lam,
          Mat &Zr) {
    const int k = Va.r;
    Mat M;
    if (!lu_solve(Vb, Va, M)) return false;
    Mat Y;
    if (!schur(M, Y)) return false;
    const Mat Vt = tri_eigvecs(M);
    const Mat Z = matmul(Y, Vt);
    std::vector<int> idx(k);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<double> dist(k);
    for (int j = 0; j < k; ++j) dist[j] = std::abs(M(j, j) - sigma);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return dist[a] < dist[b]; });
    lam.assign(k, cd(0.0, 0.0));
    Zr = Mat(k, k);
    for (int j = 0; j < k; ++j) {
        const int src = idx[j];
        lam[j] = M(src, src);
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += std::norm(Z(i, src));
        nrm = std::sqrt(nrm);
        for (int i = 0; i < k; ++i) Zr(i, j) = Z(i, src) / nrm;
    }
    return true;
}

}  // namespace small
}  // namespace gplhr
