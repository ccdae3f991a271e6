// Host-side FP64 complex dense linear algebra for the s-by-s projected step of
// GPLHR (harmonic Schur-Rayleigh-Ritz, Section 3.3) and the k-by-k Rayleigh-Ritz
// convergence check.  All matrices are column-major std::complex<double>.
#pragma once
#include <complex>
#include <vector>

namespace gplhr {
namespace small {

using cd = std::complex<double>;

// Column-major dense matrix with leading dimension = rows.
struct Mat {
    int r = 0, c = 0;
    std::vector<cd> a;
    Mat() = default;
    Mat(int rows, int cols) : r(rows), c(cols), a((size_t)rows * cols, cd(0.0, 0.0)) {}
    cd &operator()(int i, int j) { return a[(size_t)i + (size_t)j * r]; }
    const cd &operator()(int i, int j) const { return a[(size_t)i + (size_t)j * r]; }
    cd *data() { return a.data(); }
    const cd *data() const { return a.data(); }
    static Mat eye(int n) {
        Mat m(n, n);
        for (int i = 0; i < n; ++i) m(i, i) = 1.0;
        return m;
    }
};

Mat matmul(const Mat &A, const Mat &B);                 // A B
Mat matmul_hn(const Mat &A, const Mat &B);              // A^H B

// X = K^{-1} N by Gaussian elimination with partial pivoting.  Returns false
// when a pivot vanishes relative to ||K||_max * n * eps.
bool lu_solve(const Mat &K, const Mat &N, Mat &X);

// Complex Schur form M = Y T Y^H (T upper triangular, Y unitary) by Householder
// reduction to Hessenberg form and single-shift implicit QR.  Returns false if
// the QR iteration does not converge.
bool schur(Mat &T, Mat &Y);

// Reorder a Schur form so that the first `nsel` diagonal entries are those of
// largest |T(j,j)|, in non-increasing order (ties keep their current order).
// Adjacent swaps by plane rotations; Y is updated so that M = Y T Y^H holds.
void reorder_desc_abs(Mat &T, Mat &Y, int nsel);

// Thin QR of X (rows >= cols): X = Qf R, Qf with orthonormal columns, R upper
// triangular with a positive real diagonal (Householder).
void qr_thin(const Mat &X, Mat &Qf, Mat &R);

// Eigen-decomposition of an upper-triangular T: columns of Vt are unit-norm
// eigenvectors (back substitution), T Vt = Vt diag(T).
Mat tri_eigvecs(const Mat &T);

struct SrrResult {
    Mat YR;      // s-by-2b (or s-by-b when s < 2b): ordered right Schur vectors
    Mat YL;      // s-by-b
    Mat RA, RB;  // b-by-b upper triangular
    Mat MA, MB;  // b-by-b, Q-free factors (Theorem 2.2, eq. M)
    int ncols = 0;  // columns of YR that were produced
};

// Ordered generalized Schur form of the projected pencil (F, G) = (U^H A Z,
// U^H B Z), given as K = U^H (A - sigma B) Z and Gm = U^H B Z.  Returns false
// when K is singular (sigma numerically an eigenvalue, Proposition 3.1).
bool harmonic_srr(const Mat &K, const Mat &Gm, std::complex<double> sigma, int b, int nkeep,
                  SrrResult &out);

// Projected eigenproblem of the eigenvector form (Algorithm 3): eigenvectors
// of (F, G) = (K + sigma Gm, Gm), ordered by |lambda - sigma| ascending; the
// first nkeep (at most s) are returned as columns of Ybar (unit norm).
// Returns false when K is singular.
bool harmonic_eig(const Mat &K, const Mat &Gm, int nkeep, Mat &Ybar);

// M_A, M_B from R_A, R_B with the diagonal G1, G2 of eqs. G1_fix / G2_fix.
void q_free_factors(const Mat &RA, const Mat &RB, Mat &MA, Mat &MB);

// Rayleigh-Ritz on span(V): eigenpairs of (Va, Vb) = (V^H A V, V^H B V),
// ordered by |lambda - sigma|; Zr holds unit-norm coefficient vectors.
bool ritz(const Mat &Va, const Mat &Vb, std::complex<double> sigma, std::vector<cd> &lam,
          Mat &Zr);

// Solve the upper-triangular system U X = B (back substitution).
Mat tri_solve_upper(const Mat &U, const Mat &B);

}  // namespace small
}  // namespace gplhr
