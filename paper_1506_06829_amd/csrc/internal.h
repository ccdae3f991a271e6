// Internal declarations shared by the HIP kernels, the driver and the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace gplhr {

// Status carried by exceptions inside the library; converted to gplhr_status
// at the C boundary.
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string &msg) : std::runtime_error(msg), status(st) {}
};

#define GPLHR_HIP_CHECK(expr)                                                               \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::gplhr::Error(-3, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

// Library workspace (memory.cpp): device memory through a cache of freed
// blocks (kept for later handles) and pinned host buffers from a free list.
// dev_free waits for the work queued on st before the block can be reused;
// pinned_free takes the size given to pinned_alloc.
void *dev_alloc(size_t bytes, hipStream_t st);
void dev_free(void *p, hipStream_t st);
void *pinned_alloc(size_t bytes);
void pinned_free(void *p, size_t bytes);

// ---------------------------------------------------------------------------
// kernel launchers (kernels.hip).  T is double2 (complex128) or float2
// (complex64).  All blocks are row-major with explicit leading dimensions.
// ---------------------------------------------------------------------------

// Y = C X (mode 0) or, for the damped Jacobi sweep, Y = X + dw .* (Rhs - C X)
// (mode 1), where dw holds omega / C(i,i) per row; mode 2 is the first two
// sweeps from zero, Y = w + dw .* (Rhs - C w) with w = dw .* Rhs, and takes X
// = Rhs (ldx = ldr) and in val the values of C diag(dw) (launch_scale_cols).  plane > 0 runs the rows
// in the plane-slab order (plane rows per plane; must divide n and be a
// multiple of 8), 0 in natural order; the result is the same.  nnz (the
// stored entries, rp[n]) sets how many entries of a row are gathered at once;
// any value >= 0 gives the same result.
template <typename T>
void launch_spmm(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci, const T *val,
                 const T *X, int ldx, T *Y, int ldy, int b, int mode, const T *Rhs, int ldr,
                 const T *dw, int plane, int64_t nnz);
// Plane for launch_spmm: the pattern's bandwidth max |j - i| when it splits
// n into at least four planes of at least 512 rows (a multiple of 8), else 0.
// Synchronous.
int spmm_plane(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci);

// G = X^H diag(yscale) Y (bx-by-by, FP64 accumulation, fixed reduction order)
// written column-major with leading dimension ldo.  yscale (complex per row)
// may be null.  `part` is scratch of part_cap complex128 entries.
template <typename T>
void launch_gram(hipStream_t st, int64_t n, const T *X, int ldx, int bx, const T *Y, int ldy,
                 int by, const T *yscale, double2 *part, size_t part_cap, double2 *out, int ldo);

// [X^H Y1, X^H diag(yscale2) Y2] (bx-by-(by1 + by2)) in one pass over X, the
// same kernels and reduction order as launch_gram; yscale2 may be null.
template <typename T>
void launch_gram2(hipStream_t st, int64_t n, const T *X, int ldx, int bx, const T *Y1, int ldy1,
                  int by1, const T *Y2, int ldy2, int by2, const T *yscale2, double2 *part,
                  size_t part_cap, double2 *out, int ldo);

// out[p + q*ldo] = sum_blk part[(p + q*bx) * nblk + blk]  (fixed order)
void launch_reduce_partials(hipStream_t st, const double2 *part, int nblk, int bx, int by,
                            double2 *out, int ldo);

// One term of a block update: alpha * diag(rowscale) * In(:, col:col+w) * M,
// M column-major w-by-wout (leading dimension ldm), FP64 complex.
template <typename T>
struct UpdTerm {
    const T *in = nullptr;
    int ld = 0;
    int col = 0;
    int w = 0;
    const double2 *M = nullptr;
    int ldm = 0;
    double2 alpha = {1.0, 0.0};
    const T *rowscale = nullptr;
    bool upper = false;   // M(k, j) = 0 for k > j (the caller guarantees it)
};

// Out(:, map(c)) = beta * Out(:, map(c)) + Add(:, c) + sum_t term_t(:, c),
// c < wout <= 48, with map(c) = ocol + c for c < split and ocol2 + (c - split)
// otherwise; Add (ld ldadd, first column at the pointer) may be null, and
// nterms may be 0 when it is not.  Row-local, so Out may alias any input.
template <typename T>
void launch_update(hipStream_t st, int64_t n, T *out, int ldo, int wout, int ocol, int split,
                   int ocol2, double2 beta, int nterms, const UpdTerm<T> *terms,
                   const T *add = nullptr, int ldadd = 0);

// Cholesky-QR factor: given the w-by-w Gram G (column-major, Hermitian),
// writes Rinv (column-major, upper triangular) with X Rinv orthonormal for
// X^H X = G, and, when Rout is not null, the factor R = Rinv^{-1} itself
// (G = R^H R).  Diagonal scaling first; a vanishing pivot triggers a diagonal
// shift and increments status[0].
void launch_chol_rinv(hipStream_t st, int w, const double2 *G, double2 *Rinv, int *status,
                      double2 *Rout = nullptr);
// Projected Cholesky-QR factor: G is [Y X]^H X ((wy + w)-by-w, column-major,
// leading dimension wy + w) for Y with orthonormal columns; with
// P = X^H X - (Y^H X)^H (Y^H X), the Gram of X - Y (Y^H X), writes Rinv
// (w-by-w) with P = R^H R as launch_chol_rinv does, and Cy = -(Y^H X) Rinv
// (wy-by-w, leading dimension wy), so that Y Cy + X Rinv is orthonormal and
// orthogonal to Y.  With guard set, when the projection cancels more than
// 1e-8 of a column's squared norm (X nearly inside span Y) the factor would be
// unreliable: Rinv is then the identity and Cy = -(Y^H X), a plain projection,
// and the next pass normalises (the last pass of a sequence runs without the
// guard).  w <= 48, wy <= 48, wy + w <= 64.
void launch_chol_proj(hipStream_t st, int wy, int w, const double2 *G, double2 *Rinv, double2 *Cy,
                      int *status, bool guard);

// Out(:, 0:w) = rowscale .* In(:, 0:w)  (rowscale complex per row; null = copy)
template <typename T>
void launch_scale_rows(hipStream_t st, int64_t n, int w, const T *in, int ldi, const T *rowscale,
                       T *out, int ldo);

// Y = X for row-major blocks of wv 16-byte vectors per row (leading
// dimensions in vectors), a streaming copy kernel.
void launch_block_copy(hipStream_t st, int64_t n, int wv, const void *X, int64_t ldx, void *Y,
                       int64_t ldy);

// Convert between precisions (w columns).
void launch_c128_to_c64(hipStream_t st, int64_t n, int w, const double2 *in, int ldi, float2 *out,
                        int ldo);
void launch_c64_to_c128(hipStream_t st, int64_t n, int w, const float2 *in, int ldi, double2 *out,
                        int ldo);
void launch_c128_to_c64_flat(hipStream_t st, int64_t cnt, const double2 *in, float2 *out);

// Residual partials for the Rayleigh-Ritz pairs (lambda_j, x_j = V z_j):
//   ax = (CV + sigma BV) z_j, bx = BV z_j, r = ax - lambda_j bx,
// accumulating (|r|^2, |ax|^2) per j in FP64.  BV is either an explicit block
// (bv, ldb) or V scaled by bscale (complex per row; null = identity).
template <typename T>
int launch_resid_partials(hipStream_t st, int64_t n, int b, const T *CV, int ldc, const T *V,
                          int ldv, const T *bv, int ldb, const T *bscale, double2 sigma,
                          const double2 *Zr, const double2 *lam, double2 *part, int max_blocks);

// Seeded complex normal block (counter-based hash + Box-Muller).
void launch_randn(hipStream_t st, int64_t n, int w, uint64_t seed, double2 *out, int ldo);

// --- setup --------------------------------------------------------------
// Count malformed rows of a CSR (unsorted/duplicate/out-of-range columns or
// decreasing row pointers) and non-finite values; returns (bad_rows, bad_vals).
void csr_validate(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci,
                  const double2 *val, int64_t *bad_rows, int64_t *bad_vals);
// Number of rows that are not exactly one stored diagonal entry.
int64_t csr_count_nondiag_rows(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci);

// Union-pattern C = A - sigma B.  bkind: 0 identity, 1 sparse (rp/ci/val of
// B); bdiag: B stores exactly its diagonal, one entry per row.  anz = nnz(A).
// Allocates rp/ci/val of C with dev_alloc on st and returns nnz(C).
int64_t build_shifted(hipStream_t st, int64_t n, int64_t anz, const int32_t *arp,
                      const int32_t *aci, const double2 *aval, int bkind, bool bdiag,
                      const int32_t *brp, const int32_t *bci, const double2 *bval,
                      double2 sigma, int32_t **crp, int32_t **cci, double2 **cval);
// d[i] = C(i,i) (0 when not stored); returns the number of zero diagonal entries.
int64_t extract_diag(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci,
                     const double2 *val, double2 *d);
// out[i] = num / d[i]
void launch_recip_scaled(hipStream_t st, int64_t n, const double2 *d, double2 num, double2 *out);
// Values of C diag(s) on C's pattern: out[e] = val[e] * s[ci[e]] (one rounding
// per entry), for the two-sweep Jacobi product (launch_spmm mode 2).
void launch_scale_cols(hipStream_t st, int64_t nnz, const int32_t *ci, const double2 *val,
                       const double2 *s, double2 *out);
// Conjugate transpose of a CSR (count / scan / scatter).  Allocates the result.
void csr_conj_transpose(hipStream_t st, int64_t n, int64_t nnz, const int32_t *rp,
                        const int32_t *ci, const double2 *val, int32_t **trp, int32_t **tci,
                        double2 **tval);
// grad[p] = sum_e coef_e * Y[i,e] * conj(X[j,e]) for each stored (i, j) = entry p.
void launch_sddmm(hipStream_t st, int64_t n, const int32_t *rp, const int32_t *ci, int k,
                  const double2 *Y, int ldy, const double2 *X, int ldx, const double2 *coef,
                  double2 *grad);

}  // namespace gplhr
