/*
 * gplhr.h -- C ABI of the MI355X (gfx950) GPLHR eigensolver library.
 *
 * GPLHR: Generalized Preconditioned Locally Harmonic Residual method
 * (Vecharynski, Yang, Xue, arXiv 1506.06829).  The library computes the k
 * eigenvalues of a regular pencil (A, B), A x = lambda B x (eq. gevp, Section 1),
 * that lie closest to a shift sigma, together with an orthonormal basis V of
 * right generalized Schur vectors, the left basis Q and the triangular factors
 * R_A, R_B of the partial generalized Schur form A V = Q R_A, B V = Q R_B
 * (eq. gschur, Section 2.1).  The iteration is Algorithm 2 ("The GPLHR
 * algorithm", Section 3.5) with the harmonic Schur-Rayleigh-Ritz extraction of
 * Section 3.3 and the thick-restart block P of Section 3.4 (eq. P1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved (re, im) pairs of IEEE doubles
 *   ("complex128") unless a signature says complex64 (pairs of floats).
 * - Dense n-by-w blocks on the device are ROW-MAJOR with a leading dimension
 *   (elements between consecutive rows) >= w.
 * - Small matrices on the host (k-by-k) are COLUMN-MAJOR complex128.
 * - Device pointers must come from hipMalloc (or a caching allocator on top
 *   of it) on the device that is current when gplhr_create is called.
 * - Every call returns a gplhr_status; nothing throws across the ABI.  A
 *   negative status is an error; the message is available from
 *   gplhr_last_error(handle) (or gplhr_last_error(NULL) for errors raised
 *   before a handle exists).
 * - A handle is not thread-safe; separate handles are independent.  All
 *   device work of a handle runs on the stream given in gplhr_options, which
 *   must outlive the handle.
 * - Workspace released by gplhr_destroy stays cached by the library for
 *   later handles (freeing device memory is slow) until the process ends.
 */
#ifndef GPLHR_H
#define GPLHR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gplhr_ctx *gplhr_t;

typedef enum {
    GPLHR_OK = 0,
    GPLHR_NOT_CONVERGED = 1,       /* status, not an error: results are readable */
    GPLHR_ERR_ARG = -1,            /* invalid argument or malformed CSR          */
    GPLHR_ERR_ALLOC = -2,          /* device or host allocation failed           */
    GPLHR_ERR_HIP = -3,            /* a HIP runtime call failed                  */
    GPLHR_ERR_BREAKDOWN = -4,      /* orthonormalisation could not be completed  */
    GPLHR_ERR_SINGULAR_SHIFT = -5, /* sigma is (numerically) an eigenvalue:
                                      A - sigma B or the projected pencil is
                                      singular (Proposition 3.1 fails)          */
    GPLHR_ERR_NUMERIC = -6,        /* NaN/Inf in inputs or iterates              */
    GPLHR_ERR_NOT_SIMPLE = -7,     /* backward: y^H B x ~ 0, lambda not simple   */
    GPLHR_ERR_STATE = -8           /* call not valid in the handle's state       */
} gplhr_status;

/* Square sparse matrix in CSR form, all arrays on the device.
 * row_ptr: n+1 int32, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz.
 * col_idx: nnz int32 in [0, n), strictly increasing within each row.
 * val:     nnz complex128.
 * The library copies what it needs during gplhr_create; the caller may free
 * the arrays afterwards. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const void *val;
} gplhr_csr;

/* Preconditioner T ~ (A - sigma B)^{-1} (Section 4; the paper only asks T to
 * approximate the inverse of the shifted operator).  C denotes A - sigma B. */
enum {
    GPLHR_PRECOND_NONE = 0,   /* T = I                                          */
    GPLHR_PRECOND_DIAG = 1,   /* T = diag(C)^{-1}                               */
    GPLHR_PRECOND_JACOBI = 2, /* `sweeps` damped Jacobi steps on C w = r from
                                 w_0 = 0: w_{t+1} = w_t + omega diag(C)^{-1}(r - C w_t) */
    GPLHR_PRECOND_GMRES = 3   /* the stronger T of Section 4: `steps` block GMRES
                                 steps on C W = R (all columns of the block at
                                 once) from W_0 = 0, right-preconditioned by
                                 `inner` (NONE, DIAG or JACOBI with sweeps,
                                 omega): W = M X with X in the block Krylov space
                                 of (C M, R) minimising ||R - C M X||_F          */
};
typedef struct {
    int kind;
    int sweeps;    /* JACOBI (also as the GMRES inner step): >= 1 */
    double omega;  /* JACOBI (also as the GMRES inner step): damping in (0, 2) */
    int steps;     /* GMRES only: block steps s >= 1 with s * block <= 64 */
    int inner;     /* GMRES only: the right preconditioner M (a kind < GMRES) */
} gplhr_precond;

enum { GPLHR_FP64 = 0, GPLHR_MIXED = 1 };
/* Additional search directions P (Section 3.4): thick restart P = Z Ybar_R(:, b+1:2b)
 * (eq. P1, the paper's default), the previous V (with the projections of P against
 * V, W and S in Algorithm 2 this spans the same space as the LOBPCG-style eq. P_lobpcg), or none. */
enum { GPLHR_P_THICK = 0, GPLHR_P_LOBPCG = 1, GPLHR_P_NONE = 2 };
/* Iterated form: Schur vectors (Algorithm 2, the default) or approximate
 * eigenvectors with Rayleigh-quotient eigenvalues (GPLHR-EIG, Algorithm 3 of
 * Appendix A). */
enum { GPLHR_ALG_SCHUR = 0, GPLHR_ALG_EIG = 1 };

typedef struct {
    int precision;      /* GPLHR_FP64: every block in complex128.
                           GPLHR_MIXED: sparse products, preconditioner and block
                           updates in complex64 with FP32 accumulation; Gram
                           matrices, Cholesky factors, the projected pencil and
                           residual norms in FP64; once the complex64 phase has
                           converged to switch_tol or stalls, the iteration
                           continues in complex128 from the current V and P
                           until tol is met.                                      */
    double tol;         /* stop when every one of the k leading Rayleigh-Ritz
                           pairs has ||A x - lambda B x|| / ||A x|| <= tol       */
    int max_iter;       /* iteration budget of gplhr_iterate when its max_iter<=0 */
    int arnoldi_m;      /* m of Algorithms 1-2: number of S blocks (>= 1)        */
    int p_mode;         /* GPLHR_P_THICK (eq. P1, default), GPLHR_P_LOBPCG or
                           GPLHR_P_NONE                                          */
    const void *V0;     /* device n-by-block complex128 row-major (ld = block),
                           or NULL: a seeded complex normal block               */
    uint64_t seed;      /* seed of the NULL-V0 generator                         */
    void *hip_stream;   /* hipStream_t; NULL = the null stream                   */
    double switch_tol;  /* MIXED: residual at which the FP64 phase starts        */
    int stall_window;   /* MIXED: also switch after this many iterations without
                           a 10% improvement of the largest residual              */
    int timing;         /* 1: time every kernel class with HIP events (adds a
                           small overhead); read with gplhr_get_stats            */
    int proj_before_T;  /* 1 (default): apply (I - QQ^H) (B = I: (I - VV^H))
                           before T as in eq. prec_gen; 0: omit it (the variant
                           compared in Table 3)                                  */
    int locking;        /* 1: soft locking (the remarks after Algorithm 2): once
                           the q leading Rayleigh-Ritz pairs meet tol (q never
                           decreases, q < block), V and Q keep all columns but
                           W, S_l and P are built for the a = block - q trailing
                           columns from the trailing a-by-a blocks of M_A, M_B,
                           and m grows to min(floor(arnoldi_m block / a), m_max)
                           so that the trial subspace keeps its size; 0 (default)
                           disables it                                           */
    int m_max;          /* upper bound of the adaptive m under locking (>= 1)    */
    int algorithm;      /* GPLHR_ALG_SCHUR (default) or GPLHR_ALG_EIG.  EIG keeps
                           X = V R_x (V orthonormal, unit-norm columns of X),
                           Lambda_A = diag(X^H A X), Lambda_B = diag(X^H B X),
                           builds W and S_l from A X Lambda_B - B X Lambda_A,
                           and takes X and P from the eigenvectors of the
                           projected pencil nearest sigma.  Not combined with
                           locking; in MIXED precision P restarts empty when the
                           FP64 phase begins                                     */
    /* Deflation (the remarks after Algorithm 2): with converged bases V1, Q1 of
     * k1 right/left generalized Schur vectors (for instance V and Q of an
     * earlier handle), iterate on the deflated pair
     * ((I - Q1 Q1^H) A (I - V1 V1^H), (I - Q1 Q1^H) B (I - V1 V1^H)), or on
     * (I - V1 V1^H) A (I - V1 V1^H) for B = I, to obtain further Schur
     * vectors.  The trial basis is kept orthogonal to V1 (V0 and every output
     * of T are projected).  Device n-by-defl_k complex128 row-major (ld =
     * defl_k) with orthonormal columns, copied during gplhr_create; defl_Q is
     * ignored for B = I.  0 <= defl_k <= 64; the backward pass is not
     * available for a deflated handle.                                          */
    const void *defl_V;
    const void *defl_Q;
    int defl_k;
} gplhr_options;

/* Fill *opt with defaults: FP64, tol 1e-10, max_iter 500, arnoldi_m 1, thick P,
 * V0 NULL, seed 1, null stream, switch_tol 1e-8, stall_window 3, timing 0,
 * proj_before_T 1, locking 0, m_max 20, algorithm SCHUR, no deflation. */
void gplhr_default_options(gplhr_options *opt);

/* Set up the operator C = A - sigma B on the union sparsity pattern, its
 * diagonal, the preconditioner and all device workspace, then run the
 * initialisation of Algorithm 2 (V = orth(V0), Q = orth(C V),
 * ordered QZ of (Q^H A V, Q^H B V), rotation of V and Q, M_A and M_B of
 * eq. M with G1, G2 of eqs. G1_fix, G2_fix).
 *
 * A      n-by-n CSR (device).
 * B      NULL for the standard problem B = I; otherwise n-by-n CSR (device).
 *        A B with exactly one stored entry per row on the diagonal is kept as
 *        a diagonal; any other B is applied as a sparse matrix.
 * sigma  shift sigma_re + i sigma_im; must not be an eigenvalue (Algorithm 2
 *        input; see also the caution that follows it).
 * k      number of wanted eigenpairs, 1 <= k <= block.
 * block  block width b of V, W, S_l, P (the paper uses b = k); the trial and
 *        test bases have s = (arnoldi_m + 3) b columns and s must not exceed n.
 * T      preconditioner (see gplhr_precond); NULL means GPLHR_PRECOND_NONE.
 * opt    NULL for defaults.
 * out    receives the handle (NULL on error).
 * Errors: ARG (sizes, malformed CSR, bad options), NUMERIC (non-finite
 * values), SINGULAR_SHIFT (zero on diag(C) with a diagonal-based T, or a
 * singular projected pencil), BREAKDOWN (Schur form: V0 is numerically rank
 * deficient, i.e. the Cholesky-QR of V0 meets a pivot of at most 64 eps of
 * its diagonally scaled Gram matrix -- a repeated, zero or dependent column),
 * ALLOC, HIP. */
gplhr_status gplhr_create(const gplhr_csr *A, const gplhr_csr *B,
                          double sigma_re, double sigma_im, int k, int block,
                          const gplhr_precond *T, const gplhr_options *opt,
                          gplhr_t *out);

/* Run GPLHR iterations (the main loop of Algorithm 2) until the convergence test
 * of gplhr_options.tol holds or max_iter iterations have run (max_iter <= 0:
 * use opt.max_iter).  n_converged (may be NULL) receives the number of leading
 * pairs that meet tol; max_rel_resid (may be NULL) the largest relative
 * residual over the k leading pairs.  Returns OK when converged,
 * NOT_CONVERGED when the budget ran out; may be called again to continue.
 * Inside the iteration a vanishing Cholesky pivot (a block that lost rank,
 * e.g. the residual columns of pairs that have converged exactly) is
 * shifted, the second Cholesky-QR pass orthonormalises what is left, and
 * gplhr_stats.breakdowns counts it; if the projected pencil of that
 * iteration is then singular the call returns BREAKDOWN (SINGULAR_SHIFT
 * when no pivot vanished).  Resume from saved Schur vectors by creating a
 * handle with V0 = V. */
gplhr_status gplhr_iterate(gplhr_t h, int max_iter, int *n_converged,
                           double *max_rel_resid);

/* Copy out the partial generalized Schur form (Algorithm 2 output).  STATE for
 * a handle created with GPLHR_ALG_EIG, which keeps no Schur factors.
 * V, Q    device n-by-k complex128, row-major, ld = k (either may be NULL).
 * RA, RB  host k-by-k complex128 column-major (either may be NULL).  For the
 *         standard problem RA receives R = M_B^{-1} M_A and RB the identity.
 * lambda  host k complex128: Rayleigh-Ritz eigenvalues on span(V), nearest
 *         sigma first (may be NULL).
 * rel_resid host k doubles: ||A x_j - lambda_j B x_j|| / ||A x_j|| (may be NULL).
 * Synchronises the handle's stream. */
gplhr_status gplhr_get_schur(gplhr_t h, void *V, void *Q, double *RA, double *RB,
                             double *lambda, double *rel_resid);

/* Residual norms ||A x_j - lambda_j B x_j|| / ||x_j|| of the k leading
 * eigenpairs of the last convergence check (host k doubles), in the order of
 * gplhr_get_schur's lambda (gplhr_get_eig's for GPLHR-EIG): the eigen-residual
 * of Section 5.1 measured against ||x_j|| instead of ||A x_j||.  The x_j have
 * unit norm (x_j = V z_j with orthonormal V and unit z_j; unit columns of X
 * for GPLHR-EIG).  Computed in FP64 from the current blocks (complex64 ones
 * during the complex64 phase).  Returns NOT_CONVERGED (results readable) when
 * the handle has not converged, STATE before any check. */
gplhr_status gplhr_get_residual_norms(gplhr_t h, double *resid);

/* Copy the unit-norm Rayleigh-Ritz eigenvectors x_j = V z_j (device n-by-k
 * complex128 row-major, ld = k), in the order of gplhr_get_schur's lambda. */
gplhr_status gplhr_get_eigvecs(gplhr_t h, void *X);

/* Copy out the partial eigendecomposition A X Lambda_B = B X Lambda_A that
 * GPLHR-EIG (Algorithm 3) iterates; STATE for an Algorithm 2 handle.
 * X        device n-by-k complex128 row-major, ld = k, unit-norm columns
 *          (may be NULL).
 * LA, LB   host k complex128 each: diag(X^H A X), diag(X^H B X); the
 *          eigenvalue approximations are LA[j] / LB[j] (either may be NULL).
 * rel_resid host k doubles: ||A x_j - lambda_j B x_j|| / ||A x_j|| (may be NULL).
 * Synchronises the handle's stream. */
gplhr_status gplhr_get_eig(gplhr_t h, void *X, double *LA, double *LB, double *rel_resid);

/* Gradient of a real loss L(lambda_1..lambda_k) with respect to the stored
 * values of A and B.  grad_lambda (host, k complex128) holds
 * dL/dRe(lambda_j) + i dL/dIm(lambda_j).  The left eigenvectors y_j come from
 * a GPLHR run on the adjoint pencil (A^H, B^H, conj(sigma)) with the same
 * options; for a simple eigenvalue, d lambda = (y^H dA x - lambda y^H dB x) /
 * (y^H B x), so each stored entry (i, j) receives
 *   grad_valA[p] = sum_e g_e y_e[i] conj(x_e[j]) / conj(y_e^H B x_e) and
 *   grad_valB[p] = -sum_e g_e conj(lambda_e) y_e[i] conj(x_e[j]) / conj(y_e^H B x_e)
 * (device, nnz(A) and nnz(B) complex128, overwritten; grad_valB may be NULL
 * and is ignored for B = I).  Requires a converged handle (STATE otherwise);
 * NOT_SIMPLE when |y^H B x| <= 1e-12 ||y|| ||B x||. */
gplhr_status gplhr_eig_backward(gplhr_t h, const double *grad_lambda,
                                void *grad_valA, void *grad_valB);

/* Counters and timers of a handle. */
typedef struct {
    int64_t iterations;        /* GPLHR iterations since create             */
    int64_t fp64_iterations;   /* of which in complex128                    */
    int64_t spmm_calls;        /* sparse-times-block launches               */
    int64_t precond_calls;     /* applications of T to a block              */
    int64_t breakdowns;        /* orthonormalisations that needed a shift   */
    double spmm_ms;            /* summed event time of SpMM launches (timing)*/
    double spmm_bytes;         /* algorithmic bytes of those launches        */
    double gram_ms;            /* Gram/reduction kernels (timing)           */
    double update_ms;          /* block update kernels (timing)             */
    double small_host_ms;      /* host projected-pencil step (wall clock)   */
    double setup_ms;           /* gplhr_create wall clock                   */
    double iterate_ms;         /* wall clock inside gplhr_iterate           */
    double max_rel_resid;      /* last convergence check                    */
    int n_converged;
    int phase;                 /* 0 = complex64 phase, 1 = complex128        */
    int locked;                /* q: leading columns locked (soft locking)  */
    int arnoldi_m;             /* m used by the last iteration              */
} gplhr_stats;

gplhr_status gplhr_get_stats(gplhr_t h, gplhr_stats *out);

/* Release the handle and all workspace it owns (waits for the handle's
 * stream; the device memory goes to the library's cache for later handles).
 * NULL is a no-op. */
void gplhr_destroy(gplhr_t h);

/* Message of the last error on h (or of the last failed create when h is
 * NULL).  Valid until the next call on the same handle. */
const char *gplhr_last_error(gplhr_t h);

/* ---------------------------------------------------------------------------
 * Single-kernel entry points (the building blocks of the iteration, exported
 * so that each can be checked and timed on its own).
 * ------------------------------------------------------------------------ */

/* Y = M X for a CSR matrix M and a dense row-major block X (sparse matrix
 * times block, the "matblock" product the paper relies on, Section 3.5 and
 * the remarks that follow Algorithm 2).  All pointers are device pointers.
 * val, X, Y are complex128 (dtype 0) or complex64 (dtype 1, FP32
 * accumulation).  X has ldx >= b, Y has ldy >= b, Y must not overlap X.
 * col_idx and val may be NULL only when every row is empty.  plane = 0 runs
 * the rows in natural order; plane > 0 (a divisor of n and a multiple of 8,
 * e.g. from gplhr_csr_plane) runs them plane by plane, each XCD of the GPU on
 * its own slab of every plane, for matrices whose couplings stay within
 * +-plane rows; the result is the same either way.  nnz is the number of
 * stored entries (row_ptr[n]); the kernel takes the entries of a row in
 * batches of 8, 12 or 17 by the typical row length nnz / n.  Only the speed
 * depends on it: any nnz >= 0 gives the same result.
 * Returns ARG for nnz < 0, b < 1 or b > 64, bad leading dimensions or a bad
 * plane. */
gplhr_status gplhr_spmm(int dtype, int64_t n, int64_t nnz, const int32_t *row_ptr,
                        const int32_t *col_idx, const void *val, const void *X,
                        int ldx, void *Y, int ldy, int b, int plane, void *hip_stream);

/* The plane the solver uses for a CSR pattern (device row_ptr / col_idx with
 * sorted columns): its bandwidth max |j - i| when that splits n into at least
 * four planes of at least 512 rows and is a multiple of 8, else 0.  Reads the
 * pattern once on hip_stream and waits for it. */
gplhr_status gplhr_csr_plane(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int *plane, void *hip_stream);

/* G = X^H Y in complex128 (FP64 accumulation, deterministic order) for
 * row-major X (n-by-bx, ldx) and Y (n-by-by, ldy) of dtype 0 (complex128) or
 * 1 (complex64).  G is a device bx-by-by complex128 array, column-major.
 * 1 <= bx, by <= 64.  Asynchronous on hip_stream.  The per-block partial sums
 * go to a buffer the library keeps for each (device, stream) pair until the
 * process ends (at most 64 MiB; growing it waits for the stream once). */
gplhr_status gplhr_gram(int dtype, int64_t n, const void *X, int ldx, int bx,
                        const void *Y, int ldy, int by, void *G, void *hip_stream);

/* Y(:, 0:w) = X(:, 0:w) for row-major device blocks, as a hand-written
 * streaming kernel (16-byte vector loads and stores, four in flight per
 * thread): the copy-out of the Schur vectors V, Q (Algorithm 2 output) is such
 * a block copy, and timing it on large blocks gives the HBM bandwidth a
 * kernel that reads and writes each byte once attains.  dtype 0: complex128;
 * 1: complex64 with even w and leading dimensions.  X and Y 16-byte aligned,
 * not overlapping.  Returns ARG otherwise. */
gplhr_status gplhr_block_copy(int dtype, int64_t n, const void *X, int ldx, void *Y, int ldy, int w,
                              void *hip_stream);

/* Z(:, wy:wy+w) <- orth((I - Y Y^H) Z(:, wy:wy+w)) for Y = Z(:, 0:wy) with
 * orthonormal columns (wy = 0: orthonormalisation alone): the block
 * Gram-Schmidt projection and orthonormalisation with which Algorithm 2 builds
 * its trial and test bases (Sections 3.3 to 3.5; the paper leaves the
 * orthonormalisation procedure open).  Each of `passes` passes (1..3) is one
 * FP64 Gram [Y X]^H X, the Cholesky factor R of the projected block's Gram
 * X^H X - (Y^H X)^H (Y^H X), and the row-local update
 * X <- (X - Y (Y^H X)) R^{-1}; all passes but the last only project a block
 * whose projection cancels almost all of a column.  Two passes give columns
 * orthonormal and orthogonal to Y to working precision when the projected
 * block is well conditioned; the result is then the Q of the QR factorisation
 * of (I - Y Y^H) X whose R has a positive real diagonal.  Z is a row-major
 * device block (ld >= wy + w) of dtype 0 (complex128) or 1 (complex64: FP32
 * products, FP64 Grams and factors); the solver's own kernels.  Allocates its
 * scratch on the stream and waits for the result before returning.
 * A column that lies in span(Y) to working precision is only projected by the
 * first pass and comes back, from the second, as a unit vector of its
 * rounding residual, orthogonal to Y and to the other columns.
 * 1 <= w <= 48, 0 <= wy <= 48, wy + w <= 64; returns ARG otherwise, and
 * BREAKDOWN when a Cholesky pivot of the projected block vanished (columns of
 * the block itself are linearly dependent to working precision; the columns
 * written are then not orthonormal). */
gplhr_status gplhr_proj_orth(int dtype, int64_t n, void *Z, int ld, int wy, int w, int passes,
                             void *hip_stream);

/* The same G = X^H Y as gplhr_gram, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): it calls no allocating routine.  Its partial sums go to a
 * 16 MiB array that the library keeps on each GPU until the process ends;
 * the per-block partials of any bx, by <= 64 fit there (the number of row
 * blocks is chosen so that they do).  Every call on one GPU shares that GPU's
 * array, so calls that overlap in time on one GPU (concurrent streams or
 * threads) race and give wrong results: serialise them.  Nothing in the array
 * needs to start at zero; every call writes the partials it reads.
 * Arguments, layout and errors as for gplhr_gram (ARG for widths outside
 * 1..64, bad leading dimensions or NULL pointers; HIP when the device
 * address of the array cannot be obtained).  The result agrees with
 * gplhr_gram's to rounding (the partial sums may be grouped in fewer row
 * blocks for the widest shapes). */
gplhr_status gplhr_gram_noalloc(int dtype, int64_t n, const void *X, int ldx, int bx,
                                const void *Y, int ldy, int by, void *G, void *hip_stream);

/* Y = T R for the damped Jacobi preconditioner on C: T approximates C^{-1}
 * for C = A - sigma B, as Section 4 asks of the preconditioner that Algorithm
 * 2 applies to the residual block and to each Krylov block.  From w_0 = 0,
 * sweeps steps of
 * w <- w + omega diag(C)^{-1} (R - C w) (the first one is omega diag(C)^{-1} R,
 * so sweeps - 1 sparse products); the same kernels as the solver's
 * GPLHR_PRECOND_JACOBI.  C is a device CSR (n, nnz, row_ptr, col_idx with
 * sorted columns) with complex128 values val; R (ldr >= b) and Y (ldy >= b)
 * are row-major device blocks of dtype 0 (complex128) or 1 (complex64: the
 * values and omega / diag(C) are rounded to complex64 and the products
 * accumulate in FP32, as in the solver's complex64 phase).  Y must not
 * overlap R.  plane as for gplhr_spmm.  Works in scratch blocks from the
 * library's device cache and waits for the result before returning.
 * Returns ARG for a bad size, b outside 1..64, sweeps outside 1..64,
 * omega <= 0 or non-finite, a bad plane, or a zero or missing diagonal entry. */
gplhr_status gplhr_jacobi(int dtype, int64_t n, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, const void *val, double omega, int sweeps,
                          const void *R, int ldr, void *Y, int ldy, int b, int plane,
                          void *hip_stream);

/* Y(:, 0:wy) = beta Y(:, 0:wy) + X(:, 0:wx) M, the row-local block update
 * behind every basis change of Algorithm 2: the new V, P and Q from the trial
 * and test bases and the ordered Schur vectors (Section 3.5), the projections
 * (I - QQ*) and (I - VV*) (Sections 3.3 and 3.4) and the Cholesky-QR
 * normalisations.  X (n-by-wx, ldx >= wx) and Y (n-by-wy, ldy >= wy) are
 * row-major device blocks of dtype 0 (complex128) or 1 (complex64, FP32
 * accumulation); M is a device complex128 wx-by-wy array, column-major with
 * leading dimension ldm >= wx.  Every row of X is read before the same row
 * of Y is written, so Y may be X itself (same pointer and ld).
 * 1 <= wx <= 128, 1 <= wy <= 48; returns ARG otherwise, and also when the
 * coefficients (about wx * wy complex values, padded) exceed the 64 KiB of
 * LDS the kernels stage them in. */
gplhr_status gplhr_block_update(int dtype, int64_t n, const void *X, int ldx, int wx,
                                const void *M, int ldm, void *Y, int ldy, int wy,
                                double beta_re, double beta_im, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* GPLHR_H */
