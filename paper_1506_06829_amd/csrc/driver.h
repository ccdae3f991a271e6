// GPLHR solver context (one per handle).
#pragma once
#include <complex>
#include <map>
#include <utility>
#include <vector>

#include "../../include/gplhr.h"
#include "internal.h"
#include "small_dense.h"

namespace gplhr {

using cd = std::complex<double>;

enum BKind { B_IDENT = 0, B_DIAG = 1, B_SPARSE = 2 };

// Per-precision operator views and block workspace.
template <typename T>
struct Work {
    const T *cval = nullptr;   // values of C = A - sigma B
    const T *bval = nullptr;   // values of a sparse B
    const T *bd = nullptr;     // diagonal of a diagonal B
    const T *dinv = nullptr;   // 1 / diag(C)
    const T *dw = nullptr;     // omega / diag(C)
    const T *cvdw = nullptr;   // values of C diag(omega / diag(C)) (two Jacobi sweeps in one pass)
    T *Z = nullptr, *CZ = nullptr, *BZ = nullptr, *U = nullptr;   // n x smax
    T *R = nullptr, *J1 = nullptr, *J2 = nullptr;                  // n x b
    T *G = nullptr;                    // block GMRES basis, n x (steps+1) b
    T *Vd = nullptr, *Qd = nullptr;    // deflation bases, n x defl_k
    T *Gz = nullptr, *Gx = nullptr;    // block GMRES temporaries, n x b
};

struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    int used = 0;
    double ms = 0.0;
    int64_t count = 0;
};

enum { T_SPMM = 0, T_GRAM = 1, T_UPDATE = 2 };

struct Ctx {
    static constexpr size_t PART_CAP = (size_t)1024 * 64 * 64;   // complex128 scratch entries
    static constexpr int RESID_BLOCKS = 1024;
    static constexpr int REFRESH_EVERY = 20;
    static constexpr size_t GM_SLOT = 64 * 16;   // entries per block GMRES small factor

    std::string err;
    hipStream_t st = nullptr;
    gplhr_options opt{};
    gplhr_precond pre{};
    int64_t n = 0;
    // m: Krylov-Arnoldi depth requested; m_cur: depth of the current
    // iteration (grows under locking); q: locked leading columns; pw: width of
    // the P block kept at columns smax - b .. between iterations (0: none)
    int k = 0, b = 0, m = 1, smax = 0, m_cur = 1, q = 0, pw = 0;
    cd sigma;
    BKind bk = B_IDENT;
    bool mixed = false;
    int c_plane = 0, b_plane = 0;   // SpMM row schedules of C and B
    bool eig = false;   // GPLHR-EIG (Algorithm 3) instead of the Schur form
    int defl_k = 0;     // columns of the deflation bases (0: no deflation)
    // B Z kept as an explicit block (general sparse B, or any B != I under
    // deflation); otherwise B Z is Z or diag(B) Z formed on the fly
    bool bexp() const { return bk == B_SPARSE || (defl_k > 0 && bk == B_DIAG); }
    template <typename T> const T *bscale() { return (bk == B_DIAG && !bexp()) ? W<T>().bd : nullptr; }
    int phase = 1;
    bool converged = false, checked = false;

    // operator
    int32_t *c_rp = nullptr, *c_ci = nullptr;
    double2 *c_val = nullptr;
    float2 *c_val32 = nullptr;
    int64_t c_nnz = 0;
    int32_t *a_rp = nullptr, *a_ci = nullptr;
    double2 *a_val = nullptr;
    int64_t a_nnz = 0;
    int32_t *b_rp = nullptr, *b_ci = nullptr;
    double2 *b_val = nullptr;
    float2 *b_val32 = nullptr;
    int64_t b_nnz = 0;
    double2 *bd = nullptr, *dinv = nullptr, *dw = nullptr, *cvdw = nullptr;
    float2 *bd32 = nullptr, *dinv32 = nullptr, *dw32 = nullptr, *cvdw32 = nullptr;

    Work<double2> wd;
    Work<float2> wf;

    // small device buffers (FP64 complex)
    double2 *part = nullptr, *g0 = nullptr, *g1 = nullptr, *rinv = nullptr;
    double2 *coefY = nullptr, *M1 = nullptr, *M2 = nullptr;
    // packed [Y_R Y_P | Y_L | M_B | sigma M_B - M_A] of the last Schur step
    // (uploaded in one copy); M1c, M2c point at its M_B and sigma M_B - M_A
    double2 *cpack = nullptr;
    const double2 *M1c = nullptr, *M2c = nullptr;
    // coefficients of the S recursion: M_B, sigma M_B - M_A (Algorithm 2, the
    // same buffers as M1, M2) or Lambda_B, sigma Lambda_B - Lambda_A (Algorithm 3)
    double2 *M1s = nullptr, *M2s = nullptr;
    // owners of M1, M2, M1s, M2s (mbase) and of dstatus, F1 (fbase)
    double2 *mbase = nullptr, *fbase = nullptr;
    // F1 holds the projected pencil's two blocks (F2 follows F1); dZr holds
    // the Ritz coefficients followed by the eigenvalues
    double2 *F1 = nullptr, *dZr = nullptr, *rnorm = nullptr;
    double2 *gmH = nullptr, *gmY = nullptr;   // block GMRES small factors (device)
    double2 *hgm = nullptr;                   // their pinned host staging
    size_t hgm_bytes = 0;
    int *dstatus = nullptr;
    double2 *hpin = nullptr;   // pinned host staging
    size_t hpin_bytes = 0;

    // host state of the iteration
    small::Mat MA, MB, RA, RB, Zr_h;
    small::Mat Rx;                       // Algorithm 3: X = V Rx (unit columns)
    std::vector<cd> lam_h, alpha_h, beta_h;
    std::vector<double> rho_h, resid_h, history;
    double max_rho = INFINITY;
    int nconv = 0, nlead = 0;   // leading pairs meeting tol: of the k wanted, of all b

    // counters
    int64_t n_iter = 0, n_iter64 = 0, n_spmm = 0, n_prec = 0, n_breakdown = 0;
    double spmm_bytes = 0.0, small_ms = 0.0, setup_ms = 0.0, iterate_ms = 0.0;
    std::map<int, Timer> timers;

    ~Ctx();
    void setup(const gplhr_csr *A, const gplhr_csr *B, cd sig, int k_, int b_,
               const gplhr_precond *T, const gplhr_options *o);
    int run(int max_it);
    void switch_to_fp64();
    void copy_out(void *V, void *Q);
    void eigvecs(double2 *X);

    int read_breakdowns();
    void tbegin(int cls);
    void tend(int cls);
    void tflush();

    template <typename T> Work<T> &W();
    template <typename T>
    void gram(const T *X, int ldx, int bx, const T *Y, int ldy, int by, const T *yscale,
              double2 *out);
    template <typename T>
    void update(T *out, int ldo, int wout, int ocol, int split, int ocol2, bool beta1, int nterms,
                const UpdTerm<T> *terms, const T *add = nullptr, int ldadd = 0);
    template <typename T>
    void project(T *X, int ldx, int xcol, int wx, const T *Y, int ldy, int ycol, int wy,
                 T *mir1 = nullptr, const T *ymir1 = nullptr, T *mir2 = nullptr,
                 const T *ymir2 = nullptr);
    template <typename T>
    void cholqr(T *X, int ld, int col, int w, int passes, T *mir1, T *mir2);
    template <typename T>
    void proj_orth(T *X, int ld, int ycol, int wy, int xcol, int w, int passes);
    template <typename T>
    void spmm_c(const T *X, int ldx, T *Y, int ldy, int w, int mode, const T *Rhs, int ldr);
    template <typename T>
    void spmm_b(const T *X, int ldx, T *Y, int ldy, int w);
    template <typename T> void cprod(const T *X, int ldx, T *Y, int ldy, int w);
    template <typename T> void bprod(const T *X, int ldx, T *Y, int ldy, int w);
    template <typename T> void deflate_left(T *Y, int ldy, int w);
    template <typename T> void deflate_right(T *X, int ldx, int col, int w);
    template <typename T> void apply_T(T *dest, int ldd, int dcol, int w);
    template <typename T>
    void apply_inner(int kind, const T *in, int ldi, T *dest, int ldd, int w);
    template <typename T> void apply_gmres(T *dest, int ldd, int dcol, int w);
    template <typename T> void srr_and_update(int s_cur, int p_cols);
    void update_locking();
    template <typename T> void init_from_Z(int w0, bool check_rank);
    template <typename T> void init_eig();
    template <typename T> void eig_orthonormalise();
    template <typename T> void iterate_once();
    template <typename T> void refresh_products();
    template <typename T> void check();
};

}  // namespace gplhr
