// C ABI of the GPLHR library (declarations and contracts in include/gplhr.h).
// Every entry point converts internal exceptions to a gplhr_status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "driver.h"

struct gplhr_ctx {
    gplhr::Ctx c;
};

namespace {
thread_local std::string g_last_error;

template <typename F>
gplhr_status guard(gplhr_t h, F &&f) {
    try {
        return static_cast<gplhr_status>(f());
    } catch (const gplhr::Error &e) {
        if (h) h->c.err = e.what();
        g_last_error = e.what();
        return static_cast<gplhr_status>(e.status);
    } catch (const std::bad_alloc &) {
        if (h) h->c.err = "host allocation failed";
        g_last_error = "host allocation failed";
        return GPLHR_ERR_ALLOC;
    } catch (const std::exception &e) {
        if (h) h->c.err = e.what();
        g_last_error = e.what();
        return GPLHR_ERR_ARG;
    }
}
}  // namespace

// Partial sums of gplhr_gram: one buffer per (device, stream), grown on
// demand and kept until the process ends.  Calls on one stream run in stream
// order, so each may reuse the buffer the previous one filled; the lock is
// held while a call enqueues its kernels, so a buffer is only replaced (after
// its stream has drained) when no call is about to use it.
namespace {
std::mutex g_gram_mu;
std::map<std::pair<int, hipStream_t>, std::pair<double2 *, size_t>> g_gram_part;
}  // namespace

extern "C" {

void gplhr_default_options(gplhr_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = GPLHR_FP64;
    opt->tol = 1e-10;
    opt->max_iter = 500;
    opt->arnoldi_m = 1;
    opt->p_mode = GPLHR_P_THICK;
    opt->V0 = nullptr;
    opt->seed = 1;
    opt->hip_stream = nullptr;
    opt->switch_tol = 1e-8;
    opt->stall_window = 3;
    opt->timing = 0;
    opt->proj_before_T = 1;
    opt->locking = 0;
    opt->m_max = 20;
    opt->algorithm = GPLHR_ALG_SCHUR;
    opt->defl_V = nullptr;
    opt->defl_Q = nullptr;
    opt->defl_k = 0;
}

gplhr_status gplhr_create(const gplhr_csr *A, const gplhr_csr *B, double sigma_re,
                          double sigma_im, int k, int block, const gplhr_precond *T,
                          const gplhr_options *opt, gplhr_t *out) {
    if (!out) {
        g_last_error = "out must not be NULL";
        return GPLHR_ERR_ARG;
    }
    *out = nullptr;
    gplhr_t h = nullptr;
    try {
        h = new gplhr_ctx();
    } catch (...) {
        g_last_error = "host allocation failed";
        return GPLHR_ERR_ALLOC;
    }
    gplhr_status s = guard(h, [&]() {
        h->c.setup(A, B, gplhr::cd(sigma_re, sigma_im), k, block, T, opt);
        return 0;
    });
    if (s < 0) {
        g_last_error = h->c.err;
        delete h;
        return s;
    }
    *out = h;
    return GPLHR_OK;
}

gplhr_status gplhr_iterate(gplhr_t h, int max_iter, int *n_converged, double *max_rel_resid) {
    if (!h) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        const int s = h->c.run(max_iter);
        if (n_converged) *n_converged = h->c.nconv;
        if (max_rel_resid) *max_rel_resid = h->c.max_rho;
        return s;
    });
}

gplhr_status gplhr_get_schur(gplhr_t h, void *V, void *Q, double *RA, double *RB, double *lambda,
                             double *rel_resid) {
    if (!h) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        gplhr::Ctx &c = h->c;
        if (c.eig) throw gplhr::Error(-8, "the eigenvector form keeps no Schur factors (gplhr_get_eig)");
        if ((int)c.lam_h.size() < c.k || (int)c.rho_h.size() < c.k || c.MB.r < c.k)
            throw gplhr::Error(-8, "no iterate available");
        c.copy_out(V, Q);
        const int k = c.k;
        using gplhr::small::Mat;
        Mat ra(k, k), rb(k, k);
        if (c.bk == gplhr::B_IDENT) {
            // R = M_B^{-1} M_A (last line of Algorithm 2)
            Mat mb(k, k), ma(k, k);
            for (int j = 0; j < k; ++j)
                for (int i = 0; i < k; ++i) {
                    mb(i, j) = c.MB(i, j);
                    ma(i, j) = c.MA(i, j);
                }
            Mat r;
            if (!gplhr::small::lu_solve(mb, ma, r)) throw gplhr::Error(-6, "M_B is singular");
            ra = r;
            rb = Mat::eye(k);
        } else {
            for (int j = 0; j < k; ++j)
                for (int i = 0; i < k; ++i) {
                    ra(i, j) = c.RA(i, j);
                    rb(i, j) = c.RB(i, j);
                }
        }
        if (RA) std::memcpy(RA, ra.data(), sizeof(gplhr::cd) * k * k);
        if (RB) std::memcpy(RB, rb.data(), sizeof(gplhr::cd) * k * k);
        if (lambda) std::memcpy(lambda, c.lam_h.data(), sizeof(gplhr::cd) * k);
        if (rel_resid) std::memcpy(rel_resid, c.rho_h.data(), sizeof(double) * k);
        return c.converged ? 0 : 1;
    });
}

gplhr_status gplhr_get_residual_norms(gplhr_t h, double *resid) {
    if (!h || !resid) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        gplhr::Ctx &c = h->c;
        if ((int)c.resid_h.size() < c.k) throw gplhr::Error(-8, "no iterate available");
        // x_j = V z_j with orthonormal V and unit z_j, so ||x_j|| = 1
        std::memcpy(resid, c.resid_h.data(), sizeof(double) * c.k);
        return c.converged ? 0 : 1;
    });
}

gplhr_status gplhr_get_eigvecs(gplhr_t h, void *X) {
    if (!h || !X) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        h->c.eigvecs(static_cast<double2 *>(X));
        return 0;
    });
}

gplhr_status gplhr_get_eig(gplhr_t h, void *X, double *LA, double *LB, double *rel_resid) {
    if (!h) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        gplhr::Ctx &c = h->c;
        if (!c.eig) throw gplhr::Error(-8, "gplhr_get_eig needs a GPLHR_ALG_EIG handle");
        if ((int)c.alpha_h.size() < c.k || (int)c.rho_h.size() < c.k)
            throw gplhr::Error(-8, "no iterate available");
        if (X) c.eigvecs(static_cast<double2 *>(X));
        const int k = c.k;
        if (LA) std::memcpy(LA, c.alpha_h.data(), sizeof(gplhr::cd) * k);
        if (LB) std::memcpy(LB, c.beta_h.data(), sizeof(gplhr::cd) * k);
        if (rel_resid) std::memcpy(rel_resid, c.rho_h.data(), sizeof(double) * k);
        return c.converged ? 0 : 1;
    });
}

gplhr_status gplhr_eig_backward(gplhr_t h, const double *grad_lambda, void *grad_valA,
                                void *grad_valB) {
    if (!h || !grad_lambda || !grad_valA) return GPLHR_ERR_ARG;
    return guard(h, [&]() -> int {
        gplhr::Ctx &c = h->c;
        if (!c.converged) throw gplhr::Error(-8, "gplhr_eig_backward needs a converged handle");
        if (c.defl_k) throw gplhr::Error(-8, "gplhr_eig_backward is not available for a deflated handle");
        const int64_t n = c.n;
        const int k = c.k;
        hipStream_t st = c.st;
        // right eigenvectors x_e (unit norm)
        double2 *X = nullptr, *Y = nullptr, *BX = nullptr, *coef = nullptr;
        int32_t *trp = nullptr, *tci = nullptr, *brp = nullptr, *bci = nullptr;
        double2 *tval = nullptr, *bval = nullptr;
        struct Cleanup {
            std::vector<void *> p;
            ~Cleanup() {
                for (void *q : p)
                    if (q) (void)hipFree(q);
            }
        } cl;
        GPLHR_HIP_CHECK(hipMalloc((void **)&X, sizeof(double2) * n * k));
        cl.p.push_back(X);
        c.eigvecs(X);
        // left eigenvectors from the adjoint pencil (A^H, B^H, conj(sigma))
        gplhr::csr_conj_transpose(st, n, c.a_nnz, c.a_rp, c.a_ci, c.a_val, &trp, &tci, &tval);
        cl.p.push_back(trp); cl.p.push_back(tci); cl.p.push_back(tval);
        gplhr_csr AH{n, c.a_nnz, trp, tci, tval};
        gplhr_csr BH{};
        const gplhr_csr *pBH = nullptr;
        if (c.bk != gplhr::B_IDENT) {
            gplhr::csr_conj_transpose(st, n, c.b_nnz, c.b_rp, c.b_ci, c.b_val, &brp, &bci, &bval);
            cl.p.push_back(brp); cl.p.push_back(bci); cl.p.push_back(bval);
            BH = gplhr_csr{n, c.b_nnz, brp, bci, bval};
            pBH = &BH;
        }
        gplhr_options o2 = c.opt;
        o2.V0 = nullptr;
        o2.seed = c.opt.seed + 0x5bd1e995ULL;
        gplhr::Ctx adj;
        adj.setup(&AH, pBH, std::conj(c.sigma), k, c.b, &c.pre, &o2);
        const int as = adj.run(c.opt.max_iter);
        if (as != 0)
            throw gplhr::Error(1, "adjoint solve did not converge (max residual " +
                                      std::to_string(adj.max_rho) + ")");
        GPLHR_HIP_CHECK(hipMalloc((void **)&Y, sizeof(double2) * n * k));
        cl.p.push_back(Y);
        adj.eigvecs(Y);
        // pair each lambda_e with the adjoint eigenvalue nearest conj(lambda_e)
        std::vector<int> perm(k, -1);
        std::vector<bool> used(k, false);
        for (int e = 0; e < k; ++e) {
            double best = INFINITY;
            int bj = -1;
            for (int j = 0; j < k; ++j) {
                if (used[j]) continue;
                const double d = std::abs(adj.lam_h[j] - std::conj(c.lam_h[e]));
                if (d < best) { best = d; bj = j; }
            }
            perm[e] = bj;
            used[bj] = true;
        }
        {
            std::vector<double2> P(k * k, make_double2(0.0, 0.0));
            for (int e = 0; e < k; ++e) P[perm[e] + e * k] = make_double2(1.0, 0.0);
            GPLHR_HIP_CHECK(hipMemcpyAsync(c.coefY, P.data(), sizeof(double2) * k * k, hipMemcpyHostToDevice, st));
            GPLHR_HIP_CHECK(hipStreamSynchronize(st));
            gplhr::UpdTerm<double2> t;
            t.in = Y; t.ld = k; t.col = 0; t.w = k; t.M = c.coefY; t.ldm = k;
            gplhr::launch_update<double2>(st, n, Y, k, k, 0, k, 0, make_double2(0, 0), 1, &t);
        }
        // y_e^H B x_e and ||B x_e||
        const double2 *bx = X;
        const double2 *bsc = nullptr;
        if (c.bk == gplhr::B_DIAG) {
            bsc = c.bd;
        } else if (c.bk == gplhr::B_SPARSE) {
            GPLHR_HIP_CHECK(hipMalloc((void **)&BX, sizeof(double2) * n * k));
            cl.p.push_back(BX);
            gplhr::launch_spmm<double2>(st, n, c.b_rp, c.b_ci, c.b_val, X, k, BX, k, k, 0, nullptr, 0,
                                        nullptr, c.b_plane, c.b_nnz);
            bx = BX;
        }
        c.gram<double2>(Y, k, k, bx, k, k, bsc, c.g0);
        if (bsc) {
            GPLHR_HIP_CHECK(hipMalloc((void **)&BX, sizeof(double2) * n * k));
            cl.p.push_back(BX);
            gplhr::launch_scale_rows<double2>(st, n, k, X, k, bsc, BX, k);
            bx = BX;
        }
        c.gram<double2>(bx, k, k, bx, k, k, nullptr, c.g1);
        std::vector<gplhr::cd> yBx(k * k), bxn(k * k);
        GPLHR_HIP_CHECK(hipMemcpyAsync(yBx.data(), c.g0, sizeof(double2) * k * k, hipMemcpyDeviceToHost, st));
        GPLHR_HIP_CHECK(hipMemcpyAsync(bxn.data(), c.g1, sizeof(double2) * k * k, hipMemcpyDeviceToHost, st));
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        std::vector<gplhr::cd> ca(k), cb(k);
        for (int e = 0; e < k; ++e) {
            const gplhr::cd d = yBx[e + e * k];
            const double nb = std::sqrt(std::abs(bxn[e + e * k].real()));
            if (!(std::abs(d) > 1e-12 * nb))
                throw gplhr::Error(-7, "eigenvalue " + std::to_string(e) + " is not simple (y^H B x ~ 0)");
            const gplhr::cd g(grad_lambda[2 * e], grad_lambda[2 * e + 1]);
            ca[e] = g / std::conj(d);
            cb[e] = -ca[e] * std::conj(c.lam_h[e]);
        }
        GPLHR_HIP_CHECK(hipMalloc((void **)&coef, sizeof(double2) * 2 * k));
        cl.p.push_back(coef);
        GPLHR_HIP_CHECK(hipMemcpy(coef, ca.data(), sizeof(double2) * k, hipMemcpyHostToDevice));
        GPLHR_HIP_CHECK(hipMemcpy(coef + k, cb.data(), sizeof(double2) * k, hipMemcpyHostToDevice));
        gplhr::launch_sddmm(st, n, c.a_rp, c.a_ci, k, Y, k, X, k, coef,
                            static_cast<double2 *>(grad_valA));
        if (grad_valB && c.bk != gplhr::B_IDENT)
            gplhr::launch_sddmm(st, n, c.b_rp, c.b_ci, k, Y, k, X, k, coef + k,
                                static_cast<double2 *>(grad_valB));
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        return 0;
    });
}

gplhr_status gplhr_get_stats(gplhr_t h, gplhr_stats *out) {
    if (!h || !out) return GPLHR_ERR_ARG;
    return guard(h, [&]() {
        gplhr::Ctx &c = h->c;
        std::memset(out, 0, sizeof(*out));
        out->iterations = c.n_iter;
        out->fp64_iterations = c.n_iter64;
        out->spmm_calls = c.n_spmm;
        out->precond_calls = c.n_prec;
        out->breakdowns = c.n_breakdown;
        auto ms = [&](int cls) {
            auto it = c.timers.find(cls);
            return it == c.timers.end() ? 0.0 : it->second.ms;
        };
        out->spmm_ms = ms(gplhr::T_SPMM);
        out->spmm_bytes = c.spmm_bytes;
        out->gram_ms = ms(gplhr::T_GRAM);
        out->update_ms = ms(gplhr::T_UPDATE);
        out->small_host_ms = c.small_ms;
        out->setup_ms = c.setup_ms;
        out->iterate_ms = c.iterate_ms;
        out->max_rel_resid = c.max_rho;
        out->n_converged = c.nconv;
        out->phase = c.phase;
        out->locked = c.q;
        out->arnoldi_m = c.m_cur;
        return 0;
    });
}

void gplhr_destroy(gplhr_t h) { delete h; }

const char *gplhr_last_error(gplhr_t h) {
    if (h) return h->c.err.c_str();
    return g_last_error.c_str();
}

gplhr_status gplhr_spmm(int dtype, int64_t n, int64_t nnz, const int32_t *row_ptr,
                        const int32_t *col_idx, const void *val, const void *X, int ldx, void *Y,
                        int ldy, int b, int plane, void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 0 || nnz < 0 || b < 1 || b > 64 || ldx < b || ldy < b || (dtype != 0 && dtype != 1) ||
            plane < 0 || (plane > 0 && (n % plane != 0 || plane % 8 != 0)))
            throw gplhr::Error(-1, "gplhr_spmm: bad arguments");
        if (n == 0) return 0;
        if (!row_ptr || !X || !Y) throw gplhr::Error(-1, "gplhr_spmm: null pointer");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (dtype == 0)
            gplhr::launch_spmm<double2>(st, n, row_ptr, col_idx, static_cast<const double2 *>(val),
                                        static_cast<const double2 *>(X), ldx,
                                        static_cast<double2 *>(Y), ldy, b, 0, nullptr, 0, nullptr,
                                        plane, nnz);
        else
            gplhr::launch_spmm<float2>(st, n, row_ptr, col_idx, static_cast<const float2 *>(val),
                                       static_cast<const float2 *>(X), ldx,
                                       static_cast<float2 *>(Y), ldy, b, 0, nullptr, 0, nullptr,
                                       plane, nnz);
        return 0;
    });
}

gplhr_status gplhr_csr_plane(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int *plane, void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 0 || !plane || (n > 0 && !row_ptr)) throw gplhr::Error(-1, "gplhr_csr_plane: bad arguments");
        *plane = n == 0 ? 0 : gplhr::spmm_plane(static_cast<hipStream_t>(hip_stream), n, row_ptr, col_idx);
        return 0;
    });
}

gplhr_status gplhr_gram(int dtype, int64_t n, const void *X, int ldx, int bx, const void *Y,
                        int ldy, int by, void *G, void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 1 || bx < 1 || by < 1 || bx > 64 || by > 64 || ldx < bx || ldy < by ||
            (dtype != 0 && dtype != 1) || !X || !Y || !G)
            throw gplhr::Error(-1, "gplhr_gram: bad arguments");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const size_t cap = (size_t)1024 * bx * by;
        int dev = 0;
        GPLHR_HIP_CHECK(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lock(g_gram_mu);
        auto &buf = g_gram_part[{dev, st}];
        if (buf.second < cap) {
            if (buf.first) {
                GPLHR_HIP_CHECK(hipStreamSynchronize(st));
                GPLHR_HIP_CHECK(hipFree(buf.first));
                buf = {nullptr, 0};
            }
            GPLHR_HIP_CHECK(hipMalloc((void **)&buf.first, sizeof(double2) * cap));
            buf.second = cap;
        }
        double2 *part = buf.first;
        if (dtype == 0)
            gplhr::launch_gram<double2>(st, n, static_cast<const double2 *>(X), ldx, bx,
                                        static_cast<const double2 *>(Y), ldy, by, nullptr, part,
                                        cap, static_cast<double2 *>(G), bx);
        else
            gplhr::launch_gram<float2>(st, n, static_cast<const float2 *>(X), ldx, bx,
                                       static_cast<const float2 *>(Y), ldy, by, nullptr, part, cap,
                                       static_cast<double2 *>(G), bx);
        return 0;
    });
}

gplhr_status gplhr_proj_orth(int dtype, int64_t n, void *Z, int ld, int wy, int w, int passes,
                             void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 1 || w < 1 || w > 48 || wy < 0 || wy > 48 || wy + w > 64 || ld < wy + w ||
            passes < 1 || passes > 3 || (dtype != 0 && dtype != 1) || !Z)
            throw gplhr::Error(-1, "gplhr_proj_orth: bad arguments");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int wg = wy + w;
        // one allocation: Gram partials | G = [Y X]^H X | R^{-1} | C_Y | counter
        const size_t cap = (size_t)1024 * wg * w;
        const size_t nG = (size_t)wg * w, nR = (size_t)w * w, nC = (size_t)std::max(wy, 1) * w;
        double2 *buf = nullptr;
        GPLHR_HIP_CHECK(hipMallocAsync((void **)&buf, sizeof(double2) * (cap + nG + nR + nC + 1), st));
        // released on every path out, errors included
        struct Release {
            double2 *&p;
            hipStream_t s;
            ~Release() { if (p) (void)hipFreeAsync(p, s); }
        } release{buf, st};
        double2 *part = buf, *G = buf + cap, *rinv = G + nG, *cy = rinv + nR;
        int *status = reinterpret_cast<int *>(cy + nC);
        GPLHR_HIP_CHECK(hipMemsetAsync(status, 0, sizeof(int), st));
        auto run = [&](auto *X) {
            using T = std::remove_pointer_t<decltype(X)>;
            for (int p = 0; p < passes; ++p) {
                gplhr::launch_gram<T>(st, n, X, ld, wg, X + wy, ld, w, nullptr, part, cap, G, wg);
                gplhr::launch_chol_proj(st, wy, w, G, rinv, cy, status, p + 1 < passes);
                gplhr::UpdTerm<T> t[2];
                t[0].in = X; t[0].ld = ld; t[0].col = wy; t[0].w = w; t[0].M = rinv; t[0].ldm = w;
                t[0].upper = true;
                t[1].in = X; t[1].ld = ld; t[1].col = 0; t[1].w = wy; t[1].M = cy; t[1].ldm = wy;
                gplhr::launch_update<T>(st, n, X, ld, w, wy, w, 0, make_double2(0.0, 0.0),
                                        wy > 0 ? 2 : 1, t);
            }
        };
        if (dtype == 0) run(static_cast<double2 *>(Z));
        else run(static_cast<float2 *>(Z));
        int pivots = 0;
        GPLHR_HIP_CHECK(hipMemcpyAsync(&pivots, status, sizeof(int), hipMemcpyDeviceToHost, st));
        GPLHR_HIP_CHECK(hipFreeAsync(buf, st));
        buf = nullptr;
        GPLHR_HIP_CHECK(hipStreamSynchronize(st));
        if (pivots > 0)
            throw gplhr::Error(-4, "gplhr_proj_orth: a Cholesky pivot of the projected block vanished "
                                   "(the block is rank deficient to working precision)");
        return 0;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free Gram: its partial sums live in a file-scope device array.
// ---------------------------------------------------------------------------
// Each GPU the library runs on holds its own copy of this array until the
// process ends.  In host code `scratch` names a host-side stand-in, so kernels
// get the device address that hipGetSymbolAddress returns for the current
// device (kept per device below), never the array's name.
static constexpr size_t NOALLOC_SCRATCH_ENTRIES = (size_t)1 << 20;   // complex128, 16 MiB
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_ENTRIES];

namespace {
std::mutex g_scratch_mu;
std::map<int, double2 *> g_scratch_ptr;   // device ordinal -> address of `scratch`

// Device address of `scratch` on the current device; looked up once per device.
double2 *scratch_on_current_device() {
    int dev = -1;
    GPLHR_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    GPLHR_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw gplhr::Error(-3, "gplhr_gram_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double2 *>(ptr);
    return static_cast<double2 *>(ptr);
}
}  // namespace

extern "C" {

gplhr_status gplhr_block_copy(int dtype, int64_t n, const void *X, int ldx, void *Y, int ldy, int w,
                              void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 0 || w < 1 || ldx < w || ldy < w || (dtype != 0 && dtype != 1))
            throw gplhr::Error(-1, "gplhr_block_copy: bad arguments");
        if (n == 0) return 0;
        if (!X || !Y) throw gplhr::Error(-1, "gplhr_block_copy: null pointer");
        const uintptr_t al = reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y);
        // 16-byte vectors: whole complex128 entries, or complex64 pairs
        if (dtype == 1 && (w % 2 != 0 || ldx % 2 != 0 || ldy % 2 != 0 || al % 16 != 0))
            throw gplhr::Error(-1, "gplhr_block_copy: complex64 blocks need even widths, even "
                                   "leading dimensions and 16-byte alignment");
        if (dtype == 0 && al % 16 != 0) throw gplhr::Error(-1, "gplhr_block_copy: misaligned block");
        const int per = dtype == 0 ? 1 : 2;   // complex entries per vector
        gplhr::launch_block_copy(static_cast<hipStream_t>(hip_stream), n, w / per, X, ldx / per, Y,
                                 ldy / per);
        return 0;
    });
}

gplhr_status gplhr_gram_noalloc(int dtype, int64_t n, const void *X, int ldx, int bx,
                                const void *Y, int ldy, int by, void *G, void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 1 || bx < 1 || by < 1 || bx > 64 || by > 64 || ldx < bx || ldy < by ||
            (dtype != 0 && dtype != 1) || !X || !Y || !G)
            throw gplhr::Error(-1, "gplhr_gram_noalloc: bad arguments");
        // one block's real partial Gram takes 4 bx by doubles (2 bx by
        // complex128 entries); the kernel uses as many blocks as fit
        if ((size_t)2 * bx * by > NOALLOC_SCRATCH_ENTRIES)
            throw gplhr::Error(-1, "gplhr_gram_noalloc: partial sums exceed the 16 MiB scratch");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        double2 *part = scratch_on_current_device();
        if (dtype == 0)
            gplhr::launch_gram<double2>(st, n, static_cast<const double2 *>(X), ldx, bx,
                                        static_cast<const double2 *>(Y), ldy, by, nullptr, part,
                                        NOALLOC_SCRATCH_ENTRIES, static_cast<double2 *>(G), bx);
        else
            gplhr::launch_gram<float2>(st, n, static_cast<const float2 *>(X), ldx, bx,
                                       static_cast<const float2 *>(Y), ldy, by, nullptr, part,
                                       NOALLOC_SCRATCH_ENTRIES, static_cast<double2 *>(G), bx);
        return 0;
    });
}

}  // extern "C"

namespace {
// Y = T R with T the damped Jacobi iteration on C w = R from w_0 = 0:
// w_1 = dw .* R, w_{t+1} = w_t + dw .* (R - C w_t), dw = omega / diag(C).
// The same kernel sequence as the solver's preconditioner application.
template <typename T>
void jacobi_apply(hipStream_t st, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                  const T *val, const T *valdw, const T *dw, int sweeps, const T *R, int ldr, T *Y,
                  int ldy, int b, int plane) {
    if (sweeps == 1) {
        gplhr::launch_scale_rows<T>(st, n, b, R, ldr, dw, Y, ldy);
        return;
    }
    // w_1 and w_2 in one pass (mode 2), then one pass per further sweep
    T *J[2] = {nullptr, nullptr};
    if (sweeps > 2) J[0] = static_cast<T *>(gplhr::dev_alloc(sizeof(T) * n * b, st));
    if (sweeps > 3) J[1] = static_cast<T *>(gplhr::dev_alloc(sizeof(T) * n * b, st));
    int cur = -1;
    for (int t = 1; t < sweeps; ++t) {
        const bool last = (t == sweeps - 1);
        const int nxt = cur == 0 ? 1 : 0;
        T *o = last ? Y : J[nxt];
        if (t == 1)
            gplhr::launch_spmm<T>(st, n, rp, ci, valdw, R, ldr, o, last ? ldy : b, b, 2, R, ldr, dw,
                                  plane, nnz);
        else
            gplhr::launch_spmm<T>(st, n, rp, ci, val, J[cur], b, o, last ? ldy : b, b, 1, R, ldr, dw,
                                  plane, nnz);
        cur = nxt;
    }
    if (J[0]) gplhr::dev_free(J[0], st);
    if (J[1]) gplhr::dev_free(J[1], st);
}
}  // namespace

extern "C" {

gplhr_status gplhr_jacobi(int dtype, int64_t n, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, const void *val, double omega, int sweeps,
                          const void *R, int ldr, void *Y, int ldy, int b, int plane,
                          void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 0 || nnz < 0 || nnz > INT32_MAX || b < 1 || b > 64 || ldr < b || ldy < b ||
            sweeps < 1 || sweeps > 64 || !(omega > 0.0) || !std::isfinite(omega) ||
            (dtype != 0 && dtype != 1) || plane < 0 ||
            (plane > 0 && (n % plane != 0 || plane % 8 != 0)))
            throw gplhr::Error(-1, "gplhr_jacobi: bad arguments");
        if (n == 0) return 0;
        if (!row_ptr || !col_idx || !val || !R || !Y) throw gplhr::Error(-1, "gplhr_jacobi: null pointer");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const double2 *v = static_cast<const double2 *>(val);
        double2 *dg = static_cast<double2 *>(gplhr::dev_alloc(sizeof(double2) * n, st));
        const int64_t zeros = gplhr::extract_diag(st, n, row_ptr, col_idx, v, dg);
        if (zeros) {
            gplhr::dev_free(dg, st);
            throw gplhr::Error(-1, "gplhr_jacobi: diag(C) has " + std::to_string(zeros) + " zero entries");
        }
        double2 *dw = static_cast<double2 *>(gplhr::dev_alloc(sizeof(double2) * n, st));
        gplhr::launch_recip_scaled(st, n, dg, make_double2(omega, 0.0), dw);
        // values of C diag(omega / diag(C)) for the first two sweeps in one pass
        double2 *vdw = (sweeps > 1 && nnz) ? static_cast<double2 *>(gplhr::dev_alloc(sizeof(double2) * nnz, st))
                                           : nullptr;
        if (vdw) gplhr::launch_scale_cols(st, nnz, col_idx, v, dw, vdw);
        if (dtype == 0) {
            jacobi_apply<double2>(st, n, nnz, row_ptr, col_idx, v, vdw, dw, sweeps,
                                  static_cast<const double2 *>(R), ldr, static_cast<double2 *>(Y),
                                  ldy, b, plane);
        } else {
            // complex64 copies of the values, of omega / diag(C) and of the
            // scaled values, as in the solver's complex64 phase
            float2 *v32 = nnz ? static_cast<float2 *>(gplhr::dev_alloc(sizeof(float2) * nnz, st)) : nullptr;
            float2 *vdw32 = vdw ? static_cast<float2 *>(gplhr::dev_alloc(sizeof(float2) * nnz, st)) : nullptr;
            float2 *dw32 = static_cast<float2 *>(gplhr::dev_alloc(sizeof(float2) * n, st));
            if (nnz) gplhr::launch_c128_to_c64_flat(st, nnz, v, v32);
            if (vdw) gplhr::launch_c128_to_c64_flat(st, nnz, vdw, vdw32);
            gplhr::launch_c128_to_c64_flat(st, n, dw, dw32);
            jacobi_apply<float2>(st, n, nnz, row_ptr, col_idx, v32, vdw32, dw32, sweeps,
                                 static_cast<const float2 *>(R), ldr, static_cast<float2 *>(Y),
                                 ldy, b, plane);
            if (v32) gplhr::dev_free(v32, st);
            if (vdw32) gplhr::dev_free(vdw32, st);
            gplhr::dev_free(dw32, st);
        }
        if (vdw) gplhr::dev_free(vdw, st);
        gplhr::dev_free(dg, st);
        gplhr::dev_free(dw, st);
        return 0;
    });
}

gplhr_status gplhr_block_update(int dtype, int64_t n, const void *X, int ldx, int wx,
                                const void *M, int ldm, void *Y, int ldy, int wy,
                                double beta_re, double beta_im, void *hip_stream) {
    return guard(nullptr, [&]() {
        if (n < 1 || wx < 1 || wx > 128 || wy < 1 || wy > 48 || ldx < wx || ldy < wy ||
            ldm < wx || (dtype != 0 && dtype != 1) || !X || !M || !Y)
            throw gplhr::Error(-1, "gplhr_block_update: bad arguments");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const double2 beta = make_double2(beta_re, beta_im);
        if (dtype == 0) {
            gplhr::UpdTerm<double2> t;
            t.in = static_cast<const double2 *>(X); t.ld = ldx; t.w = wx;
            t.M = static_cast<const double2 *>(M); t.ldm = ldm;
            gplhr::launch_update<double2>(st, n, static_cast<double2 *>(Y), ldy, wy, 0, wy, 0,
                                          beta, 1, &t);
        } else {
            gplhr::UpdTerm<float2> t;
            t.in = static_cast<const float2 *>(X); t.ld = ldx; t.w = wx;
            t.M = static_cast<const double2 *>(M); t.ldm = ldm;
            gplhr::launch_update<float2>(st, n, static_cast<float2 *>(Y), ldy, wy, 0, wy, 0, beta,
                                         1, &t);
        }
        return 0;
    });
}

}  // extern "C"
