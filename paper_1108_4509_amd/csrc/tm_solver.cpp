// Host driver of the trace-minimization eigensolver: enqueues the kernels of
// one nonlinear-CG iteration (Fig. 1) -- energy and gradient by Algorithm-2
// (Fig. 2), Polak-Ribiere direction (Eq. 8), line step, Cholesky
// orthonormalization (Fig. 4) -- and the precision phases of Sec. 2.2.
// All scalars (gamma, alpha, convergence) live on the device; the host only
// polls a small state record every k_check iterations.
#include "tm_solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

namespace tmin {

// ------------------------------------------------------------------ buffers

DevMem::DevMem(tm_ctx *c, size_t bytes) : ctx(c), size(bytes) {
    if (bytes == 0) return;
    ptr = ctx->dalloc(bytes);
    TM_REQUIRE(ptr != nullptr, TM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
}
DevMem::~DevMem() {
    if (ptr) ctx->dfree(ptr);
}

int spmm_any(hipStream_t s, const tm_mat *H, int ld, const void *C, void *X, bool f64, int ndot,
             double *partials, const SpmmEpi &epi) {
    TM_REQUIRE(!epi.D || !H->is_stencil, TM_ENOTSUP, "batched operators are CSR");
    if (H->is_stencil) {
        if (f64)
            return spmm_stencil<double>(s, H->st, H->n, ld, (const double *)C, (double *)X, ndot,
                                        partials, epi);
        return spmm_stencil<float>(s, H->st, H->n, ld, (const float *)C, (float *)X, ndot,
                                   partials, epi);
    }
    if (f64)
        return spmm_csr<double>(s, H->csr, ld, (const double *)C, (double *)X, ndot, partials, epi);
    return spmm_csr<float>(s, H->csr, ld, (const float *)C, (float *)X, ndot, partials, epi);
}

namespace {

template <typename T> constexpr bool is_f64() { return sizeof(T) == 8; }

struct Phase {
    // storage of C and X; storage of G, G_prev, P, Y; matrix-core precision
    // of H' and G; precision of S = C^T C; precision of the TRMM's C R'
    bool c64, g64, mh64, ms64, t64;
    int id() const { return (c64 ? 1 : 0) | (g64 ? 2 : 0) | (mh64 ? 4 : 0) | (ms64 ? 8 : 0) | (t64 ? 16 : 0); }
};

Phase phase_of(int precision) {
    switch (precision) {
    case TM_FULL_DP: return {true, true, true, true, true};
    case TM_FULL_SP: return {false, false, false, false, false};
    case TM_MP2: return {true, false, false, true, false};    // Sec. 2.2 MP2
    case TM_MP1: return {true, false, true, true, false};     // Sec. 2.2 MP1 (i) and (ii)
    default: return {true, true, true, true, true};
    }
}

}  // namespace

// ------------------------------------------------------------------ footprint

size_t solve_footprint(int64_t n, int64_t nnz, int m, int precision, int precondition,
                       int history_len) {
    const size_t ld = (size_t)leading_dim(m);
    const size_t blk8 = (size_t)n * ld * 8, blk4 = (size_t)n * ld * 4;
    // blocks that can be alive together (C, C_next, X per precision of C;
    // G, G_prev, P, Y), see alloc_c / alloc_g; the FP32 set and the FP64 set
    // coexist at the MIXED switch and at the final FP64 Rayleigh-Ritz
    size_t blocks;
    switch (precision) {
    case TM_FULL_DP: blocks = 3 * blk8 + 4 * blk8; break;
    case TM_MP2:
    case TM_MP1:
    case TM_MP2_MP1: blocks = 3 * blk8 + 4 * blk4; break;
    default: blocks = 3 * blk4 + 3 * blk8 + 4 * blk4; break;   // FULL_SP, MIXED
    }
    const size_t md = (size_t)m * m * 8;
    size_t small = 3 * ld * 8 + 8 * ld * 8 + 5 * md + ld * ld * 8 + gram_workspace(n, m) +
                   std::max({coldots_workspace(n, (int)ld), spmm_partials_workspace(n, (int)ld),
                             rot_partials_workspace(n, m)}) +
                   chol_workspace(m) + jacobi_workspace(m) + 64 + sizeof(CgState) +
                   (size_t)2 * std::max(history_len, 0) * 8 + (precondition == 1 ? (size_t)n * 8 : 0) +
                   (precondition == 2 ? 3 * blk8 : 0);   // the polynomial's work blocks
    // the matrix (CSR: rowptr, col, FP64 and FP32 values, diagonal; stencil:
    // V in FP64 and FP32), plus 16 bytes of slack per upload
    const size_t mat = nnz > 0 ? (size_t)(n + 1) * 8 + (size_t)nnz * (4 + 8 + 4) + (size_t)n * 8 + 80
                               : (size_t)n * 12 + 32;
    return blocks + small + mat;
}

size_t batch_footprint(int64_t n, int64_t nnz, int k, int m, int precision, int precondition) {
    const int mb = k * batch_group_ld(k, m);
    // the solve on the whole block, each problem's diagonal in FP64 and
    // FP32, controller states and polynomial coefficients, upload slack
    // (the Gram partials of the diagonal-block launches may take more splits)
    const int ldg = batch_group_ld(k, m);
    return solve_footprint(n, nnz, mb, precision, precondition, 0) +
           (gram_workspace(n, mb, ldg) - gram_workspace(n, mb)) +
           (size_t)k * ((size_t)n * 12 + sizeof(CgState) + 16) + 256;
}

// ------------------------------------------------------------------ solver

struct Solver::Impl {
    tm_ctx *ctx;
    const tm_mat *H;
    int m, ld;
    int64_t n;
    double tol;
    tm_opts o;
    hipStream_t s;

    // the S of H x = lambda S x (Sec. 2.1), or null for the standard problem
    const tm_mat *Smat = nullptr;
    // blocks (allocated per precision of C and of G); Z = S C and W = S P
    // for the generalized problem
    std::unique_ptr<DevMem> C64, Cn64, X64, C32, Cn32, X32, Z64, W64;
    std::unique_ptr<DevMem> G, Gp, P, Y;  // element size set by g64
    std::unique_ptr<DevMem> Zc, Rc, Dc;   // polynomial preconditioner: Z = M G and its work blocks
    bool g64_alloc = false;
    // polynomial preconditioner: Chebyshev iteration for (H - sigma) z = g on
    // [a, b] = Gershgorin bounds - sigma; theta, delta its centre and half-width
    double ch_sigma = 0, ch_theta = 1, ch_delta = 1;
    // degree 2: z = ch_lin_a g + ch_lin_b H g (the two steps expanded)
    double ch_lin_a = 0, ch_lin_b = 0;
    // small buffers
    std::unique_ptr<DevMem> h, d, w, dots, dots2, Hp, S, Rinv, Amat, U, Wp;
    std::unique_ptr<DevMem> gram_ws, dot_ws, chol_ws, jac_ws, info, state, hist, M;
    CgState *st = nullptr;
    CgState *st_host = nullptr;
    int32_t *info_host = nullptr;
    int rotations = 0;
    bool bf16_bulk = false;   // the FP32 phase forms H' on BF16 matrix cores

    // a batched solve of the ng problems H_g = A + diag(d_g) of a batch
    // matrix: problem g owns columns g * ldg .. g * ldg + mg - 1 of every
    // block (zero columns pad it to ldg), m = ng * ldg; every small matrix
    // is block-diagonal, every column operation reads its problem's state.
    // One problem: ng = 1, mg = m, ldg = 0.
    bool batched = false;
    int ng = 1, mg = 0, ldg = 0;
    std::unique_ptr<DevMem> gab;   // per-problem a, b of the degree-2 polynomial
    std::vector<double> switch_g;  // per-problem switch_tol

    // captured iteration batches, keyed by the buffers they were recorded on
    // and the precision phase (which selects the kernels)
    struct GraphKey {
        const void *c32, *c64, *g, *gp, *p, *y;
        int phase;
        bool operator==(const GraphKey &o) const {
            return c32 == o.c32 && c64 == o.c64 && g == o.g && gp == o.gp && p == o.p && y == o.y &&
                   phase == o.phase;
        }
    };
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    ~Impl() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    }

    Impl(tm_ctx *c, const tm_mat *Hm, const tm_mat *Sm, int mm, double t, const tm_opts &oo)
        : ctx(c), H(Hm), m(mm), ld(leading_dim(mm)), n(Hm->n), tol(t), o(oo), s(c->stream), Smat(Sm) {
        mg = mm;
        if (Hm->batch_k > 0) {
            batched = true;
            ng = Hm->batch_k;
            ldg = batch_group_ld(ng, mm);
            m = ng * ldg;
            ld = leading_dim(m);
        }
    }

    // the block-diagonal mask of a batched solve's m x m results
    BatchCols bcols(double pad) const {
        BatchCols b;
        if (batched) {
            b.ldg = ldg;
            b.mg = mg;
            b.pad = pad;
        }
        return b;
    }
    // a batch's S = C^T C is block diagonal with the problems' ldg x ldg
    // blocks; its Cholesky runs on the smallest diagonal blocks that hold
    // whole problems and are a multiple of 64 wide (0: one m x m matrix)
    int chol_block() const {
        if (!batched) return 0;
        int a = ldg, b = 64;
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        const int sb = ldg / a * 64;   // lcm(ldg, 64), which divides m = ng * ldg
        return sb < m ? sb : 0;
    }
    // a batch's m x m matrices (A, U, R^{-1}) are block diagonal in
    // ldg x ldg blocks: the products with them skip the zero blocks
    int wgroup() const { return batched ? ldg : 0; }
    // the SpMM epilogue term of the batch: X = A C + d_g c (columns of g)
    SpmmEpi bepi(bool f64) const {
        SpmmEpi e;
        if (batched) {
            e.D = f64 ? (const void *)H->bd64 : (const void *)H->bd32;
            e.dld = ldg;
        }
        return e;
    }


    void alloc_small() {
        const size_t md = (size_t)m * m * sizeof(double);
        h.reset(new DevMem(ctx, ld * sizeof(double)));
        d.reset(new DevMem(ctx, ld * sizeof(double)));
        w.reset(new DevMem(ctx, ld * sizeof(double)));
        dots.reset(new DevMem(ctx, 4 * ld * sizeof(double)));
        dots2.reset(new DevMem(ctx, 4 * ld * sizeof(double)));
        Hp.reset(new DevMem(ctx, md));
        S.reset(new DevMem(ctx, md));
        Rinv.reset(new DevMem(ctx, md));
        Amat.reset(new DevMem(ctx, md));
        U.reset(new DevMem(ctx, md));
        Wp.reset(new DevMem(ctx, (size_t)ld * ld * sizeof(double)));
        gram_ws.reset(new DevMem(ctx, gram_workspace(n, m, batched ? ldg : 0)));
        dot_ws.reset(new DevMem(ctx, std::max({coldots_workspace(n, ld), spmm_partials_workspace(n, ld),
                                               rot_partials_workspace(n, m)})));
        chol_ws.reset(new DevMem(ctx, chol_workspace(m)));
        jac_ws.reset(new DevMem(ctx, jacobi_workspace(m)));
        info.reset(new DevMem(ctx, 64));
        state.reset(new DevMem(ctx, ng * sizeof(CgState)));
        st = (CgState *)state->ptr;
        TM_HIP(hipMemsetAsync(h->ptr, 0, ld * sizeof(double), s));
        TM_HIP(hipMemsetAsync(d->ptr, 0, ld * sizeof(double), s));
        TM_HIP(hipMemsetAsync(w->ptr, 0, ld * sizeof(double), s));
        // a batch's R^{-1} is block diagonal: the Cholesky writes only its
        // diagonal blocks, the rest stays zero from here on
        if (batched) TM_HIP(hipMemsetAsync(Rinv->ptr, 0, md, s));
        static_assert(kMaxBatch * sizeof(CgState) <= tm_ctx::kPinnedStates,
                      "the states of a batch must fit the pinned buffer");
        char *pin = (char *)ctx->pinned_buffer();
        st_host = (CgState *)pin;
        info_host = (int32_t *)(pin + tm_ctx::kPinnedStates);
        if (o.precondition == 2 && batched) {
            // each problem's own Gershgorin interval and degree-2 polynomial
            TM_REQUIRE(o.cheb_degree == 2, TM_ENOTSUP, "batched solves take the degree-2 polynomial");
            std::vector<double> ab(2 * ng);
            for (int g = 0; g < ng; ++g) {
                double th, de, sg;
                cheb_interval(H->b_lo[g], H->b_hi[g], sg, th, de);
                linear_cheb(sg, th, de, ab[2 * g], ab[2 * g + 1]);
            }
            gab.reset(new DevMem(ctx, ab.size() * sizeof(double)));
            TM_HIP(hipMemcpyAsync(gab->ptr, ab.data(), ab.size() * sizeof(double), hipMemcpyHostToDevice, s));
            TM_HIP(hipStreamSynchronize(s));
        } else if (o.precondition == 2) {
            cheb_interval(H->gersh_lo, H->gersh_hi, ch_sigma, ch_theta, ch_delta);
            linear_cheb(ch_sigma, ch_theta, ch_delta, ch_lin_a, ch_lin_b);
        }
        if (o.precondition == 1) {
            // Eq. 18 with M_ii = 1 / (H_ii - sigma), sigma = min(0, min_i H_ii - 1/2)
            // so that M is positive definite; formed on the device from H's diagonal
            TM_REQUIRE(H->diag != nullptr, TM_EINVAL, "matrix has no diagonal");
            M.reset(new DevMem(ctx, n * sizeof(double)));
            const double sigma = std::min(0.0, H->diag_min - 0.5);
            jacobi_preconditioner(s, n, H->diag, sigma, (double *)M->ptr);
        }
    }

    // shift sigma, centre theta and half-width delta of the Chebyshev
    // iteration on the Gershgorin interval [lo, hi] shifted by sigma
    void cheb_interval(double lo, double hi, double &sigma, double &theta, double &delta) const {
        sigma = lo - o.cheb_shift * (hi - lo);
        const double a = lo - sigma, b = hi - sigma;
        TM_REQUIRE(b > a && a > 0.0, TM_EINVAL, "degenerate Gershgorin interval");
        theta = 0.5 * (a + b);
        delta = 0.5 * (b - a);
    }
    // two Chebyshev steps as the linear polynomial z = a g + b H g:
    // d0 = g / theta = z1; r1 = g - (H - sigma) d0;
    // z2 = z1 + rho1 rho0 d0 + (2 rho1 / delta) r1, rho0 = delta / theta,
    // rho1 = 1 / (2 theta / delta - rho0)
    static void linear_cheb(double sigma, double theta, double delta, double &a, double &b) {
        const double rho0 = delta / theta, rho1 = 1.0 / (2.0 * theta / delta - rho0);
        const double cr = 2.0 * rho1 / delta;
        a = (1.0 + rho1 * rho0) / theta + cr * (1.0 + sigma / theta);
        b = -cr / theta;
    }

    size_t blk(bool f64) const { return (size_t)n * ld * (f64 ? 8 : 4); }

    void alloc_c(bool f64) {
        if (f64 && !C64) {
            C64.reset(new DevMem(ctx, blk(true)));
            Cn64.reset(new DevMem(ctx, blk(true)));
            X64.reset(new DevMem(ctx, blk(true)));
        }
        if (!f64 && !C32) {
            C32.reset(new DevMem(ctx, blk(false)));
            Cn32.reset(new DevMem(ctx, blk(false)));
            X32.reset(new DevMem(ctx, blk(false)));
        }
    }
    void free_c(bool f64) {
        if (f64) { C64.reset(); Cn64.reset(); X64.reset(); }
        else { C32.reset(); Cn32.reset(); X32.reset(); }
    }
    void alloc_g(bool f64) {
        if (G && g64_alloc == f64) return;
        G.reset(); Gp.reset(); P.reset(); Y.reset();
        Zc.reset(); Rc.reset(); Dc.reset();
        G.reset(new DevMem(ctx, blk(f64)));
        Gp.reset(new DevMem(ctx, blk(f64)));
        P.reset(new DevMem(ctx, blk(f64)));
        Y.reset(new DevMem(ctx, blk(f64)));
        if (o.precondition == 2) {
            Zc.reset(new DevMem(ctx, blk(f64)));
            Rc.reset(new DevMem(ctx, blk(f64)));
            Dc.reset(new DevMem(ctx, blk(f64)));
        }
        g64_alloc = f64;
    }
    void zero_g() {
        TM_HIP(hipMemsetAsync(Gp->ptr, 0, Gp->size, s));
        TM_HIP(hipMemsetAsync(P->ptr, 0, P->size, s));
    }

    void set_restart() { TM_HIP(hipMemsetD32Async((hipDeviceptr_t)&st->force_restart, 1, 1, s)); }

    // ---- orthonormalization (Fig. 4): Cn -> C
    template <typename TC, typename TS, typename TT>
    void orthonormalize(TC *Cin, TC *Cout) {
        gram<TC, TS>(s, n, m, Cin, Cin, nullptr, false, true, (double *)gram_ws->ptr, (double *)S->ptr,
                     true, nullptr, nullptr, 0, bcols(1.0));
        finish_orthonormalize<TC, TT>(Cin, Cout);
    }
    // Fig. 4 steps (2)-(4) once S = Cin^T Cin is in S: Cout = Cin R^{-1}
    template <typename TC, typename TT>
    void finish_orthonormalize(TC *Cin, TC *Cout) {
        chol_inverse(s, m, (double *)S->ptr, (double *)Rinv->ptr, (double *)chol_ws->ptr, (int32_t *)info->ptr,
                     chol_block());
        pad_matrix<TT>(s, m, (double *)Rinv->ptr, true, (TT *)Wp->ptr, (double *)d->ptr);
        rot<TC, TT, TC>(s, n, m, Cin, (TT *)Wp->ptr, EPI_TRMM, nullptr, (double *)d->ptr, Cout, nullptr,
                        nullptr, nullptr, nullptr, nullptr, wgroup());
    }

    // ---- Rayleigh-Ritz (Eq. 9): C <- C U, ascending Ritz values into w
    template <typename TC, typename TM>
    void rayleigh_ritz(TC *&C, TC *&Cn, TC *X) {
        const int nch = spmm_any(s, H, ld, C, X, is_f64<TC>(), 1, (double *)dot_ws->ptr, bepi(is_f64<TC>()));
        reduce_partials(s, 1, nch, ld, (double *)dot_ws->ptr, (double *)h->ptr);
        gram<TC, TM>(s, n, m, C, X, (double *)h->ptr, false, false, (double *)gram_ws->ptr, (double *)Hp->ptr,
                     true, nullptr, nullptr, 0, bcols(0.0));
        assemble_subspace_matrix(s, m, (double *)Hp->ptr, (double *)h->ptr, (double *)Amat->ptr);
        jacobi_eig(s, m, (double *)Amat->ptr, (double *)U->ptr, (double *)w->ptr, (double *)jac_ws->ptr,
                   (int32_t *)info->ptr + 1, ldg, mg);
        pad_matrix<TM>(s, m, (double *)U->ptr, false, (TM *)Wp->ptr, nullptr);
        rot<TC, TM, TC>(s, n, m, C, (TM *)Wp->ptr, EPI_NONE, nullptr, nullptr, Cn, nullptr, nullptr,
                        nullptr, nullptr, nullptr, wgroup());
        std::swap(C, Cn);
        ++rotations;
    }

    // ---- Z = M G with the polynomial M = p(H - sigma I) (Eq. 18): the
    // Chebyshev iteration for (H - sigma I) z = g from z = 0, in TG (G's
    // precision: single precision whenever G is stored in FP32, Sec. 4);
    // T is a free block for H d
    template <typename TG>
    void precondition_poly(const TG *Gv, TG *Z, TG *R, TG *D, TG *T) {
        const int64_t count = n * ld;
        cheb_init<TG>(s, count, Gv, 1.0 / ch_theta, D, Z);
        const double s1 = ch_theta / ch_delta;
        double rho = 1.0 / s1;
        const TG *r_in = Gv;
        for (int k = 1; k < o.cheb_degree; ++k) {
            spmm_any(s, H, ld, D, T, is_f64<TG>(), 0, nullptr, bepi(is_f64<TG>()));
            const double rho_new = 1.0 / (2.0 * s1 - rho);
            cheb_step<TG>(s, count, T, r_in, R, D, Z, ch_sigma, rho_new * rho, 2.0 * rho_new / ch_delta);
            r_in = R;
            rho = rho_new;
        }
    }

    // ---- one CG iteration (Fig. 1) with Algorithm-2 (Fig. 2).  TC: storage of
    // C and X; TG: of G, G_prev, P, Y; TMH: matrix cores of H' and C H';
    // TMS: of S = C^T C; TT: of the TRMM's C R' (Eq. 13)
    template <typename TC, typename TG, typename TMH, typename TMS, typename TT>
    void iterate(TC *&C, TC *&Cn, TC *X, bool rotate, double *hist_dev) {
        if (rotate) {
            // the rotation keeps C's own precision (FP64 C stays FP64-accurate)
            rayleigh_ritz<TC, TC>(C, Cn, X);
            if (o.transport) {
                // E(C U) = E(C) and G(C U) = G(C) U (Sec. 2.1): the previous
                // direction and gradient carried into the rotated basis keep
                // the Polak-Ribiere traces unchanged, so CG continues
                pad_matrix<TG>(s, m, (double *)U->ptr, false, (TG *)Wp->ptr, nullptr);
                rot<TG, TG, TG>(s, n, m, (TG *)P->ptr, (TG *)Wp->ptr, EPI_NONE, nullptr, nullptr, (TG *)Y->ptr,
                                nullptr, nullptr, nullptr, nullptr, nullptr, wgroup());
                std::swap(P, Y);
                rot<TG, TG, TG>(s, n, m, (TG *)Gp->ptr, (TG *)Wp->ptr, EPI_NONE, nullptr, nullptr, (TG *)G->ptr,
                                nullptr, nullptr, nullptr, nullptr, nullptr, wgroup());
                std::swap(G, Gp);
            } else {
                set_restart();
            }
        }
        TG *Gv = (TG *)G->ptr, *Gpv = (TG *)Gp->ptr, *Pv = (TG *)P->ptr, *Yv = (TG *)Y->ptr;
        const double *Mv = M ? (const double *)M->ptr : nullptr;
        // (1)-(3): X = HC with h = diag(C^T X) fused into the SpMM
        {
            const int nch = spmm_any(s, H, ld, C, X, is_f64<TC>(), 1, (double *)dot_ws->ptr, bepi(is_f64<TC>()));
            reduce_partials(s, 1, nch, ld, (double *)dot_ws->ptr, (double *)h->ptr);
        }
        // (5)-(6): H' = C^T (X - C H_D), diag(H') = 0; X' = X - C H_D is formed
        // in C's precision while staged and kept, rounded once to the matrix-core
        // precision, in Y (free until the line step) for step (7).  C is
        // orthonormal here, so H' = C^T H C - H_D is symmetric: only its upper
        // block tiles are computed and mirrored (the difference from the full
        // product, (C^T C - I) H_D, lies in span(C) and leaves E unchanged)
        // X' can be kept only where the direction blocks have the matrix-core
        // precision; MP1 (FP64 products, FP32 G) forms X' again in the
        // gradient's epilogue from X, C and h (EPI_GRAD)
        constexpr bool keep_xs = std::is_same<TG, TMH>::value;
        TMH *Xs = nullptr;
        if (!is_f64<TC>() && bf16_bulk) {
            gram_bf16x3<TC>(s, n, m, C, X, (double *)h->ptr, true, (double *)gram_ws->ptr, (double *)Hp->ptr);
            pad_matrix<TMH>(s, m, (double *)Hp->ptr, false, (TMH *)Wp->ptr, nullptr);
        } else if constexpr (keep_xs) {
            Xs = reinterpret_cast<TMH *>(Yv);
            gram<TC, TMH>(s, n, m, C, X, (double *)h->ptr, true, true, (double *)gram_ws->ptr,
                          (double *)Hp->ptr, true, Xs, (TMH *)Wp->ptr, 0, bcols(0.0));
        } else {
            gram<TC, TMH>(s, n, m, C, X, (double *)h->ptr, true, true, (double *)gram_ws->ptr,
                          (double *)Hp->ptr, true, nullptr, (TMH *)Wp->ptr, 0, bcols(0.0));
        }
        // (7): G = -2 (X' - C H'); the reduction above stored H' padded in TMH
        // with the traces for Eq. 8 and the descent test fused into the
        // epilogue (the polynomial M forms its own g.z and g_prev.z below, so
        // G_prev is not read here)
        {
            const TG *gp_dots = o.precondition == 2 ? nullptr : Gpv;
            const int nch = rot<TC, TMH, TG>(s, n, m, C, (TMH *)Wp->ptr, Xs ? EPI_GRADX : EPI_GRAD, X,
                                             (double *)h->ptr, Gv, gp_dots, Pv, Mv,
                                             (double *)dot_ws->ptr, Xs, wgroup());
            reduce_partials(s, 4, nch, ld, (double *)dot_ws->ptr, (double *)dots->ptr);
        }
        // the polynomial M: Z = M G, and the traces tr(G^T Z), tr(G_prev^T Z)
        // of the M-weighted Eq. 8 in place of the fused diagonal ones
        TG *Zv = nullptr;
        if (o.precondition == 2) {
            Zv = (TG *)Zc->ptr;
            if (o.cheb_degree == 2 && spmm_fast_path(H->is_stencil, H->st, ld, is_f64<TG>())) {
                // two Chebyshev steps are the linear polynomial a I + b H: one
                // SpMM with an affine epilogue, which also forms g.z and
                // g_prev.z
                SpmmEpi epi = bepi(is_f64<TG>());
                epi.affine = 1;
                epi.a = ch_lin_a;
                epi.b = ch_lin_b;
                epi.gab = gab ? (const double *)gab->ptr : nullptr;
                epi.E = Gpv;
                const int nch = spmm_any(s, H, ld, Gv, Zv, is_f64<TG>(), 3, (double *)dot_ws->ptr, epi);
                reduce_partials(s, 2, nch, ld, (double *)dot_ws->ptr, (double *)dots->ptr + ld);
            } else {
                TM_REQUIRE(!batched, TM_ENOTSUP, "batched solves need the fused degree-2 polynomial");
                precondition_poly<TG>(Gv, Zv, (TG *)Rc->ptr, (TG *)Dc->ptr, Yv);
                DotArgs<TG> a;
                a.nprod = 2;
                a.a[0] = Gv; a.b[0] = Zv;
                a.a[1] = Gpv; a.b[1] = Zv;
                coldots<TG>(s, n, ld, a, (double *)dot_ws->ptr, (double *)dots->ptr + ld);
            }
        }
        cg_control_gamma(s, mg, ld, (double *)h->ptr, (double *)dots->ptr, st, hist_dev, ng, ldg);
        // P = M G + gamma P
        if (Zv) p_update<TG, TG>(s, n, ld, Zv, nullptr, st, Pv, ldg);
        else p_update<TG, TG>(s, n, ld, Gv, Mv, st, Pv, ldg);
        // line step: Y = HP with p.y and p.p fused into the SpMM
        {
            const int nch = spmm_any(s, H, ld, Pv, Yv, is_f64<TG>(), 2, (double *)dot_ws->ptr, bepi(is_f64<TG>()));
            reduce_partials(s, 2, nch, ld, (double *)dot_ws->ptr, (double *)dots2->ptr);
        }
        cg_control_alpha(s, mg, ld, (double *)h->ptr, (double *)dots2->ptr, st, ng, ldg);
        // C_{i+1} = orthonormalize(C_i + alpha P): the update is formed inside
        // the Gram S = (C + alpha P)^T (C + alpha P), which also stores it
        gram_update<TC, TMS, TG>(s, n, m, C, Pv, st, Cn, (double *)gram_ws->ptr, (double *)S->ptr, bcols(1.0));
        finish_orthonormalize<TC, TT>(Cn, C);
        std::swap(G, Gp);
    }

    // ---- the generalized problem H x = lambda S x (Sec. 2.1), all FP64
    // Fig. 4 in the S inner product: Z = S Cin, Sg = Cin^T Z = R^T R,
    // Cout = Cin R^{-1}
    void orthonormalize_gen(double *Cin, double *Cout) {
        double *Z = (double *)Z64->ptr;
        spmm_any(s, Smat, ld, Cin, Z, true);
        gram<double, double>(s, n, m, Cin, Z, nullptr, false, false, (double *)gram_ws->ptr,
                             (double *)S->ptr);
        finish_orthonormalize<double, double>(Cin, Cout);
    }
    // Eq. 9 with an S-orthonormal C: A = C^T H C (the full product: H' from
    // C^T (X - C H_D) would need C^T C = I), A = U diag(w) U^T, C <- C U
    // keeps C^T S C = I
    void rayleigh_ritz_gen(double *&C, double *&Cn, double *X) {
        const int nch = spmm_any(s, H, ld, C, X, true, 1, (double *)dot_ws->ptr);
        reduce_partials(s, 1, nch, ld, (double *)dot_ws->ptr, (double *)h->ptr);
        gram<double, double>(s, n, m, C, X, nullptr, false, false, (double *)gram_ws->ptr,
                             (double *)Hp->ptr);
        assemble_subspace_matrix(s, m, (double *)Hp->ptr, (double *)h->ptr, (double *)Amat->ptr);
        jacobi_eig(s, m, (double *)Amat->ptr, (double *)U->ptr, (double *)w->ptr, (double *)jac_ws->ptr,
                   (int32_t *)info->ptr + 1);
        pad_matrix<double>(s, m, (double *)U->ptr, false, (double *)Wp->ptr, nullptr);
        rot<double, double, double>(s, n, m, C, (double *)Wp->ptr, EPI_NONE, nullptr, nullptr, Cn);
        std::swap(C, Cn);
        ++rotations;
    }
    // One CG iteration for H x = lambda S x: Algorithm-2 in the S metric
    // (X = HC, Z = SC, h = diag(C^T X), X' = X - Z H_D, H' = C^T X' with
    // diag(H') := 0, G = -2 (X' - Z H')), the Polak-Ribiere step, the line
    // step with S-norms (Y = HP, W = SP), C + alpha P and Fig. 4 in the S
    // inner product.
    void iterate_gen(double *&C, double *&Cn, double *X, bool rotate, double *hist_dev) {
        if (rotate) {
            rayleigh_ritz_gen(C, Cn, X);
            if (o.transport) {
                rot<double, double, double>(s, n, m, (double *)P->ptr, (double *)Wp->ptr, EPI_NONE, nullptr,
                                            nullptr, (double *)Y->ptr);
                std::swap(P, Y);
                rot<double, double, double>(s, n, m, (double *)Gp->ptr, (double *)Wp->ptr, EPI_NONE, nullptr,
                                            nullptr, (double *)G->ptr);
                std::swap(G, Gp);
            } else {
                set_restart();
            }
        }
        double *Gv = (double *)G->ptr, *Gpv = (double *)Gp->ptr, *Pv = (double *)P->ptr,
               *Yv = (double *)Y->ptr, *Z = (double *)Z64->ptr, *W = (double *)W64->ptr;
        const double *Mv = M ? (const double *)M->ptr : nullptr;
        double *dw = (double *)dot_ws->ptr;
        int nch = spmm_any(s, H, ld, C, X, true, 1, dw);
        reduce_partials(s, 1, nch, ld, dw, (double *)h->ptr);
        spmm_any(s, Smat, ld, C, Z, true);
        // X' in Y (free until the line step)
        shift_block(s, n, ld, X, Z, (double *)h->ptr, Yv);
        gram<double, double>(s, n, m, C, Yv, nullptr, true, false, (double *)gram_ws->ptr,
                             (double *)Hp->ptr, true, nullptr, (double *)Wp->ptr);
        nch = rot<double, double, double>(s, n, m, Z, (double *)Wp->ptr, EPI_GRADX, X, (double *)h->ptr, Gv,
                                          Gpv, Pv, Mv, dw, Yv);
        reduce_partials(s, 4, nch, ld, dw, (double *)dots->ptr);
        cg_control_gamma(s, m, ld, (double *)h->ptr, (double *)dots->ptr, st, hist_dev);
        p_update<double, double>(s, n, ld, Gv, Mv, st, Pv);
        // line step: p.(HP) and p.(SP), the S-norms of the columns of P
        double *d2 = (double *)dots2->ptr;
        nch = spmm_any(s, H, ld, Pv, Yv, true, 1, dw);
        reduce_partials(s, 1, nch, ld, dw, d2);
        nch = spmm_any(s, Smat, ld, Pv, W, true, 1, dw);
        reduce_partials(s, 1, nch, ld, dw, d2 + ld);
        cg_control_alpha(s, m, ld, (double *)h->ptr, d2, st);
        update_block<double>(s, n * ld, C, Pv, st, Cn);
        orthonormalize_gen(Cn, C);
        std::swap(G, Gp);
    }

    void reset_state(int gate, int hist_len) {
        std::vector<CgState> init(ng);
        for (int g = 0; g < ng; ++g) {
            CgState &c = init[g];
            c = CgState{};
            c.tol = tol;
            c.rise_tol = o.rise_tol;
            c.switch_tol = switch_g[g];
            c.stall_tol = o.stall_tol > 0 ? o.stall_tol : 1e-7;
            c.stall_window = gate ? 25 : 0;
            c.history_len = hist_len;
            c.phase_gate = gate;
        }
        TM_HIP(hipMemcpyAsync(st, init.data(), ng * sizeof(CgState), hipMemcpyHostToDevice, s));
        TM_HIP(hipStreamSynchronize(s));
    }

    // the host's view of the controller states after a poll
    struct View {
        int it = 0;                 // iterations of the furthest problem
        bool nan = false;           // any problem saw NaN/Inf
        bool all_done = true;       // every problem converged
        bool all_stopped = true;    // every problem converged or ended its phase
        double E = 0.0, rho = 0.0;  // sum of the energies, largest rho
    };
    View poll() {
        TM_HIP(hipMemcpyAsync(st_host, st, ng * sizeof(CgState), hipMemcpyDeviceToHost, s));
        TM_HIP(hipMemcpyAsync(info_host, info->ptr, 16, hipMemcpyDeviceToHost, s));
        TM_HIP(hipStreamSynchronize(s));
        if (info_host[0] != 0)
            throw Error{TM_ENOTSPD, "C^T C is not positive definite (pivot " + std::to_string(info_host[0]) + ")"};
        View v;
        for (int g = 0; g < ng; ++g) {
            const CgState &c = st_host[g];
            v.it = std::max(v.it, (int)c.it);
            v.nan |= c.nan_seen != 0;
            v.all_done &= c.done != 0;
            v.all_stopped &= c.done != 0 || c.phase_end != 0;
            v.E += c.E;
            v.rho = std::max(v.rho, c.rho);
        }
        return v;
    }
    // next phase: every problem that is not converged continues, with the
    // phase gate and stall window cleared (have_prev = 0 restarts CG)
    void next_phase_state(bool restart_cg) {
        std::vector<CgState> cur(st_host, st_host + ng);
        for (CgState &c : cur) {
            c.phase_end = 0;
            c.phase_gate = 0;
            c.stall_window = 0;
            c.window_it = 0;
            if (restart_cg) c.have_prev = 0;
        }
        TM_HIP(hipMemcpyAsync(st, cur.data(), ng * sizeof(CgState), hipMemcpyHostToDevice, s));
        TM_HIP(hipStreamSynchronize(s));
    }

    double auto_switch_tol(double dmin, double dmax, int mcols) const {
        // rounding floor of rho ~ u * ||H|| * sqrt(m) for the bulk phase's
        // unit roundoff u (FP32 2^-24; two-term BF16 about 2^-17); leave the
        // bulk phase a little above it (16x: measured best at 48^3, m = 256)
        const double hnorm = std::max(std::fabs(dmax), std::fabs(dmin)) * 2.0;
        if (bf16_bulk) return 4.0 * 7.63e-6 * hnorm * std::sqrt((double)mcols);
        return 16.0 * 5.96e-8 * hnorm * std::sqrt((double)mcols);
    }

    // res: ng results (one per problem); eig_out: ng * mg values, problem g
    // at g * mg
    tm_status run(const double *C0, double *C_out, double *eig_out, tm_result *res,
                  double *hist_host, int hist_len) {
        auto t0 = std::chrono::steady_clock::now();
        // graphs cannot be recorded on the legacy default stream: then the
        // solve runs on a stream of its own, after the caller's prior work
        struct OwnStream {
            hipStream_t st = nullptr;
            ~OwnStream() {
                if (st) {
                    (void)hipStreamSynchronize(st);
                    (void)hipStreamDestroy(st);
                }
            }
        } own;
        if (o.graphs && s == nullptr) {
            TM_HIP(hipStreamCreateWithFlags(&own.st, hipStreamNonBlocking));
            hipEvent_t ev;
            TM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            TM_HIP(hipEventRecord(ev, nullptr));
            TM_HIP(hipStreamWaitEvent(own.st, ev, 0));
            (void)hipEventDestroy(ev);
            s = own.st;
        }
        alloc_small();
        int hl = (o.history && hist_host) ? hist_len : 0;
        if (hl > 0) hist.reset(new DevMem(ctx, (size_t)2 * hl * sizeof(double)));
        double *hist_dev = hl > 0 ? (double *)hist->ptr : nullptr;
        TM_HIP(hipMemsetAsync(info->ptr, 0, 64, s));

        const int prec = o.precision;
        const bool mixed = prec == TM_MIXED || prec == TM_MIXED_BF16;
        const bool mp2_mp1 = prec == TM_MP2_MP1;
        bf16_bulk = prec == TM_MIXED_BF16 || prec == TM_FULL_BF16;
        TM_REQUIRE(!batched || (!bf16_bulk && o.precondition != 1 && hl == 0 && !Smat), TM_ENOTSUP,
                   "batched solves take no BF16 policy, diagonal preconditioner, history or S");
        Phase ph = phase_of((mixed || prec == TM_FULL_BF16) ? TM_FULL_SP : (mp2_mp1 ? TM_MP2 : prec));
        alloc_c(ph.c64);
        alloc_g(ph.g64);
        // no start block given: the seeded standard normal block (Sec. 3:
        // random numbers, then orthonormalization)
        std::unique_ptr<DevMem> c0_own;
        if (!C0) {
            c0_own.reset(new DevMem(ctx, blk(true)));
            if (batched) {
                // problem g: the block tm_random_block gives with seed + g
                for (int g = 0; g < ng; ++g)
                    random_block(s, n, mg, o.seed + (uint64_t)g, (double *)c0_own->ptr, ldg, ld, g * ldg);
            } else {
                random_block(s, n, m, o.seed, (double *)c0_own->ptr);
            }
            C0 = (const double *)c0_own->ptr;
        }
        // start block -> C (cast), orthonormalize
        if (ph.c64) {
            TM_HIP(hipMemcpyAsync(Cn64->ptr, C0, blk(true), hipMemcpyDeviceToDevice, s));
        } else {
            convert_block<double, float>(s, n * ld, C0, (float *)Cn32->ptr);
        }
        const bool gate = mixed || mp2_mp1 || prec == TM_FULL_SP || prec == TM_FULL_BF16;
        switch_g.assign(ng, o.switch_tol);
        for (int g = 0; g < ng; ++g)
            if (!(o.switch_tol > 0))
                switch_g[g] = batched ? auto_switch_tol(H->b_diag_min[g], H->b_diag_max[g], mg)
                                      : auto_switch_tol(H->diag_min, H->diag_max, m);
        reset_state(gate ? 1 : 0, hl);
        zero_g();

        double *c64 = C64 ? (double *)C64->ptr : nullptr, *cn64 = Cn64 ? (double *)Cn64->ptr : nullptr;
        float *c32 = C32 ? (float *)C32->ptr : nullptr, *cn32 = Cn32 ? (float *)Cn32->ptr : nullptr;
        if (Smat) {
            Z64.reset(new DevMem(ctx, blk(true)));
            W64.reset(new DevMem(ctx, blk(true)));
            orthonormalize_gen(cn64, c64);
        } else if (ph.c64) {
            orthonormalize<double, double, double>(cn64, c64);
        } else {
            orthonormalize<float, float, float>(cn32, c32);
        }
        TM_HIP(hipStreamSynchronize(s));
        c0_own.reset();
        const auto t_loop = std::chrono::steady_clock::now();
        auto t_switch = t_loop;
        bool switched = false;

        int it_host = 0;        // active iterations known to the host
        std::vector<int> iters_sp(ng, 0);
        View view;
        bool sp_phase = !ph.c64;
        bool first_phase = true;   // MP2 part of TM_MP2_MP1
        const int kcheck = std::max(1, o.k_check);
        auto step = [&](bool rotate) {
            if (Smat) iterate_gen(c64, cn64, (double *)X64->ptr, rotate, hist_dev);
            else if (!ph.c64) iterate<float, float, float, float, float>(c32, cn32, (float *)X32->ptr, rotate, hist_dev);
            else if (ph.g64) iterate<double, double, double, double, double>(c64, cn64, (double *)X64->ptr, rotate, hist_dev);
            else if (ph.mh64) iterate<double, float, double, double, float>(c64, cn64, (double *)X64->ptr, rotate, hist_dev);
            else iterate<double, float, float, double, float>(c64, cn64, (double *)X64->ptr, rotate, hist_dev);
        };
        while (true) {
            int it_dev_done = 0;
            const int nb = std::min(kcheck, o.max_iter - it_host);
            bool any_rotation = false;
            for (int b = 0; b < nb; ++b) {
                const int i = it_host + b;
                any_rotation |= o.k_rot > 0 && i > 0 && (i % o.k_rot) == 0;
            }
            if (o.graphs && nb == kcheck && !any_rotation) {
                // a batch of k_check iterations without a rotation is the same
                // launch sequence every time for the same buffers: replay it
                // from a captured HIP graph (no memset nodes are recorded)
                const GraphKey key{c32, c64, G->ptr, Gp->ptr, P->ptr, Y->ptr, ph.id()};
                hipGraphExec_t exec = nullptr;
                for (auto &kv : graphs)
                    if (kv.first == key) exec = kv.second;
                if (!exec) {
                    // recording runs the host side of the batch (buffer roles
                    // advance as they will on the device) but not the kernels
                    hipGraph_t g = nullptr;
                    TM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                    for (int b = 0; b < nb; ++b) step(false);
                    TM_HIP(hipStreamEndCapture(s, &g));
                    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    TM_HIP(e);
                    graphs.push_back({key, exec});
                } else if (nb % 2) {
                    std::swap(G, Gp);   // the roles a replay leaves behind
                }
                TM_HIP(hipGraphLaunch(exec, s));
                it_dev_done = nb;
            } else {
                for (int b = 0; b < nb; ++b) {
                    const int i = it_host + b;
                    step(o.k_rot > 0 && i > 0 && (i % o.k_rot) == 0);
                    it_dev_done = b + 1;
                }
            }
            view = poll();
            it_host = view.it;
            if (o.progress) o.progress(view.it, view.E, view.rho, switched ? 1 : 0, o.progress_user);
            if (view.nan) throw Error{TM_ENAN, "NaN or Inf in the energy or gradient"};
            if (view.all_done) break;
            // a batched solve changes phase once every problem has ended the
            // phase (or converged); problems that ended it early take no steps
            // (alpha = 0) meanwhile
            if (view.all_stopped) {
                for (int g = 0; g < ng; ++g) iters_sp[g] = st_host[g].it;
                if (mp2_mp1 && first_phase) {
                    // MP2 done: MP1 from here on.  C, X and the FP32 G, G_prev, P
                    // keep their buffers and meaning, so CG continues
                    t_switch = std::chrono::steady_clock::now();
                    switched = true;
                    ph = phase_of(TM_MP1);
                    next_phase_state(false);
                    first_phase = false;
                    continue;
                }
                if (mixed && sp_phase) {
                    // FP32 bulk done: cast C up (exact), re-orthonormalize in FP64,
                    // restart CG under MP2 (Sec. 3: switch when the residual is small)
                    t_switch = std::chrono::steady_clock::now();
                    switched = true;
                    ph = phase_of(TM_MP2);
                    alloc_c(true);
                    c64 = (double *)C64->ptr;
                    cn64 = (double *)Cn64->ptr;
                    convert_block<float, double>(s, n * ld, c32, cn64);
                    free_c(false);
                    c32 = cn32 = nullptr;
                    alloc_g(ph.g64);
                    zero_g();
                    orthonormalize<double, double, double>(cn64, c64);
                    next_phase_state(true);
                    sp_phase = false;
                    continue;
                }
                break;   // FULL_SP: the FP32 phase ends the solve
            }
            if (it_host >= o.max_iter || it_dev_done == 0) break;
        }
        std::vector<int> iterations(ng);
        bool all_converged = true;
        for (int g = 0; g < ng; ++g) {
            const CgState &c = st_host[g];
            iterations[g] = c.done ? c.it - 1 : c.it;
            all_converged &= c.done != 0;
        }
        const auto t_iter_end = std::chrono::steady_clock::now();
        // one-phase policies (and a two-phase policy that never switched)
        // count every iteration as the first phase's
        if (!switched) {
            iters_sp = iterations;
            t_switch = t_iter_end;
        }

        // ---- final FP64 Rayleigh-Ritz, residuals and orthonormality
        if (!c64) {
            alloc_c(true);
            c64 = (double *)C64->ptr;
            cn64 = (double *)Cn64->ptr;
            convert_block<float, double>(s, n * ld, c32, c64);
            free_c(false);
        }
        double *X = (double *)X64->ptr;
        if (Smat) rayleigh_ritz_gen(c64, cn64, X);
        else rayleigh_ritz<double, double>(c64, cn64, X);
        --rotations;   // the final one is not a subspace rotation of the iteration
        spmm_any(s, H, ld, c64, X, true, 0, nullptr, bepi(true));
        // residuals ||H c_j - lambda_j S c_j|| and C^T S C - I (S = I for the
        // standard problem)
        const double *SC = c64;
        if (Smat) {
            spmm_any(s, Smat, ld, c64, (double *)Z64->ptr, true);
            SC = (const double *)Z64->ptr;
        }
        {
            DotArgs<double> a;
            a.nprod = 1; a.kind = 1; a.a[0] = X; a.b[0] = SC; a.sc = (double *)w->ptr;
            coldots<double>(s, n, ld, a, (double *)dot_ws->ptr, (double *)dots->ptr);
        }
        // (unmasked: a batch's orthonormality is read from its diagonal blocks)
        gram<double, double>(s, n, m, c64, SC, nullptr, false, !Smat, (double *)gram_ws->ptr, (double *)S->ptr);
        std::vector<double> wv(m), res2(m), Sh((size_t)m * m);
        TM_HIP(hipMemcpyAsync(wv.data(), w->ptr, m * sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipMemcpyAsync(res2.data(), dots->ptr, m * sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipMemcpyAsync(Sh.data(), S->ptr, Sh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        if (C_out) TM_HIP(hipMemcpyAsync(C_out, c64, blk(true), hipMemcpyDeviceToDevice, s));
        if (eig_out) {
            // problem g's values are columns g * ldg .. g * ldg + mg - 1
            const int stride = batched ? ldg : m;
            TM_HIP(hipMemcpy2DAsync(eig_out, mg * sizeof(double), w->ptr, stride * sizeof(double),
                                    mg * sizeof(double), ng, hipMemcpyDeviceToDevice, s));
        }
        if (hl > 0) TM_HIP(hipMemcpyAsync(hist_host, hist_dev, (size_t)2 * hl * sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipStreamSynchronize(s));

        auto t1 = std::chrono::steady_clock::now();
        auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
            return std::chrono::duration<double>(b - a).count();
        };
        const int stride = batched ? ldg : m;
        for (int g = 0; g < ng; ++g) {
            const int c0 = g * stride;
            double eg = 0.0, mx = 0.0, fr = 0.0, orth = 0.0;
            for (int j = c0; j < c0 + mg; ++j) {
                eg += wv[j];
                mx = std::max(mx, std::sqrt(res2[j]));
                fr += res2[j];
            }
            for (int i = c0; i < c0 + mg; ++i)
                for (int j = c0; j < c0 + mg; ++j)
                    orth = std::max(orth, std::fabs(Sh[(size_t)i * m + j] - (i == j ? 1.0 : 0.0)));
            tm_result &r = res[g];
            const CgState &c = st_host[g];
            r.E_G = eg;
            r.rho = c.rho;
            r.max_residual = mx;
            r.frob_residual = std::sqrt(fr);
            r.orth_err = orth;
            r.seconds = secs(t0, t1);
            r.seconds_phase[0] = secs(t_loop, t_switch);
            r.seconds_phase[1] = secs(t_switch, t_iter_end);
            r.seconds_phase[2] = secs(t0, t_loop) + secs(t_iter_end, t1);
            r.iterations = iterations[g];
            r.iters_sp = iters_sp[g];
            r.iters_phase2 = iterations[g] - iters_sp[g];
            r.converged = c.done ? 1 : 0;
            r.restarts = c.restarts;
            r.rotations = rotations;
        }
        return all_converged ? TM_OK : TM_ENOCONV;
    }
};

Solver::Solver(tm_ctx *ctx, const tm_mat *H, int m, double tol, const tm_opts &o, const tm_mat *S)
    : impl_(new Impl(ctx, H, S, m, tol, o)) {}
Solver::~Solver() = default;
tm_status Solver::run(const double *C0, double *C_out, double *eig_out, tm_result *res,
                      double *hist, int hist_len) {
    return impl_->run(C0, C_out, eig_out, res, hist, hist_len);
}

}  // namespace tmin
