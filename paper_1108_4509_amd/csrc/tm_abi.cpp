// extern "C" entry points declared in include/tracemin.h.  Validates
// arguments, owns the matrix uploads, and converts internal errors into
// tm_status codes (no exception leaves this file).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <vector>

#include "tm_solver.h"

using namespace tmin;

// Device memory of tm_gram_noalloc: the padded h and the split-K partials of
// one Gram product.  Every device the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Called with `device` current (from tm_create).
void bind_scratch(int device) {
    TM_REQUIRE(device >= 0 && device < kMaxDevices, TM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    TM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TM_REQUIRE(p != nullptr, TM_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = p;
}

void *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

thread_local std::string g_last_error;

template <typename F>
tm_status guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return TM_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return TM_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return TM_EINVAL;
    }
}

void use_device(const tm_ctx *ctx) {
    TM_REQUIRE(ctx != nullptr, TM_EINVAL, "null context");
    TM_HIP(hipSetDevice(ctx->device));
}

void sync(const tm_ctx *ctx) { TM_HIP(hipStreamSynchronize(ctx->stream)); }

template <typename T>
T *upload(tm_ctx *ctx, const T *host, size_t count) {
    T *d = (T *)ctx->dalloc(count * sizeof(T) + 16);
    TM_REQUIRE(d != nullptr, TM_ENOMEM, "device allocation failed");
    TM_HIP(hipMemcpyAsync(d, host, count * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    return d;
}

void free_matrix_arrays(tm_mat *m) {
    tm_ctx *c = m->ctx;
    void *arrs[] = {m->rowptr, m->col, m->val64, m->val32, m->V64, m->V32, m->diag, m->bd64, m->bd32};
    for (void *p : arrs)
        if (p) c->dfree(p);
}

void check_block_args(const tm_ctx *ctx, int64_t n, int32_t m) {
    use_device(ctx);
    TM_REQUIRE(n >= 1, TM_EINVAL, "n must be positive");
    TM_REQUIRE(m >= 1 && m <= 4096, TM_EINVAL, "m must be in [1, 4096]");
    TM_REQUIRE(m <= n, TM_EINVAL, "m must not exceed n");
}

}  // namespace

void tmin::set_last_error(const std::string &msg) { g_last_error = msg; }

void *tm_ctx::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (custom_alloc) return alloc.alloc(bytes, alloc.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void *tm_ctx::pinned_buffer() {
    if (!pinned) TM_HIP(hipHostMalloc(&pinned, kPinnedBytes, hipHostMallocDefault));
    return pinned;
}

tm_ctx::~tm_ctx() {
    if (pinned) (void)hipHostFree(pinned);
}

void tm_ctx::dfree(void *p) {
    if (!p) return;
    if (custom_alloc) alloc.free(p, alloc.user);
    else (void)hipFree(p);
}

extern "C" {

int32_t tm_leading_dim(int32_t m) { return leading_dim(m); }

const char *tm_last_error(void) { return g_last_error.c_str(); }

const char *tm_status_string(int32_t status) {
    switch (status) {
    case TM_OK: return "ok";
    case TM_EINVAL: return "invalid argument";
    case TM_ENOMEM: return "out of device memory";
    case TM_ENOTSPD: return "C^T C not positive definite";
    case TM_ENOCONV: return "not converged within max_iter";
    case TM_ENAN: return "NaN or Inf encountered";
    case TM_EDEVICE: return "HIP runtime error";
    case TM_ENOTSUP: return "not supported";
    case TM_EAGAIN: return "not finished yet";
    default: return "unknown status";
    }
}

tm_status tm_create(int32_t device, const tm_allocator *alloc, void *stream, tm_ctx **out) {
    return guarded([&]() {
        TM_REQUIRE(out != nullptr, TM_EINVAL, "out is null");
        *out = nullptr;
        int count = 0;
        TM_HIP(hipGetDeviceCount(&count));
        TM_REQUIRE(device >= 0 && device < count, TM_EINVAL, "no such device");
        TM_HIP(hipSetDevice(device));
        bind_scratch(device);
        tm_ctx *c = new tm_ctx;
        c->device = device;
        c->stream = (hipStream_t)stream;
        if (alloc) {
            if (!alloc->alloc || !alloc->free) {
                delete c;
                throw Error{TM_EINVAL, "allocator needs alloc and free"};
            }
            c->alloc = *alloc;
            c->custom_alloc = true;
        }
        *out = c;
        return TM_OK;
    });
}

void tm_destroy(tm_ctx *ctx) { delete ctx; }

void tm_opts_default(tm_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = TM_FULL_DP;
    o->max_iter = 20000;
    o->k_rot = 50;
    o->k_check = 10;
    o->precondition = 0;
    o->history = 0;
    o->transport = 1;
    o->graphs = 0;
    o->switch_tol = 0.0;
    o->rise_tol = 1e-13;
    o->stall_tol = 0.0;
    o->seed = 0;
    o->cheb_degree = 2;
    o->cheb_shift = 0.02;
    o->progress = nullptr;
    o->progress_user = nullptr;
}

tm_status tm_set_matrix_csr(tm_ctx *ctx, int64_t n, const int64_t *rowptr_in, const int32_t *col_in,
                            const double *val_in, uint32_t flags, tm_mat **out) {
    return guarded([&]() {
        use_device(ctx);
        TM_REQUIRE(out && rowptr_in && col_in && val_in, TM_EINVAL, "null argument");
        *out = nullptr;
        TM_REQUIRE((flags & ~(TM_CHECK_SYMMETRY | TM_DEVICE_PTRS)) == 0, TM_EINVAL, "unknown flag bits");
        TM_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), TM_EINVAL, "n out of range");
        // device arrays are validated (and their FP32 copy and diagonal
        // formed) through a host copy; host arrays are used in place
        std::vector<int64_t> rp_h;
        std::vector<int32_t> col_h;
        std::vector<double> val_h;
        const int64_t *rowptr = rowptr_in;
        const int32_t *col = col_in;
        const double *val = val_in;
        if (flags & TM_DEVICE_PTRS) {
            rp_h.resize(n + 1);
            TM_HIP(hipMemcpy(rp_h.data(), rowptr_in, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
            TM_REQUIRE(rp_h[0] == 0 && rp_h[n] >= 0 && rp_h[n] < ((int64_t)1 << 40), TM_EINVAL,
                       "rowptr[0] must be 0 and rowptr[n] a valid count");
            col_h.resize(rp_h[n]);
            val_h.resize(rp_h[n]);
            TM_HIP(hipMemcpy(col_h.data(), col_in, rp_h[n] * sizeof(int32_t), hipMemcpyDeviceToHost));
            TM_HIP(hipMemcpy(val_h.data(), val_in, rp_h[n] * sizeof(double), hipMemcpyDeviceToHost));
            rowptr = rp_h.data();
            col = col_h.data();
            val = val_h.data();
        }
        TM_REQUIRE(rowptr[0] == 0, TM_EINVAL, "rowptr[0] must be 0");
        for (int64_t r = 0; r < n; ++r)
            TM_REQUIRE(rowptr[r + 1] >= rowptr[r], TM_EINVAL, "rowptr must be non-decreasing");
        const int64_t nnz = rowptr[n];
        std::vector<double> diag(n, 0.0);
        std::vector<float> v32(nnz);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                TM_REQUIRE(col[k] >= 0 && col[k] < n, TM_EINVAL, "column index out of range");
                TM_REQUIRE(std::isfinite(val[k]), TM_EINVAL, "non-finite matrix value");
                if (col[k] == r) diag[r] += val[k];
            }
        for (int64_t k = 0; k < nnz; ++k) v32[k] = (float)val[k];
        if (flags & TM_CHECK_SYMMETRY) {
            // H = H^T (Sec. 2.1): every row's entries, duplicates summed, must
            // equal the transposed ones; compared through the transpose built
            // by a counting sort on the columns
            std::vector<int64_t> tp(n + 1, 0);
            for (int64_t k = 0; k < nnz; ++k) ++tp[col[k] + 1];
            for (int64_t r = 0; r < n; ++r) tp[r + 1] += tp[r];
            std::vector<int32_t> tcol(nnz);
            std::vector<double> tval(nnz);
            std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
            for (int64_t r = 0; r < n; ++r)
                for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                    const int64_t d = fill[col[k]]++;
                    tcol[d] = (int32_t)r;
                    tval[d] = val[k];
                }
            // (a duplicated entry may be summed in another order on the two
            // sides: allowed to differ by a few units of rounding)
            std::vector<double> acc(n, 0.0), mag(n, 0.0);
            std::vector<int32_t> touched;
            for (int64_t r = 0; r < n; ++r) {
                touched.clear();
                for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                    acc[col[k]] += val[k];
                    mag[col[k]] += std::fabs(val[k]);
                    touched.push_back(col[k]);
                }
                for (int64_t k = tp[r]; k < tp[r + 1]; ++k) {
                    acc[tcol[k]] -= tval[k];
                    mag[tcol[k]] += std::fabs(tval[k]);
                    touched.push_back(tcol[k]);
                }
                for (int32_t c : touched) {
                    TM_REQUIRE(std::fabs(acc[c]) <= 4.0 * 2.220446049250313e-16 * mag[c], TM_EINVAL,
                               "matrix is not symmetric (row " + std::to_string(r) + ", column " +
                                   std::to_string(c) + ")");
                }
                for (int32_t c : touched) acc[c] = mag[c] = 0.0;
            }
        }
        tm_mat *m = new tm_mat;
        m->ctx = ctx;
        m->n = n;
        try {
            m->rowptr = upload(ctx, rowptr, n + 1);
            m->col = upload(ctx, col, nnz);
            m->val64 = upload(ctx, val, nnz);
            m->val32 = upload(ctx, v32.data(), nnz);
            m->diag = upload(ctx, diag.data(), n);
            sync(ctx);
        } catch (...) {
            free_matrix_arrays(m);
            delete m;
            throw;
        }
        m->diag_min = *std::min_element(diag.begin(), diag.end());
        m->diag_max = *std::max_element(diag.begin(), diag.end());
        // Gershgorin-type scale of ||H|| for the automatic switch tolerance
        double gmax = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) s += std::fabs(val[k]);
            gmax = std::max(gmax, s);
        }
        m->diag_max = std::max(m->diag_max, 0.5 * gmax);
        m->gersh_lo = 1e300;
        m->gersh_hi = -1e300;
        for (int64_t r = 0; r < n; ++r) {
            double off = 0.0;
            for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
                if (col[k] != r) off += std::fabs(val[k]);
            m->gersh_lo = std::min(m->gersh_lo, diag[r] - off);
            m->gersh_hi = std::max(m->gersh_hi, diag[r] + off);
        }
        m->csr.n = n;
        m->csr.nnz = nnz;
        m->csr.rowptr = m->rowptr;
        m->csr.col = m->col;
        m->csr.val64 = m->val64;
        m->csr.val32 = m->val32;
        *out = m;
        return TM_OK;
    });
}

tm_status tm_set_matrix_stencil(tm_ctx *ctx, const tm_stencil *s, tm_mat **out) {
    return guarded([&]() {
        use_device(ctx);
        TM_REQUIRE(out && s, TM_EINVAL, "null argument");
        *out = nullptr;
        TM_REQUIRE(s->ndim == 2 || s->ndim == 3, TM_EINVAL, "ndim must be 2 or 3");
        TM_REQUIRE(s->order == 2 || s->order == 4, TM_EINVAL, "order must be 2 or 4");
        TM_REQUIRE(std::isfinite(s->kinetic_scale), TM_EINVAL, "bad kinetic_scale");
        const int nz = s->ndim == 3 ? s->dims[2] : 1;
        TM_REQUIRE(s->dims[0] >= 1 && s->dims[1] >= 1 && nz >= 1, TM_EINVAL, "bad grid extents");
        const int64_t n = (int64_t)s->dims[0] * s->dims[1] * nz;
        TM_REQUIRE(n < ((int64_t)1 << 31), TM_EINVAL, "grid too large");
        tm_mat *m = new tm_mat;
        m->ctx = ctx;
        m->n = n;
        m->is_stencil = true;
        const double ks = s->kinetic_scale;
        StencilDev &d = m->st;
        d.ndim = s->ndim;
        d.nx = s->dims[0];
        d.ny = s->dims[1];
        d.nz = nz;
        d.order = s->order;
        d.periodic = s->periodic ? 1 : 0;
        if (s->order == 2) {
            d.c0 = s->ndim * 2.0 * ks;
            d.c1 = -ks;
            d.c2 = 0.0;
        } else {
            d.c0 = s->ndim * (30.0 / 12.0) * ks;
            d.c1 = -(16.0 / 12.0) * ks;
            d.c2 = (1.0 / 12.0) * ks;
        }
        std::vector<double> diag(n, d.c0);
        try {
            if (s->V) {
                std::vector<float> v32(n);
                for (int64_t r = 0; r < n; ++r) {
                    TM_REQUIRE(std::isfinite(s->V[r]), TM_EINVAL, "non-finite potential value");
                    v32[r] = (float)s->V[r];
                    diag[r] += s->V[r];
                }
                m->V64 = upload(ctx, s->V, n);
                m->V32 = upload(ctx, v32.data(), n);
                d.V64 = m->V64;
                d.V32 = m->V32;
            }
            m->diag = upload(ctx, diag.data(), n);
            sync(ctx);
        } catch (...) {
            free_matrix_arrays(m);
            delete m;
            throw;
        }
        m->diag_min = *std::min_element(diag.begin(), diag.end());
        const double off = s->ndim * (2.0 * std::fabs(d.c1) + 2.0 * std::fabs(d.c2));
        m->diag_max = std::max(*std::max_element(diag.begin(), diag.end()),
                               0.5 * (std::fabs(d.c0) + off));
        // Gershgorin bounds row by row, with the stencil's neighbours merged
        // as the matrix would hold them (wrapped offsets that meet on one
        // point are summed; a wrap onto the point itself adds to the diagonal)
        {
            const int ext[3] = {d.nx, d.ny, d.nz};
            std::vector<double> axis_off[3], axis_self[3];
            for (int ax = 0; ax < d.ndim; ++ax) {
                const int e = ext[ax];
                axis_off[ax].assign(e, 0.0);
                axis_self[ax].assign(e, 0.0);
                for (int c = 0; c < e; ++c) {
                    std::vector<std::pair<int, double>> tgt;
                    for (int o = -(d.order / 2); o <= d.order / 2; ++o) {
                        if (o == 0) continue;
                        int t = c + o;
                        if (d.periodic) t = ((t % e) + e) % e;
                        else if (t < 0 || t >= e) continue;
                        const double coef = (o == 1 || o == -1) ? d.c1 : d.c2;
                        bool merged = false;
                        for (auto &pr : tgt)
                            if (pr.first == t) { pr.second += coef; merged = true; }
                        if (!merged) tgt.push_back({t, coef});
                    }
                    for (auto &pr : tgt) {
                        if (pr.first == c) axis_self[ax][c] += pr.second;
                        else axis_off[ax][c] += std::fabs(pr.second);
                    }
                }
            }
            m->gersh_lo = 1e300;
            m->gersh_hi = -1e300;
            for (int64_t r = 0; r < n; ++r) {
                const int crd[3] = {(int)(r % d.nx), (int)((r / d.nx) % d.ny),
                                    d.ndim == 3 ? (int)(r / ((int64_t)d.nx * d.ny)) : 0};
                double dg = diag[r], of = 0.0;
                for (int ax = 0; ax < d.ndim; ++ax) {
                    dg += axis_self[ax][crd[ax]];
                    of += axis_off[ax][crd[ax]];
                }
                m->gersh_lo = std::min(m->gersh_lo, dg - of);
                m->gersh_hi = std::max(m->gersh_hi, dg + of);
            }
        }
        *out = m;
        return TM_OK;
    });
}

void tm_free_matrix(tm_mat *mat) {
    if (!mat) return;
    (void)hipSetDevice(mat->ctx->device);
    (void)hipStreamSynchronize(mat->ctx->stream);
    free_matrix_arrays(mat);
    delete mat;
}

int64_t tm_matrix_rows(const tm_mat *mat) { return mat ? mat->n : -1; }

tm_status tm_solve(tm_ctx *ctx, const tm_mat *H, int32_t m, double tol, const tm_opts *opts,
                   const double *C0, double *C_out, double *eig_out, tm_result *res,
                   double *history, int32_t history_len) {
    return guarded([&]() {
        TM_REQUIRE(H && res, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(H->ctx == ctx, TM_EINVAL, "matrix belongs to another context");
        TM_REQUIRE(H->batch_k == 0, TM_EINVAL, "a batch matrix is solved by tm_solve_batch");
        TM_REQUIRE(tol > 0.0 && std::isfinite(tol), TM_EINVAL, "tol must be positive");
        TM_REQUIRE(m <= 2048, TM_ENOTSUP, "m > 2048 is not supported");
        tm_opts o;
        if (opts) o = *opts; else tm_opts_default(&o);
        TM_REQUIRE(o.max_iter >= 0, TM_EINVAL, "max_iter must be >= 0");
        TM_REQUIRE(o.precision >= TM_FULL_DP && o.precision <= TM_MP2_MP1, TM_EINVAL, "unknown precision");
        TM_REQUIRE(history_len >= 0, TM_EINVAL, "history_len must be >= 0");
        TM_REQUIRE(o.graphs == 0 || o.graphs == 1, TM_EINVAL, "tm_opts.graphs must be 0 or 1");
        TM_REQUIRE(o.precondition >= 0 && o.precondition <= 2, TM_EINVAL, "tm_opts.precondition must be 0, 1 or 2");
        TM_REQUIRE(o.precondition != 2 || (o.cheb_degree >= 1 && o.cheb_degree <= 64 &&
                                           o.cheb_shift > 0.0 && std::isfinite(o.cheb_shift)),
                   TM_EINVAL, "polynomial preconditioner: cheb_degree in [1, 64], cheb_shift > 0");
        std::memset(res, 0, sizeof(*res));
        Solver solver(ctx, H, m, tol, o);
        return solver.run(C0, C_out, eig_out, res, history, history_len);
    });
}

tm_status tm_solve_generalized(tm_ctx *ctx, const tm_mat *H, const tm_mat *S, int32_t m, double tol,
                               const tm_opts *opts, const double *C0, double *C_out, double *eig_out,
                               tm_result *res, double *history, int32_t history_len) {
    return guarded([&]() {
        TM_REQUIRE(H && S && res, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(H->batch_k == 0 && S->batch_k == 0, TM_EINVAL, "batch matrices take tm_solve_batch");
        TM_REQUIRE(H->ctx == ctx && S->ctx == ctx, TM_EINVAL, "matrix belongs to another context");
        TM_REQUIRE(S->n == H->n, TM_EINVAL, "H and S differ in size");
        TM_REQUIRE(S->diag_min > 0.0, TM_EINVAL, "S has a diagonal entry <= 0: not positive definite");
        TM_REQUIRE(tol > 0.0 && std::isfinite(tol), TM_EINVAL, "tol must be positive");
        TM_REQUIRE(m <= 2048, TM_ENOTSUP, "m > 2048 is not supported");
        tm_opts o;
        if (opts) o = *opts; else tm_opts_default(&o);
        TM_REQUIRE(o.max_iter >= 0, TM_EINVAL, "max_iter must be >= 0");
        TM_REQUIRE(o.precision == TM_FULL_DP, TM_ENOTSUP, "the generalized problem runs in TM_FULL_DP");
        TM_REQUIRE(o.precondition == 0 || o.precondition == 1, TM_ENOTSUP,
                   "the generalized problem takes no preconditioner or the diagonal one");
        TM_REQUIRE(history_len >= 0, TM_EINVAL, "history_len must be >= 0");
        TM_REQUIRE(o.graphs == 0 || o.graphs == 1, TM_EINVAL, "tm_opts.graphs must be 0 or 1");
        std::memset(res, 0, sizeof(*res));
        Solver solver(ctx, H, m, tol, o, S);
        return solver.run(C0, C_out, eig_out, res, history, history_len);
    });
}

tm_status tm_set_matrix_batch(tm_ctx *ctx, int64_t n, const int64_t *rowptr, const int32_t *col,
                              const double *val, int32_t k, const double *d, uint32_t flags,
                              tm_mat **out) {
    return guarded([&]() {
        TM_REQUIRE(out && rowptr && col && val && d, TM_EINVAL, "null argument");
        *out = nullptr;
        TM_REQUIRE(k >= 1 && k <= kMaxBatch, TM_EINVAL, "k must be in [1, 256]");
        TM_REQUIRE((flags & TM_DEVICE_PTRS) == 0, TM_ENOTSUP, "a batch matrix takes host arrays");
        tm_mat *base = nullptr;
        const tm_status st = tm_set_matrix_csr(ctx, n, rowptr, col, val, flags, &base);
        if (st != TM_OK) throw Error{st, g_last_error};
        std::unique_ptr<tm_mat, void (*)(tm_mat *)> m(base, tm_free_matrix);
        // A's diagonal and off-diagonal row sums; each H_g's diagonal
        // extremes, |row| maximum and Gershgorin interval as tm_set_matrix_csr
        // forms them for one matrix
        std::vector<double> adiag(n, 0.0), off(n, 0.0);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t q = rowptr[r]; q < rowptr[r + 1]; ++q) {
                if (col[q] == r) adiag[r] += val[q];
                else off[r] += std::fabs(val[q]);
            }
        const size_t total = (size_t)k * n;
        std::vector<float> d32(total);
        m->b_diag_min.assign(k, 1e300);
        m->b_diag_max.assign(k, -1e300);
        m->b_lo.assign(k, 1e300);
        m->b_hi.assign(k, -1e300);
        for (int g = 0; g < k; ++g) {
            double rmax = 0.0;
            for (int64_t r = 0; r < n; ++r) {
                const double dv = d[(size_t)g * n + r];
                TM_REQUIRE(std::isfinite(dv), TM_EINVAL, "non-finite diagonal term");
                d32[(size_t)g * n + r] = (float)dv;
                const double hd = adiag[r] + dv;
                m->b_diag_min[g] = std::min(m->b_diag_min[g], hd);
                m->b_diag_max[g] = std::max(m->b_diag_max[g], hd);
                m->b_lo[g] = std::min(m->b_lo[g], hd - off[r]);
                m->b_hi[g] = std::max(m->b_hi[g], hd + off[r]);
                rmax = std::max(rmax, off[r] + std::fabs(hd));
            }
            m->b_diag_max[g] = std::max(m->b_diag_max[g], 0.5 * rmax);
        }
        m->bd64 = upload(ctx, d, total);
        m->bd32 = upload(ctx, d32.data(), total);
        sync(ctx);
        m->batch_k = k;
        *out = m.release();
        return TM_OK;
    });
}

tm_status tm_batch_layout(int32_t k, int32_t m, int32_t *ldg, int32_t *ld) {
    return guarded([&]() {
        TM_REQUIRE(ldg && ld, TM_EINVAL, "null argument");
        TM_REQUIRE(k >= 1 && k <= kMaxBatch, TM_EINVAL, "k must be in [1, 256]");
        TM_REQUIRE(m >= 1 && m <= 2048, TM_EINVAL, "m must be in [1, 2048]");
        *ldg = batch_group_ld(k, m);
        *ld = leading_dim(k * *ldg);
        return TM_OK;
    });
}

tm_status tm_solve_batch(tm_ctx *ctx, const tm_mat *H, int32_t m, double tol, const tm_opts *opts,
                         const double *C0, double *C_out, double *eig_out, tm_result *res) {
    return guarded([&]() {
        TM_REQUIRE(H && res, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(H->ctx == ctx, TM_EINVAL, "matrix belongs to another context");
        TM_REQUIRE(H->batch_k > 0, TM_EINVAL, "not a batch matrix (tm_set_matrix_batch)");
        TM_REQUIRE(tol > 0.0 && std::isfinite(tol), TM_EINVAL, "tol must be positive");
        const int k = H->batch_k;
        TM_REQUIRE((int64_t)k * batch_group_ld(k, m) <= 2048, TM_ENOTSUP,
                   "a batch of more than 2048 columns is not supported");
        tm_opts o;
        if (opts) o = *opts; else tm_opts_default(&o);
        TM_REQUIRE(o.max_iter >= 0, TM_EINVAL, "max_iter must be >= 0");
        TM_REQUIRE(o.precision >= TM_FULL_DP && o.precision <= TM_MP2_MP1, TM_EINVAL, "unknown precision");
        TM_REQUIRE(o.precision != TM_MIXED_BF16 && o.precision != TM_FULL_BF16, TM_ENOTSUP,
                   "batched solves take no BF16 policy");
        TM_REQUIRE(o.graphs == 0 || o.graphs == 1, TM_EINVAL, "tm_opts.graphs must be 0 or 1");
        TM_REQUIRE(o.precondition == 0 || (o.precondition == 2 && o.cheb_degree == 2 &&
                                           o.cheb_shift > 0.0 && std::isfinite(o.cheb_shift)),
                   TM_ENOTSUP, "batched solves take no preconditioner or the degree-2 polynomial");
        o.history = 0;
        std::memset(res, 0, (size_t)k * sizeof(*res));
        Solver solver(ctx, H, m, tol, o);
        return solver.run(C0, C_out, eig_out, res, nullptr, 0);
    });
}

tm_status tm_random_block(tm_ctx *ctx, int64_t n, int32_t m, uint64_t seed, double *out) {
    return guarded([&]() {
        TM_REQUIRE(out, TM_EINVAL, "null argument");
        check_block_args(ctx, n, m);
        random_block(ctx->stream, n, m, seed, out);
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_spmm(tm_ctx *ctx, const tm_mat *H, int32_t m, int32_t dtype, const void *C, void *X) {
    return guarded([&]() {
        TM_REQUIRE(H && C && X, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(dtype == TM_F64 || dtype == TM_F32, TM_EINVAL, "dtype");
        if (H->batch_k > 0) {
            // the batch layout: problem g's m columns at g * ldg
            const int ldg = batch_group_ld(H->batch_k, m);
            SpmmEpi epi;
            epi.D = dtype == TM_F64 ? (const void *)H->bd64 : (const void *)H->bd32;
            epi.dld = ldg;
            spmm_any(ctx->stream, H, leading_dim(H->batch_k * ldg), C, X, dtype == TM_F64, 0, nullptr, epi);
        } else {
            spmm_any(ctx->stream, H, leading_dim(m), C, X, dtype == TM_F64);
        }
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_gram(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype, const void *A, const void *B,
                  const double *h, double *out) {
    return guarded([&]() {
        TM_REQUIRE(A && B && out, TM_EINVAL, "null argument");
        check_block_args(ctx, n, m);
        TM_REQUIRE(dtype == TM_F64 || dtype == TM_F32 || dtype == TM_BF16X3, TM_EINVAL, "dtype");
        const int ld = leading_dim(m);
        DevMem ws(ctx, gram_workspace(n, m));
        DevMem hp(ctx, ld * sizeof(double));
        const double *hv = nullptr;
        if (h) {
            TM_HIP(hipMemsetAsync(hp.ptr, 0, ld * sizeof(double), ctx->stream));
            TM_HIP(hipMemcpyAsync(hp.ptr, h, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
            hv = (const double *)hp.ptr;
        }
        const bool sym = (A == B) && !h;
        if (dtype == TM_F64)
            gram<double, double>(ctx->stream, n, m, (const double *)A, (const double *)B, hv, false, sym,
                                 (double *)ws.ptr, out);
        else if (dtype == TM_BF16X3)
            gram_bf16x3<float>(ctx->stream, n, m, (const float *)A, (const float *)B, hv, false,
                               (double *)ws.ptr, out);
        else
            gram<float, float>(ctx->stream, n, m, (const float *)A, (const float *)B, hv, false, sym,
                               (double *)ws.ptr, out);
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_gram_noalloc(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype, const void *A,
                          const void *B, const double *h, double *out) {
    return guarded([&]() {
        TM_REQUIRE(A && B && out, TM_EINVAL, "null argument");
        check_block_args(ctx, n, m);
        TM_REQUIRE(dtype == TM_F64 || dtype == TM_F32 || dtype == TM_BF16X3, TM_EINVAL, "dtype");
        char *base = (char *)scratch_of(ctx->device);
        TM_REQUIRE(base != nullptr, TM_EDEVICE, "scratch not bound on this device");
        const int ld = leading_dim(m);
        const size_t hbytes = ((size_t)ld * sizeof(double) + 255) / 256 * 256;
        const size_t avail = kScratchBytes - hbytes;
        const bool sym = (A == B) && !h;
        const size_t need = gram_partials_bytes(n, m, sym && dtype != TM_BF16X3, avail);
        TM_REQUIRE(need <= avail, TM_ENOMEM,
                   "m = " + std::to_string(m) + " needs " + std::to_string(need + hbytes) +
                       " bytes of scratch; the allocation-free Gram holds " +
                       std::to_string(kScratchBytes));
        hipStream_t s = ctx->stream;
        const double *hv = nullptr;
        if (h) {
            pad_vector(s, m, ld, h, (double *)base);
            hv = (const double *)base;
        }
        double *partials = (double *)(base + hbytes);
        if (dtype == TM_F64)
            gram<double, double>(s, n, m, (const double *)A, (const double *)B, hv, false, sym, partials,
                                 out, true, nullptr, nullptr, avail);
        else if (dtype == TM_BF16X3)
            gram_bf16x3<float>(s, n, m, (const float *)A, (const float *)B, hv, false, partials, out,
                               true, nullptr, avail);
        else
            gram<float, float>(s, n, m, (const float *)A, (const float *)B, hv, false, sym, partials,
                               out, true, nullptr, nullptr, avail);
        return TM_OK;
    });
}

tm_status tm_rotate(tm_ctx *ctx, int64_t n, int32_t m, int32_t dtype, const void *A, const double *W,
                    void *out) {
    return guarded([&]() {
        TM_REQUIRE(A && W && out, TM_EINVAL, "null argument");
        check_block_args(ctx, n, m);
        TM_REQUIRE(dtype == TM_F64 || dtype == TM_F32, TM_EINVAL, "dtype");
        TM_REQUIRE(A != out, TM_EINVAL, "out must not alias A");
        const int ld = leading_dim(m);
        DevMem wp(ctx, (size_t)ld * ld * sizeof(double));
        if (dtype == TM_F64) {
            pad_matrix<double>(ctx->stream, m, W, false, (double *)wp.ptr, nullptr);
            rot<double, double, double>(ctx->stream, n, m, (const double *)A, (const double *)wp.ptr,
                                        EPI_NONE, nullptr, nullptr, (double *)out);
        } else {
            pad_matrix<float>(ctx->stream, m, W, false, (float *)wp.ptr, nullptr);
            rot<float, float, float>(ctx->stream, n, m, (const float *)A, (const float *)wp.ptr,
                                     EPI_NONE, nullptr, nullptr, (float *)out);
        }
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_energy_grad(tm_ctx *ctx, const tm_mat *H, int32_t m, int32_t precision, const double *C,
                         double *X, double *G, double *h, double *Hp, double *E) {
    return guarded([&]() {
        TM_REQUIRE(H && C && X && G && h && Hp && E, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(H->batch_k == 0, TM_EINVAL, "not defined for a batch matrix");
        TM_REQUIRE(precision == TM_FULL_DP || precision == TM_MP2 || precision == TM_MP1, TM_EINVAL,
                   "precision must be TM_FULL_DP, TM_MP1 or TM_MP2");
        const int ld = leading_dim(m);
        const int64_t n = H->n;
        hipStream_t s = ctx->stream;
        const bool dp = precision != TM_MP2;
        DevMem hv(ctx, ld * sizeof(double)), dws(ctx, spmm_partials_workspace(n, ld)),
            gws(ctx, gram_workspace(n, m)), wp(ctx, (size_t)ld * ld * sizeof(double)),
            xs(ctx, (size_t)n * ld * (dp ? sizeof(double) : sizeof(float)));
        const int nch = spmm_any(s, H, ld, C, X, true, 1, (double *)dws.ptr);
        reduce_partials(s, 1, nch, ld, (double *)dws.ptr, (double *)hv.ptr);
        // X' = X - C diag(h) is kept by the Gram in the matrix-core precision
        // and read back by the gradient; H' from its upper block tiles,
        // mirrored, also stored padded for the gradient GEMM: as in the solver
        if (precision == TM_MP1) {
            // MP1 (i): FP64 products, G formed in FP64 and stored in FP32 (the
            // epilogue forms X' again from X, C and h); returned widened to FP64
            float *G32 = (float *)xs.ptr;
            gram<double, double>(s, n, m, C, X, (double *)hv.ptr, true, true, (double *)gws.ptr, Hp,
                                 true, nullptr, (double *)wp.ptr);
            rot<double, double, float>(s, n, m, C, (double *)wp.ptr, EPI_GRAD, X, (double *)hv.ptr, G32);
            convert_block<float, double>(s, n * ld, G32, G);
        } else if (dp) {
            double *Xs = (double *)xs.ptr;
            gram<double, double>(s, n, m, C, X, (double *)hv.ptr, true, true, (double *)gws.ptr, Hp,
                                 true, Xs, (double *)wp.ptr);
            rot<double, double, double>(s, n, m, C, (double *)wp.ptr, EPI_GRADX, X, (double *)hv.ptr, G,
                                        nullptr, nullptr, nullptr, nullptr, Xs);
        } else {
            float *Xs = (float *)xs.ptr;
            gram<double, float>(s, n, m, C, X, (double *)hv.ptr, true, true, (double *)gws.ptr, Hp,
                                true, Xs, (float *)wp.ptr);
            rot<double, float, double>(s, n, m, C, (float *)wp.ptr, EPI_GRADX, X, (double *)hv.ptr, G,
                                       nullptr, nullptr, nullptr, nullptr, Xs);
        }
        sum_vector(s, m, (double *)hv.ptr, E);
        TM_HIP(hipMemcpyAsync(h, hv.ptr, m * sizeof(double), hipMemcpyDeviceToDevice, s));
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_orthonormalize(tm_ctx *ctx, int64_t n, int32_t m, int32_t precision, double *C) {
    return guarded([&]() {
        TM_REQUIRE(C, TM_EINVAL, "null argument");
        check_block_args(ctx, n, m);
        TM_REQUIRE(precision == TM_FULL_DP || precision == TM_MP2 || precision == TM_MP1, TM_EINVAL,
                   "precision must be TM_FULL_DP, TM_MP1 or TM_MP2");
        const int ld = leading_dim(m);
        hipStream_t s = ctx->stream;
        const size_t md = (size_t)m * m * sizeof(double);
        DevMem S(ctx, md), R(ctx, md), ws(ctx, gram_workspace(n, m)), cw(ctx, chol_workspace(m)),
            info(ctx, 16), wp(ctx, (size_t)ld * ld * sizeof(double)), dv(ctx, ld * sizeof(double)),
            Cout(ctx, (size_t)n * ld * sizeof(double));
        TM_HIP(hipMemsetAsync(info.ptr, 0, 16, s));
        gram<double, double>(s, n, m, C, C, nullptr, false, true, (double *)ws.ptr, (double *)S.ptr);
        chol_inverse(s, m, (double *)S.ptr, (double *)R.ptr, (double *)cw.ptr, (int32_t *)info.ptr);
        int32_t bad = 0;
        TM_HIP(hipMemcpyAsync(&bad, info.ptr, 4, hipMemcpyDeviceToHost, s));
        sync(ctx);
        TM_REQUIRE(bad == 0, TM_ENOTSPD, "C^T C is not positive definite");
        if (precision == TM_FULL_DP) {
            pad_matrix<double>(s, m, (double *)R.ptr, true, (double *)wp.ptr, (double *)dv.ptr);
            rot<double, double, double>(s, n, m, C, (double *)wp.ptr, EPI_TRMM, nullptr, (double *)dv.ptr,
                                        (double *)Cout.ptr);
        } else {
            pad_matrix<float>(s, m, (double *)R.ptr, true, (float *)wp.ptr, (double *)dv.ptr);
            rot<double, float, double>(s, n, m, C, (float *)wp.ptr, EPI_TRMM, nullptr, (double *)dv.ptr,
                                       (double *)Cout.ptr);
        }
        TM_HIP(hipMemcpyAsync(C, Cout.ptr, (size_t)n * ld * sizeof(double), hipMemcpyDeviceToDevice, s));
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_cholesky_inverse(tm_ctx *ctx, int32_t m, const double *S, double *Rinv) {
    return guarded([&]() {
        TM_REQUIRE(S && Rinv, TM_EINVAL, "null argument");
        use_device(ctx);
        TM_REQUIRE(m >= 1 && m <= 2048, TM_EINVAL, "m must be in [1, 2048]");
        DevMem cw(ctx, chol_workspace(m)), info(ctx, 16);
        TM_HIP(hipMemsetAsync(info.ptr, 0, 16, ctx->stream));
        chol_inverse(ctx->stream, m, S, Rinv, (double *)cw.ptr, (int32_t *)info.ptr);
        int32_t bad = 0;
        TM_HIP(hipMemcpyAsync(&bad, info.ptr, 4, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        TM_REQUIRE(bad == 0, TM_ENOTSPD, "S is not positive definite (pivot " + std::to_string(bad) + ")");
        return TM_OK;
    });
}

tm_status tm_sym_eig(tm_ctx *ctx, int32_t m, const double *A, double *U, double *w) {
    return guarded([&]() {
        TM_REQUIRE(A && U && w, TM_EINVAL, "null argument");
        use_device(ctx);
        TM_REQUIRE(m >= 1 && m <= 2048, TM_EINVAL, "m must be in [1, 2048]");
        DevMem jw(ctx, jacobi_workspace(m)), info(ctx, 16);
        jacobi_eig(ctx->stream, m, A, U, w, (double *)jw.ptr, (int32_t *)info.ptr);
        sync(ctx);
        return TM_OK;
    });
}

tm_status tm_time_kernel(tm_ctx *ctx, const tm_mat *H, int32_t kernel, int32_t m, int32_t dtype,
                         int32_t reps, double *avg_ms) {
    return guarded([&]() {
        TM_REQUIRE(H && avg_ms, TM_EINVAL, "null argument");
        check_block_args(ctx, H->n, m);
        TM_REQUIRE(H->batch_k == 0, TM_EINVAL, "not defined for a batch matrix");
        TM_REQUIRE(reps >= 1 && reps <= 100000, TM_EINVAL, "reps out of range");
        TM_REQUIRE(dtype == TM_F64 || dtype == TM_F32, TM_EINVAL, "dtype");
        TM_REQUIRE(kernel >= TM_K_SPMM && kernel <= TM_K_GRAM_BF16X3, TM_EINVAL, "unknown kernel");
        const int ld = leading_dim(m);
        const int64_t n = H->n;
        const bool mp2 = kernel == TM_K_GRAM_MP2 || kernel == TM_K_ROT_GRAD_MP2 || kernel == TM_K_TRMM_MP2;
        const bool f64 = (dtype == TM_F64 || mp2) && kernel != TM_K_GRAM_BF16X3;
        const size_t blk = (size_t)n * ld * (f64 ? 8 : 4);
        hipStream_t s = ctx->stream;
        DevMem A(ctx, blk), B(ctx, blk), O(ctx, blk), vec(ctx, ld * sizeof(double)),
            ws(ctx, gram_workspace(n, m)), wp(ctx, (size_t)ld * ld * sizeof(double)),
            mm(ctx, (size_t)m * m * sizeof(double)), g32(ctx, mp2 ? blk / 2 : 8),
            ch(ctx, kernel == TM_K_CHOL ? chol_workspace(m) : 8), rinv(ctx, (size_t)m * m * sizeof(double)),
            info(ctx, 64), dp(ctx, rot_partials_workspace(n, m));
        TM_HIP(hipMemsetAsync(A.ptr, 0x3c, blk, s));
        TM_HIP(hipMemsetAsync(O.ptr, 0x3c, blk, s));
        TM_HIP(hipMemsetAsync(B.ptr, 0x3c, blk, s));
        TM_HIP(hipMemsetAsync(vec.ptr, 0, ld * sizeof(double), s));
        TM_HIP(hipMemsetAsync(wp.ptr, 0x3c, (size_t)ld * ld * sizeof(double), s));
        if (kernel == TM_K_CHOL) {
            // a well-conditioned SPD matrix: identity plus a small symmetric perturbation
            std::vector<double> Sh((size_t)m * m);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j)
                    Sh[(size_t)i * m + j] = (i == j ? 1.0 : 0.0) + 1e-3 / (1.0 + i + j);
            TM_HIP(hipMemcpyAsync(mm.ptr, Sh.data(), Sh.size() * sizeof(double), hipMemcpyHostToDevice, s));
            TM_HIP(hipStreamSynchronize(s));
        }
        auto launch = [&]() {
            double *ws_p = (double *)ws.ptr, *mm_p = (double *)mm.ptr, *v = (double *)vec.ptr;
            switch (kernel) {
            case TM_K_SPMM: spmm_any(s, H, ld, A.ptr, O.ptr, f64); break;
            case TM_K_GRAM_SHIFT:
                // as in the solver: X' kept for the gradient
                if (f64) gram<double, double>(s, n, m, (double *)A.ptr, (double *)B.ptr, v, true, true, ws_p, mm_p, false, (double *)O.ptr);
                else gram<float, float>(s, n, m, (float *)A.ptr, (float *)B.ptr, v, true, true, ws_p, mm_p, false, (float *)O.ptr);
                break;
            case TM_K_GRAM_SYM:
                if (f64) gram<double, double>(s, n, m, (double *)A.ptr, (double *)A.ptr, nullptr, false, true, ws_p, mm_p, false);
                else gram<float, float>(s, n, m, (float *)A.ptr, (float *)A.ptr, nullptr, false, true, ws_p, mm_p, false);
                break;
            case TM_K_ROT_GRAD:
                // as in the solver: G from X' (B here) and C H'
                if (f64) rot<double, double, double>(s, n, m, (double *)A.ptr, (double *)wp.ptr, EPI_GRADX, nullptr, v, (double *)O.ptr, nullptr, nullptr, nullptr, nullptr, (double *)B.ptr);
                else rot<float, float, float>(s, n, m, (float *)A.ptr, (float *)wp.ptr, EPI_GRADX, nullptr, v, (float *)O.ptr, nullptr, nullptr, nullptr, nullptr, (float *)B.ptr);
                break;
            case TM_K_TRMM:
                if (f64) rot<double, double, double>(s, n, m, (double *)A.ptr, (double *)wp.ptr, EPI_TRMM, nullptr, v, (double *)O.ptr);
                else rot<float, float, float>(s, n, m, (float *)A.ptr, (float *)wp.ptr, EPI_TRMM, nullptr, v, (float *)O.ptr);
                break;
            case TM_K_GRAM_MP2:
                gram<double, float>(s, n, m, (double *)A.ptr, (double *)B.ptr, v, true, true, ws_p, mm_p, false, (float *)g32.ptr);
                break;
            case TM_K_ROT_GRAD_MP2: {
                // the refinement-phase gradient: FP64 C, FP32 X' (from the Gram), FP32 H'
                // and FP32 G, fused traces
                float *G = (float *)g32.ptr, *Gprev = (float *)O.ptr, *Pprev = Gprev + n * ld;
                rot<double, float, float>(s, n, m, (double *)A.ptr, (float *)wp.ptr, EPI_GRADX, nullptr, v,
                                          G, Gprev, Pprev, nullptr, (double *)dp.ptr, (float *)B.ptr);
                break;
            }
            case TM_K_TRMM_MP2:
                rot<double, float, double>(s, n, m, (double *)A.ptr, (float *)wp.ptr, EPI_TRMM, nullptr, v, (double *)O.ptr);
                break;
            case TM_K_CHOL:
                chol_inverse(s, m, mm_p, (double *)rinv.ptr, (double *)ch.ptr, (int32_t *)info.ptr);
                break;
            case TM_K_GRAM_BF16X3:
                gram_bf16x3<float>(s, n, m, (float *)A.ptr, (float *)B.ptr, v, true, ws_p, mm_p, false);
                break;
            }
        };
        launch();
        launch();
        hipEvent_t e0, e1;
        TM_HIP(hipEventCreate(&e0));
        TM_HIP(hipEventCreate(&e1));
        TM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        TM_HIP(hipEventRecord(e1, s));
        TM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TM_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_ms = (double)ms / reps;
        sync(ctx);
        return TM_OK;
    });
}

}  // extern "C"
