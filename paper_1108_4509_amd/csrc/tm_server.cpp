// Serving: continuous batching of independent trace-minimization solves on
// one GPU.  Requests (host CSR matrix, m, tol, start block) queue in arrival
// order; a request is admitted as soon as a slot is idle and its memory bound
// fits the free part of the server's HBM budget.  Each slot is a host thread
// with its own HIP stream and context, so the kernels of admitted requests
// overlap on the device while later arrivals wait.  Every solve runs the same
// kernels with the same launch shapes and fixed-order reductions as tm_solve
// alone, so a result does not depend on what else is running.
//
// Batching (max_batch > 1): requests on one grid with one kinetic operator
// (same pattern and off-diagonal values; the potential differs) and the same
// m, tol and options are solved together by tm_solve_batch, one batch per
// slot, which turns many launch-bound small solves into one.
//
// Memory: one hipMalloc of the whole budget at creation; admission carves a
// chunk of solve_footprint() bytes from it (first fit), and the request's
// context allocates inside its chunk (first fit again), so an admitted
// request cannot run out of memory and the budget is never exceeded.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tm_solver.h"

using namespace tmin;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
  public:
    static constexpr size_t kAlign = 256;
    void reset(size_t size) {
        free_.clear();
        used_.clear();
        size_ = size;
        if (size) free_[0] = size;
    }
    // returns the offset or SIZE_MAX
    size_t alloc(size_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_[off] = bytes;
                in_use_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t size = u->second;
        used_.erase(u);
        in_use_ -= size;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }
    size_t in_use() const { return in_use_; }

  private:
    std::map<size_t, size_t> free_, used_;
    size_t size_ = 0, in_use_ = 0;
};

struct Request {
    uint64_t id = 0;
    int64_t n = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<double> C0;      // n x ld, zero-padded
    int32_t m = 0;
    double tol = 0;
    tm_opts opts{};
    size_t footprint = 0;
    // batching: hash of (n, pattern, off-diagonal values), row sums of the
    // diagonal entries, and whether the options allow a batched solve
    bool batchable = false;
    uint64_t key = 0;
    std::vector<double> diag;
    // results
    tm_status status = TM_EAGAIN;
    std::string error;
    tm_result res{};
    std::vector<double> eig;
    Clock::time_point t_submit, t_start, t_done;
    bool finished = false;
};

struct Slot {
    tm_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    char *chunk = nullptr;   // device base of the current request's chunk
    Arena arena;             // allocations inside the chunk
    std::thread thread;
};

void *slot_alloc(size_t bytes, void *user) {
    Slot *s = (Slot *)user;
    const size_t off = s->arena.alloc(bytes);
    return off == SIZE_MAX ? nullptr : s->chunk + off;
}

void slot_free(void *p, void *user) {
    Slot *s = (Slot *)user;
    s->arena.release((size_t)((char *)p - s->chunk));
}

}  // namespace

struct tm_server {
    tm_server_opts opts{};
    char *base = nullptr;
    Arena budget;
    size_t peak = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    uint64_t next_id = 1;
    bool stop = false;
    int running = 0;
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, solves = 0;
    std::vector<double> latencies, waits, services;
    Clock::time_point t0 = Clock::now(), t_first, t_last;
    bool any_submit = false;

    void worker(Slot *slot);
    void execute(Slot *slot, Request *r);
    void execute_batch(Slot *slot, const std::vector<Request *> &b);
    // the next admission: the head of the queue and the compatible requests
    // queued behind it, cut to the largest batch whose memory bound fits
    bool admit(std::vector<Request *> &batch, size_t &off, size_t &bytes);
    int max_cols() const { return opts.max_batch_cols > 0 ? opts.max_batch_cols : 512; }
};

namespace {

// Batches stay within n x (k * ldg) <= 2^25 block entries.  Below that a
// lone solve is bound by launch latency (its kernels do not fill the GPU) or
// k problems in one block cost less than k alone; above it the k-fold Gram
// work of the block-diagonal products (all tiles run when problems and Gram
// tiles do not nest) outweighs the saved launches.  Measured on the serving
// classes (MIXED, degree-2 polynomial, 8 problems): 16^3, m = 16: 0.166 s
// alone, 0.046 s in one batch of 8 (5.2e5 entries); 24^3, m = 32: 0.212 s,
// 0.092 s in batches of 4 (1.8e6); 32^3, m = 76: 0.82 s, 0.54 s in pairs
// (6.3e6); 40^3, m = 148: 2.60 s, 2.33 s in pairs (2.0e7) and 3.20 s in
// batches of 4 (4.1e7).  On the 200-request stream (4 slots, batches of up
// to 8): 2^23 entries 5.93-5.98 solves/s, 2^25 5.97-6.12, 2^26 (48^3 pairs,
// 5.7e7) 5.22-5.31.
constexpr int64_t kBatchEntries = (int64_t)1 << 25;

bool same_options(const tm_opts &a, const tm_opts &b) {
    return a.precision == b.precision && a.max_iter == b.max_iter && a.k_rot == b.k_rot &&
           a.k_check == b.k_check && a.precondition == b.precondition && a.transport == b.transport &&
           a.graphs == b.graphs && a.switch_tol == b.switch_tol && a.rise_tol == b.rise_tol &&
           a.stall_tol == b.stall_tol && a.cheb_degree == b.cheb_degree && a.cheb_shift == b.cheb_shift;
}

// b can join a batched solve led by a: same problem class and options, the
// same pattern, and equal off-diagonal values (the diagonals may differ)
bool same_batch(const Request &a, const Request &b) {
    if (!a.batchable || !b.batchable || a.key != b.key || a.n != b.n || a.m != b.m || a.tol != b.tol ||
        !same_options(a.opts, b.opts))
        return false;
    if (a.rowptr != b.rowptr || a.col != b.col) return false;
    for (int64_t r = 0; r < a.n; ++r)
        for (int64_t k = a.rowptr[r]; k < a.rowptr[r + 1]; ++k)
            if (a.col[k] != r && a.val[k] != b.val[k]) return false;
    return true;
}

uint64_t fnv1a(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

bool tm_server::admit(std::vector<Request *> &batch, size_t &off, size_t &bytes) {
    batch.clear();
    if (queue.empty()) return false;
    Request *h = queue.front();
    batch.push_back(h);
    // the largest batch the column and entry caps allow for this class
    // (checked first: requests too large to batch skip the scan)
    auto fits = [&](int k) {
        const int64_t cols = (int64_t)k * batch_group_ld(k, h->m);
        return cols <= max_cols() && h->n * cols <= kBatchEntries;
    };
    int kmax = 1;
    if (opts.max_batch > 1 && h->batchable)
        for (int k = 2; k <= opts.max_batch; ++k)
            if (fits(k)) kmax = k;
    for (size_t i = 1; i < queue.size() && (int)batch.size() < kmax; ++i)
        if (same_batch(*h, *queue[i])) batch.push_back(queue[i]);
    const int64_t nnz = h->rowptr[h->n];
    while (!batch.empty()) {
        const int k = (int)batch.size();
        if (k > 1 && !fits(k)) {
            batch.pop_back();
            continue;
        }
        if (k == 1) {
            bytes = h->footprint;
        } else {
            int32_t ldg = 0, ld = 0;
            (void)tm_batch_layout(k, h->m, &ldg, &ld);
            bytes = batch_footprint(h->n, nnz, k, h->m, h->opts.precision, h->opts.precondition) +
                    (size_t)h->n * ld * 8 + (size_t)k * h->m * 8 + 64 * Arena::kAlign;
        }
        off = budget.alloc(bytes);
        if (off != SIZE_MAX) return true;
        batch.pop_back();
    }
    return false;
}

void tm_server::execute(Slot *slot, Request *r) {
    tm_ctx *ctx = slot->ctx;
    tm_mat *H = nullptr;
    tm_status st = tm_set_matrix_csr(ctx, r->n, r->rowptr.data(), r->col.data(), r->val.data(), 0u, &H);
    if (st != TM_OK) {
        r->status = st;
        r->error = tm_last_error();
        return;
    }
    const int ld = leading_dim(r->m);
    void *C0d = ctx->dalloc((size_t)r->n * ld * sizeof(double));
    void *eigd = ctx->dalloc((size_t)ld * sizeof(double));
    if (!C0d || !eigd) {
        r->status = TM_ENOMEM;
        r->error = "request chunk too small";
    } else if (hipMemcpyAsync(C0d, r->C0.data(), r->C0.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx->stream) != hipSuccess) {
        r->status = TM_EDEVICE;
        r->error = "start block upload failed";
    } else {
        st = tm_solve(ctx, H, r->m, r->tol, &r->opts, (const double *)C0d, nullptr, (double *)eigd,
                      &r->res, nullptr, 0);
        r->status = st;
        if (st != TM_OK) r->error = tm_last_error();
        if (st == TM_OK || st == TM_ENOCONV) {
            r->eig.resize(r->m);
            if (hipMemcpyAsync(r->eig.data(), eigd, r->m * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess) {
                r->status = TM_EDEVICE;
                r->error = "result download failed";
            }
        }
    }
    if (C0d) ctx->dfree(C0d);
    if (eigd) ctx->dfree(eigd);
    tm_free_matrix(H);
    // inputs are no longer needed
    std::vector<int64_t>().swap(r->rowptr);
    std::vector<int32_t>().swap(r->col);
    std::vector<double>().swap(r->val);
    std::vector<double>().swap(r->C0);
}

void tm_server::execute_batch(Slot *slot, const std::vector<Request *> &b) {
    tm_ctx *ctx = slot->ctx;
    const Request *h = b[0];
    const int k = (int)b.size(), m = h->m;
    const int64_t n = h->n;
    auto fail_all = [&](tm_status st, const std::string &msg) {
        for (Request *r : b) {
            r->status = st;
            r->error = msg;
        }
    };
    // A: the shared pattern and off-diagonal values with zero diagonal
    // entries; d_g: request g's diagonal
    std::vector<double> valA = h->val;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t q = h->rowptr[r]; q < h->rowptr[r + 1]; ++q)
            if (h->col[q] == r) valA[q] = 0.0;
    std::vector<double> d((size_t)k * n);
    for (int g = 0; g < k; ++g) std::memcpy(&d[(size_t)g * n], b[g]->diag.data(), n * sizeof(double));
    tm_mat *H = nullptr;
    tm_status st = tm_set_matrix_batch(ctx, n, h->rowptr.data(), h->col.data(), valA.data(), k, d.data(), 0u, &H);
    if (st != TM_OK) {
        fail_all(st, tm_last_error());
        return;
    }
    int32_t ldg = 0, ld = 0;
    (void)tm_batch_layout(k, m, &ldg, &ld);
    // the start blocks side by side (each stored n x leading_dim(m))
    const int lds = leading_dim(m);
    std::vector<double> C0h((size_t)n * ld, 0.0);
    for (int g = 0; g < k; ++g)
        for (int64_t r = 0; r < n; ++r)
            std::memcpy(&C0h[(size_t)r * ld + (size_t)g * ldg], &b[g]->C0[(size_t)r * lds], m * sizeof(double));
    void *C0d = ctx->dalloc(C0h.size() * sizeof(double));
    void *eigd = ctx->dalloc((size_t)k * m * sizeof(double));
    std::vector<tm_result> res(k);
    if (!C0d || !eigd) {
        fail_all(TM_ENOMEM, "request chunk too small");
    } else if (hipMemcpyAsync(C0d, C0h.data(), C0h.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx->stream) != hipSuccess) {
        fail_all(TM_EDEVICE, "start block upload failed");
    } else {
        st = tm_solve_batch(ctx, H, m, h->tol, &h->opts, (const double *)C0d, nullptr, (double *)eigd,
                            res.data());
        if (st != TM_OK && st != TM_ENOCONV) {
            fail_all(st, tm_last_error());
        } else {
            std::vector<double> eig((size_t)k * m);
            if (hipMemcpyAsync(eig.data(), eigd, eig.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess) {
                fail_all(TM_EDEVICE, "result download failed");
            } else {
                for (int g = 0; g < k; ++g) {
                    Request *r = b[g];
                    r->res = res[g];
                    r->status = res[g].converged ? TM_OK : TM_ENOCONV;
                    if (r->status != TM_OK) r->error = "maximum iterations reached";
                    r->eig.assign(eig.begin() + (size_t)g * m, eig.begin() + (size_t)(g + 1) * m);
                }
            }
        }
    }
    if (C0d) ctx->dfree(C0d);
    if (eigd) ctx->dfree(eigd);
    tm_free_matrix(H);
    for (Request *r : b) {
        std::vector<int64_t>().swap(r->rowptr);
        std::vector<int32_t>().swap(r->col);
        std::vector<double>().swap(r->val);
        std::vector<double>().swap(r->C0);
        std::vector<double>().swap(r->diag);
    }
}

void tm_server::worker(Slot *slot) {
    (void)hipSetDevice(opts.device);
    std::unique_lock<std::mutex> lk(mu);
    std::vector<Request *> batch;
    while (true) {
        size_t off = SIZE_MAX, bytes = 0;
        // first in, first out: the head waits until its memory is free
        cv_work.wait(lk, [&] { return stop || admit(batch, off, bytes); });
        if (stop) {
            if (off != SIZE_MAX) budget.release(off);
            break;
        }
        for (Request *r : batch) queue.erase(std::find(queue.begin(), queue.end(), r));
        running += (int)batch.size();
        peak = std::max(peak, budget.in_use());
        lk.unlock();

        slot->chunk = base + off;
        slot->arena.reset(bytes);
        const Clock::time_point t_start = Clock::now();
        for (Request *r : batch) r->t_start = t_start;
        if (batch.size() == 1) execute(slot, batch[0]);
        else execute_batch(slot, batch);
        const Clock::time_point t_done = Clock::now();

        lk.lock();
        budget.release(off);
        for (Request *r : batch) {
            r->t_done = t_done;
            r->finished = true;
            --running;
            if (r->status == TM_OK || r->status == TM_ENOCONV) ++completed;
            else ++failed;
            latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
            waits.push_back(std::chrono::duration<double>(r->t_start - r->t_submit).count());
            services.push_back(std::chrono::duration<double>(r->t_done - r->t_start).count());
        }
        ++solves;
        t_last = t_done;
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" {

tm_status tm_solve_footprint(int64_t n, int64_t nnz, int32_t m, const tm_opts *opts,
                             uint64_t *bytes) {
    if (!bytes || n < 1 || m < 1 || m > n || nnz < 0) return TM_EINVAL;
    tm_opts o;
    if (opts) o = *opts; else tm_opts_default(&o);
    *bytes = solve_footprint(n, nnz, m, o.precision, o.precondition, 0) +
             (uint64_t)n * leading_dim(m) * 8 + (uint64_t)leading_dim(m) * 8 + 64 * Arena::kAlign;
    return TM_OK;
}

tm_status tm_server_create(const tm_server_opts *o, tm_server **out) {
    if (!o || !out) return TM_EINVAL;
    *out = nullptr;
    if (o->max_slots < 1 || o->max_slots > 16 || o->hbm_budget < ((uint64_t)1 << 20)) return TM_EINVAL;
    if (o->max_batch < 0 || o->max_batch > kMaxBatch) return TM_EINVAL;
    if (o->max_batch_cols != 0 && (o->max_batch_cols < 64 || o->max_batch_cols > 2048)) return TM_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || o->device < 0 || o->device >= count) return TM_EINVAL;
    if (hipSetDevice(o->device) != hipSuccess) return TM_EDEVICE;
    auto srv = std::make_unique<tm_server>();
    srv->opts = *o;
    void *base = nullptr;
    if (hipMalloc(&base, o->hbm_budget) != hipSuccess) return TM_ENOMEM;
    srv->base = (char *)base;
    srv->budget.reset(o->hbm_budget);
    for (int i = 0; i < o->max_slots; ++i) {
        auto slot = std::make_unique<Slot>();
        if (hipStreamCreateWithFlags(&slot->stream, hipStreamNonBlocking) != hipSuccess) {
            tm_server_destroy(srv.release());
            return TM_EDEVICE;
        }
        tm_allocator a;
        a.alloc = slot_alloc;
        a.free = slot_free;
        a.user = slot.get();
        if (tm_create(o->device, &a, slot->stream, &slot->ctx) != TM_OK) {
            (void)hipStreamDestroy(slot->stream);
            tm_server_destroy(srv.release());
            return TM_EDEVICE;
        }
        srv->slots.push_back(std::move(slot));
    }
    for (auto &s : srv->slots) {
        tm_server *p = srv.get();
        Slot *sp = s.get();
        s->thread = std::thread([p, sp] { p->worker(sp); });
    }
    *out = srv.release();
    return TM_OK;
}

tm_status tm_server_submit(tm_server *s, const tm_request *q, uint64_t *id) {
    if (!s || !q || !id) return TM_EINVAL;
    if (!q->rowptr || !q->col || !q->val || !q->C0 || q->n < 1 || q->m < 1 || q->m > q->n || q->reserved != 0 ||
        !(q->tol > 0))
        return TM_EINVAL;
    auto r = std::make_unique<Request>();
    r->n = q->n;
    r->m = q->m;
    r->tol = q->tol;
    if (q->opts) r->opts = *q->opts;
    else {
        tm_opts_default(&r->opts);
        r->opts.precision = TM_MIXED;
    }
    r->opts.history = 0;
    const int64_t nnz = q->rowptr[q->n];
    if (nnz < 0) return TM_EINVAL;
    uint64_t fp = 0;
    if (tm_solve_footprint(q->n, nnz, q->m, &r->opts, &fp) != TM_OK) return TM_EINVAL;
    r->footprint = fp;
    if (fp > s->opts.hbm_budget) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->rejected;
        return TM_ENOMEM;
    }
    r->rowptr.assign(q->rowptr, q->rowptr + q->n + 1);
    r->col.assign(q->col, q->col + nnz);
    r->val.assign(q->val, q->val + nnz);
    const tm_opts &o = r->opts;
    r->batchable = s->opts.max_batch > 1 && o.progress == nullptr && o.precision != TM_MIXED_BF16 &&
                   o.precision != TM_FULL_BF16 &&
                   (o.precondition == 0 || (o.precondition == 2 && o.cheb_degree == 2)) && q->rowptr[0] == 0;
    if (r->batchable) {
        for (int64_t i = 0; i < q->n && r->batchable; ++i)
            r->batchable = q->rowptr[i + 1] >= q->rowptr[i];
    }
    if (r->batchable) {
        r->diag.assign(q->n, 0.0);
        uint64_t h = fnv1a(1469598103934665603ull, &q->n, sizeof(q->n));
        h = fnv1a(h, r->rowptr.data(), r->rowptr.size() * sizeof(int64_t));
        h = fnv1a(h, r->col.data(), r->col.size() * sizeof(int32_t));
        for (int64_t i = 0; i < q->n; ++i)
            for (int64_t k = r->rowptr[i]; k < r->rowptr[i + 1]; ++k) {
                if (r->col[k] == i) r->diag[i] += r->val[k];
                else h = fnv1a(h, &r->val[k], sizeof(double));
            }
        r->key = h;
    }
    const int ld = leading_dim(q->m);
    r->C0.assign((size_t)q->n * ld, 0.0);
    for (int64_t i = 0; i < q->n; ++i)
        std::memcpy(&r->C0[(size_t)i * ld], q->C0 + (size_t)i * q->m, q->m * sizeof(double));
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *id = r->id;
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first = r->t_submit;
    }
    ++s->submitted;
    s->queue.push_back(r.get());
    s->requests[r->id] = std::move(r);
    s->cv_work.notify_all();
    return TM_OK;
}

static tm_status take_result(tm_server *s, uint64_t id, tm_result *res, double *eig_out,
                             std::unique_lock<std::mutex> &lk, double timeout_s) {
    auto it = s->requests.find(id);
    if (it == s->requests.end()) return TM_EINVAL;
    Request *r = it->second.get();
    auto ready = [&] { return r->finished; };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (timeout_s > 0) s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    if (!r->finished) return TM_EAGAIN;
    if (res) *res = r->res;
    if (eig_out && !r->eig.empty()) std::memcpy(eig_out, r->eig.data(), r->eig.size() * sizeof(double));
    const tm_status st = r->status;
    set_last_error(r->error);
    s->requests.erase(it);
    return st;
}

tm_status tm_server_poll(tm_server *s, uint64_t id, tm_result *res, double *eig_out) {
    if (!s) return TM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, id, res, eig_out, lk, 0.0);
}

tm_status tm_server_wait(tm_server *s, uint64_t id, double timeout_s, tm_result *res,
                         double *eig_out) {
    if (!s) return TM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, id, res, eig_out, lk, timeout_s < 0 ? -1.0 : std::max(timeout_s, 1e-9));
}

tm_status tm_server_get_stats(tm_server *s, tm_server_stats *out) {
    if (!s || !out) return TM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->rejected = s->rejected;
    out->queued = (int64_t)s->queue.size();
    out->running = s->running;
    out->hbm_budget = s->opts.hbm_budget;
    out->solver_runs = s->solves;
    out->hbm_peak = s->peak;
    std::vector<double> lat = s->latencies;
    // nearest-rank percentile of a sorted sample
    auto pct = [](const std::vector<double> &v, double q) {
        size_t k = (size_t)std::ceil(q * v.size());
        if (k < 1) k = 1;
        return v[std::min(k, v.size()) - 1];
    };
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        std::vector<double> wt = s->waits, sv = s->services;
        std::sort(wt.begin(), wt.end());
        std::sort(sv.begin(), sv.end());
        out->p50_latency_s = pct(lat, 0.50);
        out->p99_latency_s = pct(lat, 0.99);
        out->p50_wait_s = pct(wt, 0.50);
        out->p99_wait_s = pct(wt, 0.99);
        out->p50_service_s = pct(sv, 0.50);
        out->p99_service_s = pct(sv, 0.99);
        out->max_latency_s = lat.back();
        double sum = 0;
        for (double v : lat) sum += v;
        out->mean_latency_s = sum / lat.size();
        const double span = std::chrono::duration<double>(s->t_last - s->t_first).count();
        out->span_s = span;
        out->solves_per_s = span > 0 ? (double)lat.size() / span : 0.0;
    }
    return TM_OK;
}

void tm_server_destroy(tm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;   // queued requests are dropped; running ones finish
        s->queue.clear();
    }
    s->cv_work.notify_all();
    for (auto &slot : s->slots)
        if (slot->thread.joinable()) slot->thread.join();
    for (auto &slot : s->slots) {
        if (slot->ctx) tm_destroy(slot->ctx);
        if (slot->stream) (void)hipStreamDestroy(slot->stream);
    }
    if (s->base) (void)hipFree(s->base);
    delete s;
}

}  // extern "C"
