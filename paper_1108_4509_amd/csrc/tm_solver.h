// Host-side solver object behind tm_solve().
#pragma once

#include <memory>

#include "tm_common.h"

namespace tmin {

// Device allocation through the context's allocator hook (RAII).
struct DevMem {
    tm_ctx *ctx = nullptr;
    void *ptr = nullptr;
    size_t size = 0;
    DevMem(tm_ctx *c, size_t bytes);
    ~DevMem();
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
};

// X = H C for a CSR or stencil H, FP64 (f64) or FP32 blocks, with the fused
// column dots of spmm_csr (ndot, partials); returns the number of chunks.
int spmm_any(hipStream_t s, const tm_mat *H, int ld, const void *C, void *X, bool f64,
             int ndot = 0, double *partials = nullptr, const SpmmEpi &epi = SpmmEpi());

// Upper bound of the device bytes one tm_solve() allocates for an n x m
// problem with nnz stored nonzeros (0 for a stencil), at the given
// precision, history length and preconditioner setting: the blocks that can
// be alive together, the workspaces, the m x m matrices and the matrix itself.
size_t solve_footprint(int64_t n, int64_t nnz, int m, int precision, int precondition,
                       int history_len);

// The same bound for tm_solve_batch of k problems of m columns each on a
// batch matrix with nnz stored nonzeros in its shared A.
size_t batch_footprint(int64_t n, int64_t nnz, int k, int m, int precision, int precondition);

class Solver {
  public:
    // S: the positive definite S of H x = lambda S x (FULL_DP only), or null
    Solver(tm_ctx *ctx, const tm_mat *H, int m, double tol, const tm_opts &o,
           const tm_mat *S = nullptr);
    ~Solver();
    tm_status run(const double *C0, double *C_out, double *eig_out, tm_result *res,
                  double *hist, int hist_len);

  private:
    struct Impl;
    std::unique_ptr<Impl> impl_;
};

}  // namespace tmin
