// Internal declarations shared by the host driver and the HIP kernels of the
// trace-minimization library.  Not part of the public ABI (include/tracemin.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tracemin.h"

namespace tmin {

// Sets the calling thread's tm_last_error() text.
void set_last_error(const std::string &msg);


// Internal error, converted to a tm_status at the C boundary.
struct Error {
    tm_status status;
    std::string msg;
};

#define TM_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            throw ::tmin::Error{TM_EDEVICE, std::string(#call) + ": " +         \
                                              hipGetErrorString(e_)};         \
    } while (0)

#define TM_REQUIRE(cond, st, text)                                            \
    do {                                                                      \
        if (!(cond)) throw ::tmin::Error{(st), (text)};                         \
    } while (0)

inline int leading_dim(int m) { return (m + 31) / 32 * 32; }

// Batched solves: at most kMaxBatch problems; problem g of k with m columns
// owns ldg = batch_group_ld(k, m) columns (m rounded up to 16, then up to a
// k * ldg that is a multiple of 64: the column-chunked SpMM's FP32 width).
constexpr int kMaxBatch = 256;
inline int batch_group_ld(int k, int m) {
    int ldg = (m + 15) / 16 * 16;
    while ((int64_t)k * ldg % 64) ldg += 16;
    return ldg;
}

// Device-resident scalars of the CG controller (one per solve).
struct CgState {
    // inputs set by the host
    double tol;          // stop when rho <= tol
    double rise_tol;     // restart when E > E_prev + rise_tol |E_prev|
    double switch_tol;   // phase switch when rho <= switch_tol
    double stall_tol;    // phase switch when E decreased by < stall_tol |E| over stall_window
    int32_t stall_window;
    int32_t history_len;
    int32_t force_restart;   // host sets to 1 before an iteration that must restart
    int32_t phase_gate;      // 1: this phase ends at switch_tol/stall (sets phase_end)
    // evolving state
    double E, E_prev, rho, gz_prev, gamma, pg, alpha;
    double E_window;         // E at the start of the stall window
    int32_t it;              // iterations recorded (stops advancing once done)
    int32_t done;            // rho <= tol reached
    int32_t phase_end;       // switch requested (FP32 phase)
    int32_t restarts;
    int32_t nan_seen;
    int32_t window_it;
    int32_t have_prev;       // E_prev, G_prev valid
    int32_t pad_;
};

// ---------------------------------------------------------------- kernels
// All launchers enqueue on `s` and return immediately.  Blocks are n x ld
// row-major.  "partials" arguments are device workspaces sized by the
// matching *_workspace() helper.

// SpMM X = H C ---------------------------------------------------------------
struct CsrDev {
    int64_t n = 0, nnz = 0;
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const double *val64 = nullptr;
    const float *val32 = nullptr;
};
struct StencilDev {
    int32_t ndim = 3, nx = 1, ny = 1, nz = 1, order = 2, periodic = 1;
    double c0 = 0;          // kinetic diagonal
    double c1 = 0, c2 = 0;  // per-axis coefficients of offsets +-1, +-2
    const double *V64 = nullptr;
    const float *V32 = nullptr;
};
// Optional epilogue of the SpMM: affine: X = a C + b (H C) (a polynomial of
// degree one in H, e.g. the degree-2 Chebyshev preconditioner); E: the extra
// block of the third dot mode.  Only the column-chunked CSR kernel and the
// 3-D 7-point stencil kernel take it (spmm_fast_path tells).
// Batched operators H_g = A + diag(d_g) (one shared A, a diagonal per
// problem; problem g owns columns g * dld .. (g + 1) * dld - 1): D holds the
// d_g in the block's precision, problem-major (d_g at D + g * n), and is
// added to A C in the epilogue; gab (2 per problem, FP64) replaces a, b of
// the affine form per problem.
struct SpmmEpi {
    double a = 0.0, b = 1.0;
    int affine = 0;
    const void *E = nullptr;
    const void *D = nullptr;
    int dld = 0;
    const double *gab = nullptr;
};
// ndot = 0: X = H C only.  ndot = 1: also per-workgroup partial sums of
// c_j . x_j; ndot = 2: of c_j . x_j and c_j . c_j; ndot = 3 (fast path
// only): of c_j . x_j and e_j . x_j (E from the epilogue), written to
// partials[(p * nchunk + chunk) * ld + j].  Returns nchunk (for
// reduce_partials).  partials needs spmm_partials_workspace(n, ld) bytes.
size_t spmm_partials_workspace(int64_t n, int ld);
template <typename T>
int spmm_csr(hipStream_t s, const CsrDev &H, int ld, const T *C, T *X, int ndot,
             double *partials, const SpmmEpi &epi = SpmmEpi());
template <typename T>
int spmm_stencil(hipStream_t s, const StencilDev &H, int64_t n, int ld,
                 const T *C, T *X, int ndot, double *partials, const SpmmEpi &epi = SpmmEpi());
// True when the kernel chosen for this operator and width takes SpmmEpi and
// ndot = 3.
bool spmm_fast_path(bool stencil, const StencilDev &st, int ld, bool f64);
// out[p * ld + j] = sum over chunks of partials[(p * nchunk + c) * ld + j],
// in a fixed order.
void reduce_partials(hipStream_t s, int nprod, int nchunk, int ld,
                     const double *partials, double *out);

// Column dot products ----------------------------------------------------
// out[p * ld + j] = sum_r w_p(r) * f_p(a_p[r, j], b_p[r, j]) for p < nprod,
// with f = a*b (kind 0) or (a - sc[j] * b)^2 (kind 1, sc device m-vector).
// Accumulated in FP64, reduced in a fixed order (deterministic).
template <typename T>
struct DotArgs {
    int nprod = 0;
    const T *a[4] = {nullptr, nullptr, nullptr, nullptr};
    const T *b[4] = {nullptr, nullptr, nullptr, nullptr};
    int weighted[4] = {0, 0, 0, 0};
    int kind = 0;
    const double *w = nullptr;   // per-row weights (n)
    const double *sc = nullptr;  // per-column scale (kind 1)
};
size_t coldots_workspace(int64_t n, int ld);
template <typename T>
void coldots(hipStream_t s, int64_t n, int ld, const DotArgs<T> &args,
             double *partials, double *out);

// Block-diagonal results of batched solves: with ldg > 0, entries (i, j) of
// different problems (i / ldg != j / ldg) and of the zero columns that pad
// each problem to ldg (i % ldg >= mg or j % ldg >= mg) are stored as 0, the
// padding's diagonal as pad (1 keeps a Gram matrix positive definite).
struct BatchCols {
    int ldg = 0, mg = 0;
    double pad = 0.0;
};

// Gram products out = A^T B' (m x m, FP64), B' = B - A diag(h) if h --------
// Partials workspace of the Gram products; ldg > 0: also of the batched
// launches over the diagonal blocks of a block-diagonal result (BatchCols).
size_t gram_workspace(int64_t n, int m, int ldg = 0);
// Bytes of FP64 partials gram() (symmetric or not) uses when its workspace
// holds ws_bytes (0: the default workspace, gram_workspace): fewer row
// splits when the workspace is smaller.
size_t gram_partials_bytes(int64_t n, int m, bool symmetric, size_t ws_bytes);
// reduce = false launches only the split-K product (used to time it alone).
// xshift (with h): B' itself, n x ld in the matrix-core precision TM, is also
// stored there (the EPI_GRADX input of rot()).  wpad: the result is also
// stored as the zero-padded ld x ld matrix in TM (the W of rot(), as
// pad_matrix would write it).  symmetric: only the upper block tiles are
// computed and mirrored (exact for A = B; with h, the symmetric H' of an
// orthonormal A).  ws_bytes > 0: partials holds only that many bytes (the
// split count is lowered to fit, see gram_partials_bytes).
template <typename TA, typename TM>
void gram(hipStream_t s, int64_t n, int m, const TA *A, const TA *B,
          const double *h, bool zero_diag, bool symmetric, double *partials,
          double *out, bool reduce = true, TM *xshift = nullptr, TM *wpad = nullptr,
          size_t ws_bytes = 0, BatchCols bc = BatchCols());

// S = Cn^T Cn with Cn = C + alpha P formed while staged (alpha from st) and
// written to Cn: the update of Fig. 1 fused into Fig. 4 step (1).  Batched
// solves (bc.ldg > 0): column j takes the alpha of st[j / bc.ldg].
template <typename TA, typename TM, typename TP>
void gram_update(hipStream_t s, int64_t n, int m, const TA *C, const TP *P, const CgState *st,
                 TA *Cn, double *partials, double *out, BatchCols bc = BatchCols());

// The Gram product with h (H' = A^T (B - A diag(h)), or A^T B without h) on
// BF16 matrix cores with two-term BF16 operands (about 2^-16 relative to
// sum |a||b|); full m x m, same partials layout and workspace as gram().
template <typename TA>
void gram_bf16x3(hipStream_t s, int64_t n, int m, const TA *A, const TA *B, const double *h,
                 bool zero_diag, double *partials, double *out, bool reduce = true,
                 float *wpad = nullptr, size_t ws_bytes = 0);

// Tall-skinny products out = A W (+ epilogue) ------------------------------
enum RotEpi { EPI_NONE = 0, EPI_GRAD = 1, EPI_TRMM = 2, EPI_GRADX = 3 };
// EPI_NONE:  out = A W
// EPI_GRAD:  out = -2 ((X - A diag(h)) - A W)          (Fig. 2, step (7))
// EPI_GRADX: out = -2 (X' - A W), X' = X - A diag(h) given in the matrix-core
//            precision (stored by the Gram that formed it, see gram())
// EPI_TRMM:  out = A diag(d) + A W, W strictly upper   (Eq. 13)
// With EPI_GRAD and partials != nullptr the epilogue also accumulates, per
// output column j, the traces of the Polak-Ribiere step (Eq. 8) and the descent
// test: p = 0: g.g, 1: g.(M g), 2: g_prev.(M g), 3: p_prev.g, written to
// partials[(p * nchunk + chunk) * ld + j]; returns nchunk (row blocks).
// Gp = nullptr skips trace 2 (it reads 0) and the pass over G_prev.
// partials needs rot_partials_workspace(n, m) bytes.  wg > 0: W is block
// diagonal with wg x wg diagonal blocks (wg a multiple of 16), and each
// column tile loops only over the rows of its blocks.
size_t rot_partials_workspace(int64_t n, int m);
template <typename TA, typename TM, typename TO>
int rot(hipStream_t s, int64_t n, int m, const TA *A, const TM *Wpad,
        int epi, const TA *X, const double *vec, TO *out, const TO *Gp = nullptr,
        const TO *Pp = nullptr, const double *M = nullptr, double *partials = nullptr,
        const TM *Xs = nullptr, int wg = 0);
// Copy an m x m FP64 matrix into an ld x ld zero-padded matrix of type TM,
// keeping the strict upper triangle only (strict_upper) and returning the
// diagonal in diag (when not null).
template <typename TM>
void pad_matrix(hipStream_t s, int m, const double *W, bool strict_upper,
                TM *Wpad, double *diag);

// Dense m x m FP64 kernels -------------------------------------------------
size_t chol_workspace(int m);
// Rinv = R^{-1}, S = R^T R.  info[0] = 0 or the 1-based failing pivot.
// sb > 0 and < m: S is block diagonal in sb x sb blocks (sb a multiple of
// 64 dividing m), factored side by side; Rinv's entries outside those blocks
// are not written (the caller keeps them zero).
void chol_inverse(hipStream_t s, int m, const double *S, double *Rinv,
                  double *work, int32_t *info, int sb = 0);
size_t jacobi_workspace(int m);
// Eigenpairs of symmetric A: w ascending, U columns.  info[0] = sweeps.
// Batched (block-diagonal) A: ascending within each group of ldg indices,
// of which the first mg are real (ldg = 0: one group).
void jacobi_eig(hipStream_t s, int m, const double *A, double *U, double *w,
                double *work, int32_t *info, int ldg = 0, int mg = 0);
// A = 0.5 (H' + H'^T) + diag(h): the m x m H of Eq. 9 from Algorithm-2 pieces.
void assemble_subspace_matrix(hipStream_t s, int m, const double *Hp,
                              const double *h, double *A);

// Elementwise block kernels -------------------------------------------------
// P = M G + gamma P   (gamma read from st->gamma; M = per-row weights or null).
// Batched solves: column j takes the gamma of st[j / ldg] (ldg = 0: one group).
template <typename TG, typename TP>
void p_update(hipStream_t s, int64_t n, int ld, const TG *G, const double *M,
              const CgState *st, TP *P, int ldg = 0);
template <typename TI, typename TO>
void convert_block(hipStream_t s, int64_t count, const TI *in, TO *out);
// The seeded standard normal start block of tm_random_block (n x ld FP64).
// With width > 0 only columns col0 .. col0 + width - 1 of an n x ld_out block
// are written (entries of columns >= m of that range are 0): one problem of a
// batched start block.
void random_block(hipStream_t s, int64_t n, int m, uint64_t seed, double *out, int width = 0,
                  int ld_out = 0, int col0 = 0);
// Chebyshev iteration steps (polynomial preconditioner): d = z = g * inv_theta;
// r_out = r_in - (t - sigma d), d = c_dd d + c_r r_out, z += d (t = H d).
// r_out may alias r_in.
template <typename T>
void cheb_init(hipStream_t s, int64_t count, const T *g, double inv_theta, T *d, T *z);
template <typename T>
void cheb_step(hipStream_t s, int64_t count, const T *t, const T *r_in, T *r_out, T *d, T *z,
               double sigma, double c_dd, double c_r);
// Cn = C + alpha P (alpha = st->alpha), count elements.
template <typename TP>
void update_block(hipStream_t s, int64_t count, const double *C, const TP *P, const CgState *st,
                  double *Cn);
// Xs = X - Z diag(h) for n x ld blocks (h: ld entries).
void shift_block(hipStream_t s, int64_t n, int ld, const double *X, const double *Z,
                 const double *h, double *Xs);
// out[0..ld) = v[0..m) followed by zeros (a kernel, no memset node).
void pad_vector(hipStream_t s, int m, int ld, const double *v, double *out);
// M_ii = 1 / (diag_i - sigma) (Eq. 18's diagonal M), n entries.
void jacobi_preconditioner(hipStream_t s, int64_t n, const double *diag, double sigma,
                           double *M);

// CG controller (one workgroup per problem) --------------------------------
// After the gradient: dots = [gg | gz | gprev_z | pprev_g] (4 x ld), h (ld).
// Batched solves: ngroups problems of m columns each, problem g in columns
// g * ldg .. g * ldg + m - 1 with its state st[g].
void cg_control_gamma(hipStream_t s, int m, int ld, const double *h,
                      const double *dots, CgState *st, double *history, int ngroups = 1,
                      int ldg = 0);
// After Y = HP: dots2 = [py | pp] (2 x ld).
void cg_control_alpha(hipStream_t s, int m, int ld, const double *h,
                      const double *dots2, CgState *st, int ngroups = 1, int ldg = 0);
// Sum of the m entries of v into *out (single workgroup, fixed order).
void sum_vector(hipStream_t s, int m, const double *v, double *out);

}  // namespace tmin

// Objects behind the opaque handles of the C ABI ----------------------------
struct tm_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    tm_allocator alloc{};
    bool custom_alloc = false;
    // pinned host memory for polling, made on first use: the controller
    // states of up to kMaxBatch problems, then 64 bytes of status words
    static constexpr size_t kPinnedStates = 48 << 10;
    static constexpr size_t kPinnedBytes = kPinnedStates + 64;
    void *pinned = nullptr;
    void *dalloc(size_t bytes);
    void dfree(void *p);
    void *pinned_buffer();
    ~tm_ctx();
};

struct tm_mat {
    tm_ctx *ctx = nullptr;
    int64_t n = 0;
    bool is_stencil = false;
    tmin::CsrDev csr;
    tmin::StencilDev st;
    // owned device arrays
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val64 = nullptr;
    float *val32 = nullptr;
    double *V64 = nullptr;
    float *V32 = nullptr;
    double *diag = nullptr;      // H_ii (n), FP64
    double diag_min = 0, diag_max = 0;
    // Gershgorin bounds of the spectrum: min / max over rows of
    // H_ii -+ sum_{j != i} |H_ij|
    double gersh_lo = 0, gersh_hi = 0;
    // a batch of batch_k operators H_g = A + diag(d_g) (CSR A above): d_g in
    // FP64 and FP32 (problem-major), each H_g's diagonal extremes and
    // Gershgorin bounds
    int32_t batch_k = 0;
    double *bd64 = nullptr;
    float *bd32 = nullptr;
    std::vector<double> b_diag_min, b_diag_max, b_lo, b_hi;
};
