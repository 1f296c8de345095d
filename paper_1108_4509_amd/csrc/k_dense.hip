// Dense m x m FP64 kernels of the iteration: the Cholesky factorization and
// triangular inverse of Fig. 4 (steps (2) and (3)), and the assembly of the
// m x m H of Eq. 9 from the pieces of Algorithm-2.
//
// The factorization is O(m^3) with m <= 2048, so it is latency-bound: the
// serial part (the 64-wide diagonal blocks) runs in LDS inside one workgroup,
// the panel and trailing products of each block column spread over many
// workgroups, with the matrices in a device workspace resident in L2.
#include "tm_common.h"

#include <algorithm>
#include <cmath>

namespace tmin {
namespace {


typedef double d4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i % 4), register i / 4.
__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline int mfma64_row(int lane, int r) { return 4 * r + (lane >> 4); }

// A pivot below kPivotTol times the original diagonal entry counts as a
// breakdown: C^T C is then numerically singular (dependent columns of C).
constexpr double kPivotTol = 1e-14;

__device__ inline void lower_pair(int p, int &bi, int &bj) {
    int i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > p) --i;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    bi = i;
    bj = p - i * (i + 1) / 2;
}

__device__ inline double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Invert the Cholesky factor of an NB x NB diagonal block D = L L^T by one
// wave, on the augmented NB x 2NB matrix [D | I] held in registers: lane c
// keeps column c (rows a[0..NB)); for NB = 16 the upper 32 lanes repeat the
// last column.  Gaussian elimination without pivoting: at step k every lane
// takes the column of multipliers from lane k by readlane and updates its
// own column, so no barrier and no memory round trip is needed.  Afterwards
// the I half holds L1^{-1}, where D = L1 diag(d) L1^T with L1 unit lower, so
// L^{-1} = diag(d)^{-1/2} L1^{-1}; it goes to Dinv (zero above the
// diagonal).  Returns the pivot d_l in lane l < NB (1 in the other lanes).
template <int NB>
__device__ __attribute__((always_inline)) double diag_inv_wave(int lane, double (&a)[NB],
                                                               double (*Dinv)[NB + 1]) {
    constexpr int NC = 2 * NB;
    double dl = 1.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const double dk = readlane_f64(a[k], k);
        dl = (lane == k) ? dk : dl;
        // 1 / d_k: the hardware reciprocal refined by two Newton steps
        double r = __builtin_amdgcn_rcp(dk);
        r = fma(r, fma(-dk, r, 1.0), r);
        r = fma(r, fma(-dk, r, 1.0), r);
        // a_ic -= a_ik (a_kc / d_k): one scaling per lane, one FMA per row
        const double rk = a[k] * r;
#pragma unroll
        for (int i = k + 1; i < NB; ++i) a[i] = fma(-readlane_f64(a[i], k), rk, a[i]);
    }
    const double sl = 1.0 / sqrt(dl);   // lane l < NB: d_l^{-1/2}
    double sc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) sc[i] = readlane_f64(sl, i);
    if (lane >= NB && lane < NC) {
        const int col = lane - NB;
#pragma unroll
        for (int i = 0; i < NB; ++i) Dinv[i][col] = (i >= col) ? a[i] * sc[i] : 0.0;
    }
    return dl;
}

// S = L L^T (L lower; S = R^T R with R = L^T) and Rinv = R^{-1} = L^{-T},
// right-looking over kBlk-wide block columns, each in three steps (K3 of a
// block column shares its launch with K1 of the next one):
//   K1 (one workgroup): the diagonal block S_kk = L_kk L_kk^T is factored and
//      inverted in LDS (X_kk = L_kk^{-1}), over 16-wide sub-panels, carrying
//      the same block forward substitution L X = I inside the block;
//   K2 (many workgroups): the panel below, L_ik = S_ik X_kk^T, and the block
//      row of the inverse left of the diagonal, X_kj = X_kk W_kj, where W
//      holds the off-diagonal part of I minus the updates of the earlier
//      block columns (W_kj = -sum_{l<k} L_kl X_lj);
//   K3 (many workgroups): the trailing matrix S_ij -= L_ik L_jk^T (lower
//      tiles) and the rows of W below, W_ij -= L_ik X_kj.
// All products are FP64 matrix-core tiles of 16 x 16.  Only the lower
// triangles of S and of the updated trailing matrix are read.  work: L
// (m*m; the trailing matrix, then the panels), X (m*m; W, then X = L^{-1})
// doubles.  Rinv is written whole (zeros below the diagonal).
constexpr int kBlk = 64;           // block column of the launches
constexpr int kSub = 16;           // sub-panel inside K1
constexpr int kBlkThreads = 256;   // 4 waves per workgroup
constexpr int kAS = kBlk + 1;      // LDS row stride of the K1 block

// The kernels below factor an m x m matrix stored with row stride lda.  A
// block-diagonal matrix of m x m diagonal blocks (lda = their number times m)
// is factored one block per blockIdx.y: the Cholesky factor and the inverse
// of a block-diagonal matrix are block diagonal, so the blocks are
// independent and nothing outside them is read or written.
__device__ inline size_t diag_offset(int m, int lda) {
    return (size_t)blockIdx.y * (size_t)m * (size_t)(lda + 1);
}

// K1 body.  upd: the trailing update of the previous block column is still
// to be applied to this diagonal block (it runs beside that update's launch,
// which skips these tiles): the block is read from where that update would
// read it and the update is formed here, in the same order and precision.
__device__ __attribute__((always_inline)) void chol_block_body(
    int m, int lda, int kb, const double *__restrict__ S, const double *__restrict__ L,
    double *__restrict__ X, double *__restrict__ Rinv, int32_t *__restrict__ info, bool upd) {
    constexpr int NB = kSub, nwaves = kBlkThreads / 64;
    __shared__ double A[kBlk * kAS];   // the block; the sub-panel columns become L
    __shared__ double W[kBlk * kAS];   // W, then X_kk (lower, zero above)
    __shared__ double Dinv[NB][NB + 1];
    __shared__ double Sd[kBlk];
    __shared__ int ok_flag;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (m - kb < kBlk) ? (m - kb) : kBlk;
    const int kp = upd ? kb - kBlk : kb;   // the block column last applied to the source
    const double *src = (kp == 0) ? S : L;
    {
        // lower triangle of the block; identity beyond nb (pivots 1)
        // (with upd, the previous block column's panel rows of this block,
        // L_kp, are loaded into W in the same round trip)
        constexpr int U = kBlk * kBlk / kBlkThreads;
        double v[U], lp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + u * kBlkThreads, i = e / kBlk, c = e % kBlk;
            v[u] = (i == c) ? 1.0 : 0.0;
            if (i < nb && c <= i) v[u] = src[(size_t)(kb + i) * lda + kb + c];
            lp[u] = (upd && i < nb) ? L[(size_t)(kb + i) * lda + kp + c] : 0.0;
        }
        const double sd = (tid < nb) ? S[(size_t)(kb + tid) * lda + kb + tid] : 1.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + u * kBlkThreads, i = e / kBlk, c = e % kBlk;
            A[i * kAS + c] = v[u];
            W[i * kAS + c] = lp[u];
        }
        if (tid < kBlk) Sd[tid] = sd;
    }
    __syncthreads();
    if (upd) {
        // A_ij -= L_ip L_jp^T over the previous block column p = kb - kBlk,
        // one wave per lower 16 x 16 tile (the products and their order are
        // those of the trailing kernel)
        constexpr int KS = kBlk / 4;
        const int nt = (nb + 15) / 16;
        for (int t = wave; t < nt * (nt + 1) / 2; t += nwaves) {
            int bi, bj;
            lower_pair(t, bi, bj);
            const int ia = bi * 16 + (lane & 15), ja = bj * 16 + (lane & 15);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < KS; ++u) {
                const int tk = 4 * u + (lane >> 4);
                acc = mfma64(W[ia * kAS + tk], W[ja * kAS + tk], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < nb && j <= i) A[i * kAS + j] -= acc[r];
            }
        }
        __syncthreads();
        for (int e = tid; e < kBlk * kAS; e += kBlkThreads) W[e] = 0.0;
        __syncthreads();
    }
    const int np = (nb + NB - 1) / NB;
    for (int p = 0; p < np; ++p) {
        const int q = p * NB;
        // (1) the 16 x 16 diagonal sub-block, factored and inverted by wave 0
        if (wave == 0) {
            const int c = lane < 2 * NB ? lane : 2 * NB - 1;
            double a[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i)
                a[i] = c < NB ? A[(q + (i > c ? i : c)) * kAS + q + (i > c ? c : i)]
                              : (i == c - NB ? 1.0 : 0.0);
            const double dl = diag_inv_wave<NB>(lane, a, Dinv);
            // breakdown: the first pivot below kPivotTol times its S diagonal
            const double sd = lane < NB ? Sd[q + lane] : 1.0;
            const unsigned long long bad = __ballot(lane < NB && !(dl > kPivotTol * fabs(sd)));
            if (lane == 0) ok_flag = bad ? __ffsll(bad) - 1 : -1;
        }
        __syncthreads();
        if (ok_flag >= 0) {   // uniform
            if (tid == 0 && info[0] == 0) info[0] = (int)blockIdx.y * m + kb + q + ok_flag + 1;
            return;
        }
        // (2) X of the sub-panel's rows: Dinv on the diagonal, X_pj = Dinv W_pj
        //     left of it (one wave per 16-column strip, read before written);
        // (3) the sub-panel below: L_ip = A_ip Dinv^T (one wave per tile)
        for (int e = tid; e < NB * NB; e += kBlkThreads)
            W[(q + e / NB) * kAS + q + e % NB] = Dinv[e / NB][e % NB];
        const int nbelow = np - 1 - p;
        for (int t = wave; t < p + nbelow; t += nwaves) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            if (t < p) {
                const int jc = t * NB + (lane & 15);
                double bv[NB / 4];
#pragma unroll
                for (int u = 0; u < NB / 4; ++u) bv[u] = W[(q + 4 * u + (lane >> 4)) * kAS + jc];
#pragma unroll
                for (int u = 0; u < NB / 4; ++u)
                    acc = mfma64(Dinv[lane & 15][4 * u + (lane >> 4)], bv[u], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) W[(q + mfma64_row(lane, r)) * kAS + jc] = acc[r];
            } else {
                const int r0 = (t + 1) * NB;   // sub-panel row tile t + 1
                double av[NB / 4];
#pragma unroll
                for (int u = 0; u < NB / 4; ++u) av[u] = A[(r0 + (lane & 15)) * kAS + q + 4 * u + (lane >> 4)];
#pragma unroll
                for (int u = 0; u < NB / 4; ++u)
                    acc = mfma64(av[u], Dinv[lane & 15][4 * u + (lane >> 4)], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) A[(r0 + mfma64_row(lane, r)) * kAS + q + (lane & 15)] = acc[r];
            }
        }
        __syncthreads();
        // (4) trailing: A_ij -= L_ip L_jp^T (tiles below the sub-panel, lower)
        //     and W_ij -= L_ip X_pj (rows below, columns up to the sub-panel)
        const int nr = nbelow, npairs = nr * (nr + 1) / 2, nwork = npairs + nr * (p + 1);
        for (int t = wave; t < nwork; t += nwaves) {
            const bool sym = t < npairs;
            int bi, bj;
            if (sym) {
                lower_pair(t, bi, bj);
                bi += p + 1;
                bj += p + 1;
            } else {
                const int u = t - npairs;
                bi = p + 1 + u / (p + 1);
                bj = u % (p + 1);
            }
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < NB / 4; ++u) {
                const int k = q + 4 * u + (lane >> 4);
                const double a = A[(bi * NB + (lane & 15)) * kAS + k];
                const double b = sym ? A[(bj * NB + (lane & 15)) * kAS + k]
                                     : W[k * kAS + bj * NB + (lane & 15)];
                acc = mfma64(a, b, acc);
            }
            double *T = sym ? A : W;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int idx = (bi * NB + mfma64_row(lane, r)) * kAS + bj * NB + (lane & 15);
                T[idx] -= acc[r];
            }
        }
        __syncthreads();
    }
    // X_kk out, and the whole diagonal block of Rinv = X^T (zero below the
    // diagonal); each written along its rows
    constexpr int U = kBlk * kBlk / kBlkThreads;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * kBlkThreads, i = e / kBlk, c = e % kBlk;
        if (i < nb && c <= i) X[(size_t)(kb + i) * lda + kb + c] = W[i * kAS + c];
        // Rinv row i, column c: X_kk[c][i]
        if (i < nb && c < nb) Rinv[(size_t)(kb + i) * lda + kb + c] = (i <= c) ? W[c * kAS + i] : 0.0;
    }
}

__global__ __launch_bounds__(kBlkThreads) void chol_block_kernel(
    int m, int lda, int kb, const double *__restrict__ S, const double *__restrict__ L,
    double *__restrict__ X, double *__restrict__ Rinv, int32_t *__restrict__ info) {
    const size_t off = diag_offset(m, lda);
    chol_block_body(m, lda, kb, S + off, L + off, X + off, Rinv + off, info, false);
}

// K2: workgroups [0, nA) form the panel L_ik = S_ik X_kk^T, 16 rows each (one
// 16-column tile per wave); workgroups [nA, nA + kb/16) finish a 16-column
// strip of the block row of X, X_kj = X_kk W_kj (the strip is staged in LDS
// before it is overwritten), with Rinv's mirror entries and the zeros below
// its diagonal.
__global__ __launch_bounds__(kBlkThreads) void chol_panel_kernel(
    int m, int lda, int kb, const double *__restrict__ S, double *__restrict__ L,
    double *__restrict__ X, double *__restrict__ Rinv) {
    {
        const size_t off = diag_offset(m, lda);
        S += off;
        L += off;
        X += off;
        Rinv += off;
    }
    constexpr int KS = kBlk / 4;   // MFMA k-steps over the block width
    __shared__ double Ws[kBlk][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (m - kb < kBlk) ? (m - kb) : kBlk, R = m - kb - nb;
    const int nA = (R + 15) / 16;
    const double *src = (kb == 0) ? S : L;
    const int g = blockIdx.x;
    if (g < nA) {
        // R > 0 here, so the block is full (nb == kBlk)
        const int i0 = kb + nb + 16 * g, c0 = 16 * wave;
        const int ia = i0 + (lane & 15), cb = c0 + (lane & 15);
        double av[KS], bv[KS];
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int t = 4 * u + (lane >> 4);
            av[u] = (ia < m) ? src[(size_t)ia * lda + kb + t] : 0.0;
            bv[u] = (t <= cb) ? X[(size_t)(kb + cb) * lda + kb + t] : 0.0;   // X_kk[c][t]
        }
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < KS; ++u) acc = mfma64(av[u], bv[u], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + mfma64_row(lane, r);
            if (i < m) L[(size_t)i * lda + kb + cb] = acc[r];
        }
        return;
    }
    const int j0 = 16 * (g - nA);
    for (int e = tid; e < kBlk * 16; e += kBlkThreads) {
        const int i = e >> 4, j = e & 15;
        Ws[i][j] = (i < nb) ? X[(size_t)(kb + i) * lda + j0 + j] : 0.0;
    }
    __syncthreads();
    const int r0 = 16 * wave;
    if (r0 >= nb) return;   // no barrier follows
    const int ra = r0 + (lane & 15);
    double av[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
        const int t = 4 * u + (lane >> 4);
        av[u] = (ra < nb && t <= ra) ? X[(size_t)(kb + ra) * lda + kb + t] : 0.0;   // X_kk lower
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < KS; ++u) acc = mfma64(av[u], Ws[4 * u + (lane >> 4)][lane & 15], acc);
    const int j = j0 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = r0 + mfma64_row(lane, r);
        if (i < nb) {
            X[(size_t)(kb + i) * lda + j] = acc[r];
            Rinv[(size_t)j * lda + kb + i] = acc[r];
            Rinv[(size_t)(kb + i) * lda + j] = 0.0;
        }
    }
}

// K3: one wave per 16 x 16 tile below the block column: the lower tiles of
// the trailing matrix (lower_pair order), then the W tiles left of the
// trailing matrix.  A tile is read and written by its own wave only.
// skip: the first skip lower tiles (those of the next diagonal block, which
// its own K1 updates) are left out.
__device__ __attribute__((always_inline)) void chol_trail_body(
    int m, int lda, int kb, const double *__restrict__ S, double *__restrict__ L,
    double *__restrict__ X, int skip) {
    constexpr int KS = kBlk / 4;
    const int lane = threadIdx.x & 63;
    const int t = skip + blockIdx.x * (kBlkThreads / 64) + (threadIdx.x >> 6);
    const int k0 = kb + kBlk;   // first row below the block (the block is full)
    const int R = m - k0, nr = (R + 15) / 16, npairs = nr * (nr + 1) / 2;
    const int nc = k0 / 16;
    if (t >= npairs + nr * nc) return;
    const double *src = (kb == 0) ? S : L;
    const bool sym = t < npairs;
    int bi, bj;
    if (sym) {
        lower_pair(t, bi, bj);
    } else {
        bi = (t - npairs) / nc;
        bj = (t - npairs) - bi * nc;
    }
    const int ia = k0 + bi * 16 + (lane & 15);
    const int jb = (sym ? k0 : 0) + bj * 16 + (lane & 15);   // column of B (and of the tile)
    double av[KS], bv[KS], old[4];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
        const int tk = 4 * u + (lane >> 4);
        av[u] = (ia < m) ? L[(size_t)ia * lda + kb + tk] : 0.0;
        if (sym) {
            bv[u] = (jb < m) ? L[(size_t)jb * lda + kb + tk] : 0.0;
        } else {
            // X_kj: the block row of X left of the diagonal, X_kk (lower) on it
            const bool valid = jb < kb || jb - kb <= tk;
            bv[u] = valid ? X[(size_t)(kb + tk) * lda + jb] : 0.0;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = k0 + bi * 16 + mfma64_row(lane, r);
        double v = 0.0;
        if (sym) {
            if (i < m && jb <= i) v = src[(size_t)i * lda + jb];
        } else {
            if (i < m && jb < kb) v = X[(size_t)i * lda + jb];   // W; zero right of kb
        }
        old[r] = v;
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < KS; ++u) acc = mfma64(av[u], bv[u], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = k0 + bi * 16 + mfma64_row(lane, r);
        if (sym) {
            if (i < m && jb <= i) L[(size_t)i * lda + jb] = old[r] - acc[r];
        } else {
            if (i < m) X[(size_t)i * lda + jb] = old[r] - acc[r];
        }
    }
}

// K3 of block column kb beside K1 of block column kb + kBlk: the last
// workgroup factors the next diagonal block (applying its share of this
// update itself), the others update the rest of the trailing matrix and W.
__global__ __launch_bounds__(kBlkThreads) void chol_trail_block_kernel(
    int m, int lda, int kb, const double *__restrict__ S, double *__restrict__ L,
    double *__restrict__ X, double *__restrict__ Rinv, int32_t *__restrict__ info, int skip) {
    const size_t off = diag_offset(m, lda);
    if (blockIdx.x == gridDim.x - 1) {
        chol_block_body(m, lda, kb + kBlk, S + off, L + off, X + off, Rinv + off, info, true);
        return;
    }
    chol_trail_body(m, lda, kb, S + off, L + off, X + off, skip);
}

__global__ void assemble_kernel(int m, const double *__restrict__ Hp,
                                const double *__restrict__ h, double *__restrict__ A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
    double v = 0.5 * (Hp[idx] + Hp[(int64_t)j * m + i]);
    if (i == j) v = h[i];
    A[idx] = v;
}

}  // namespace

size_t chol_workspace(int m) {
    return (size_t)2 * m * m * sizeof(double);
}

void chol_inverse(hipStream_t s, int m, const double *S, double *Rinv,
                  double *work, int32_t *info, int sb) {
    TM_REQUIRE(m >= 1 && m <= 2048, TM_ENOTSUP, "Cholesky supports m <= 2048");
    const int b = (sb > 0 && sb < m) ? sb : m;   // diagonal block size
    TM_REQUIRE(b == m || (b % kBlk == 0 && m % b == 0), TM_EINVAL,
               "block-diagonal Cholesky: the block size must divide m and be a multiple of 64");
    const unsigned nd = (unsigned)(m / b);
    double *L = work, *X = work + (size_t)m * m;
    // K1 of block column 0; then per block column K2 and, while rows remain,
    // K3 together with the next block column's K1 (all diagonal blocks of a
    // block-diagonal S side by side)
    hipLaunchKernelGGL(chol_block_kernel, dim3(1, nd), dim3(kBlkThreads), 0, s, b, m, 0, S, L, X,
                       Rinv, info);
    for (int kb = 0; kb < b; kb += kBlk) {
        const int nb = std::min(kBlk, b - kb), R = b - kb - nb;
        const int nA = (R + 15) / 16, nB = kb / 16;
        if (nA + nB > 0)
            hipLaunchKernelGGL(chol_panel_kernel, dim3(nA + nB, nd), dim3(kBlkThreads), 0, s, b, m,
                               kb, S, L, X, Rinv);
        if (R > 0) {
            const int nr = (R + 15) / 16, tiles = nr * (nr + 1) / 2 + nr * ((kb + kBlk) / 16);
            const int nt = (std::min(kBlk, R) + 15) / 16, skip = nt * (nt + 1) / 2;
            const int per = kBlkThreads / 64;
            hipLaunchKernelGGL(chol_trail_block_kernel,
                               dim3((tiles - skip + per - 1) / per + 1, nd), dim3(kBlkThreads), 0, s,
                               b, m, kb, S, L, X, Rinv, info, skip);
        }
        TM_HIP(hipGetLastError());
    }
}

void assemble_subspace_matrix(hipStream_t s, int m, const double *Hp,
                              const double *h, double *A) {
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, m, Hp, h, A);
    TM_HIP(hipGetLastError());
}

}  // namespace tmin
