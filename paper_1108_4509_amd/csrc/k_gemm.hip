// Tall-skinny products on CDNA4 matrix cores (v_mfma_*_16x16x4):
//
//   gram : out = A^T B'        (m x m, reduction over the N rows) -- the
//          Gram products H' = C^T X' (Fig. 2, step (6)) and S = C^T C
//          (Fig. 4, step (1)); B' = B - A diag(h) forms X' = X - C H_D
//          (Fig. 2, step (5)) while the tile is loaded.
//   rot  : out = A W (+ epilogue)  (N x m times m x m) -- C H' with the
//          gradient epilogue of Fig. 2 step (7), the triangular product
//          C R^{-1} = C D + C R' of Fig. 4 step (4) / Eq. 13, and the
//          subspace rotation C U of the Rayleigh-Ritz step (Eq. 9).
//
// Operands are staged through LDS by 256-lane workgroups (2 x 2 waves); each
// wave owns a (B/2) x (B/2) output patch made of 16 x 16 MFMA blocks.  Matrix
// core precision TM is FP64 or FP32; loads may convert from FP64 storage
// (the MP2 policy keeps C in FP64 but runs steps (6) and (7) in FP32).
// Workgroup b runs on XCD b % 8, so the launch maps consecutive logical tiles
// to one XCD: row chunks of the tall operand stay in that XCD's L2.
#include "tm_common.h"

namespace tmin {
namespace {

// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  They differ in where D[i][j] lands: the FP32 form puts it in
// lane j + 16 (i / 4), register i % 4; the FP64 form in lane j + 16 (i % 4),
// register i / 4.  row(lane, r) returns i for register r of a lane.
template <typename TM> struct Mfma;
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    __device__ static inline acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    __device__ static inline acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

constexpr int kThreads = 256;
constexpr int kGramKT = 16;   // rows of A and B per LDS stage
constexpr int kRotKT = 16;    // columns of A (rows of W) per LDS stage

__device__ inline int xcd_logical(int grid) {
    const int b = blockIdx.x;
    return (b & 7) * (grid >> 3) + (b >> 3);
}

// Decode the upper-triangular tile index t into (ti, tj), ti <= tj < T.
__device__ inline void upper_tile(int t, int T, int &ti, int &tj) {
    int i = 0;
    while (t >= T - i) {
        t -= T - i;
        ++i;
    }
    ti = i;
    tj = i + t;
}

template <typename TA, typename TM, int BM, bool SHIFT>
__global__ __launch_bounds__(kThreads) void gram_kernel(
    int64_t n, int m, int ld, const TA *__restrict__ A, const TA *__restrict__ B,
    const double *__restrict__ h, int T, int ntiles, bool symmetric,
    int64_t rows_per_split, double *__restrict__ partials) {
    constexpr int PAD = 4;
    constexpr int WM = BM / 2;
    constexpr int NB = WM / 16;
    constexpr int PER = kGramKT * BM / kThreads;   // elements per lane per operand
    using Acc = typename Mfma<TM>::acc_t;

    __shared__ TM As[kGramKT][BM + PAD];
    __shared__ TM Bs[kGramKT][BM + PAD];

    const int logical = xcd_logical(gridDim.x);
    const int split = logical / ntiles;
    const int tile = logical - split * ntiles;
    int ti, tj;
    if (symmetric) upper_tile(tile, T, ti, tj);
    else { ti = tile / T; tj = tile - ti * T; }
    const int i0 = ti * BM, j0 = tj * BM;
    const int64_t k_begin = (int64_t)split * rows_per_split;
    int64_t k_end = k_begin + rows_per_split;
    if (k_end > n) k_end = n;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave >> 1, wj = wave & 1;

    Acc acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    TM ra[PER], rb[PER];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kThreads;
            const int row = e / BM, col = e - (e / BM) * BM;
            const int64_t k = k0 + row;
            const bool rok = k < k_end;
            const int ci = i0 + col, cj = j0 + col;
            ra[q] = (rok && ci < ld) ? (TM)A[k * ld + ci] : (TM)0;
            if (rok && cj < ld) {
                if constexpr (SHIFT) {
                    const double x = (double)B[k * ld + cj] - (double)A[k * ld + cj] * h[cj];
                    rb[q] = (TM)x;
                } else {
                    rb[q] = (TM)B[k * ld + cj];
                }
            } else {
                rb[q] = (TM)0;
            }
        }
    };

    if (k_begin < k_end) load(k_begin);
    for (int64_t k0 = k_begin; k0 < k_end; k0 += kGramKT) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kThreads;
            const int row = e / BM, col = e - (e / BM) * BM;
            As[row][col] = ra[q];
            Bs[row][col] = rb[q];
        }
        __syncthreads();
        if (k0 + kGramKT < k_end) load(k0 + kGramKT);
#pragma unroll
        for (int kk = 0; kk < kGramKT; kk += 4) {
            TM fa[NB], fb[NB];
            const int kr = kk + (lane >> 4);
#pragma unroll
            for (int a = 0; a < NB; ++a) fa[a] = As[kr][wi * WM + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < NB; ++b) fb[b] = Bs[kr][wj * WM + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = Mfma<TM>::op(fa[a], fb[b], acc[a][b]);
        }
    }

    double *P = partials + (int64_t)split * m * m;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi * WM + a * 16 + Mfma<TM>::row(lane, r);
                const int j = j0 + wj * WM + b * 16 + (lane & 15);
                if (i < m && j < m) P[(int64_t)i * m + j] = (double)acc[a][b][r];
            }
}

__global__ void gram_reduce_kernel(int m, int nsplit, int BM, bool symmetric,
                                   bool zero_diag,
                                   const double *__restrict__ partials,
                                   double *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
    int64_t src = idx;
    if (symmetric && (i / BM) > (j / BM)) src = (int64_t)j * m + i;
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += partials[(int64_t)p * m * m + src];
    if (zero_diag && i == j) s = 0.0;
    out[idx] = s;
}

int gram_tile(int ld) { return ld >= 512 ? 128 : 64; }

void gram_shape(int64_t n, int m, int &BM, int &T, int &nsplit) {
    const int ld = leading_dim(m);
    BM = gram_tile(ld);
    T = (ld + BM - 1) / BM;
    // aim at ~1024 workgroups, at most 16 MiB of FP64 partials, and at least
    // 64 rows per split; nsplit is a multiple of 8 (XCD mapping)
    const int ntiles_full = T * T;
    int64_t ns = 1024 / ntiles_full;
    const int64_t cap_bytes = (int64_t)16 << 20;
    int64_t cap = cap_bytes / ((int64_t)m * m * 8);
    if (ns > cap) ns = cap;
    int64_t cap_rows = n / 64;
    if (ns > cap_rows) ns = cap_rows;
    ns = (ns + 7) / 8 * 8;
    if (ns < 8) ns = 8;
    nsplit = (int)ns;
}

template <typename TA, typename TM, typename TO, int EPI, int BR, int BC>
__global__ __launch_bounds__(kThreads) void rot_kernel(
    int64_t n, int m, int ld, const TA *__restrict__ A, const TM *__restrict__ W,
    const TA *__restrict__ X, const double *__restrict__ vec, TO *__restrict__ out,
    int nrb, int ncb) {
    constexpr int WR = BR / 2, WC = BC / 2;
    constexpr int NBR = WR / 16, NBC = WC / 16;
    constexpr int PA = BR * kRotKT / kThreads;
    constexpr int PW = BC * kRotKT / kThreads;
    using Acc = typename Mfma<TM>::acc_t;

    __shared__ TM As[BR][kRotKT + 1];
    __shared__ TM Ws[kRotKT][BC + 4];

    const int logical = xcd_logical(gridDim.x);
    if (logical >= nrb * ncb) return;
    const int rb = logical / ncb, cb = logical - (logical / ncb) * ncb;
    const int64_t r0 = (int64_t)rb * BR;
    const int c0 = cb * BC;
    int kend = ld;
    if (EPI == EPI_TRMM && c0 + BC < kend) kend = c0 + BC;   // W strictly upper

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = wave >> 1, wc = wave & 1;

    Acc acc[NBR][NBC];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    TM ra[PA], rw[PW];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int e = tid + q * kThreads;
            const int row = e / kRotKT, col = e - (e / kRotKT) * kRotKT;
            const int64_t r = r0 + row;
            ra[q] = (r < n) ? (TM)A[r * ld + k0 + col] : (TM)0;
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int e = tid + q * kThreads;
            const int row = e / BC, col = e - (e / BC) * BC;
            const int c = c0 + col;
            rw[q] = (c < ld) ? W[(int64_t)(k0 + row) * ld + c] : (TM)0;
        }
    };

    load(0);
    for (int k0 = 0; k0 < kend; k0 += kRotKT) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int e = tid + q * kThreads;
            As[e / kRotKT][e - (e / kRotKT) * kRotKT] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int e = tid + q * kThreads;
            Ws[e / BC][e - (e / BC) * BC] = rw[q];
        }
        __syncthreads();
        if (k0 + kRotKT < kend) load(k0 + kRotKT);
#pragma unroll
        for (int kk = 0; kk < kRotKT; kk += 4) {
            TM fa[NBR], fb[NBC];
            const int kc = kk + (lane >> 4);
#pragma unroll
            for (int a = 0; a < NBR; ++a) fa[a] = As[wr * WR + a * 16 + (lane & 15)][kc];
#pragma unroll
            for (int b = 0; b < NBC; ++b) fb[b] = Ws[kc][wc * WC + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < NBR; ++a)
#pragma unroll
                for (int b = 0; b < NBC; ++b) acc[a][b] = Mfma<TM>::op(fa[a], fb[b], acc[a][b]);
        }
    }

#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + wr * WR + a * 16 + Mfma<TM>::row(lane, r);
                const int col = c0 + wc * WC + b * 16 + (lane & 15);
                if (row >= n || col >= ld) continue;
                const int64_t e = row * ld + col;
                const TA v = (TA)acc[a][b][r];
                if constexpr (EPI == EPI_NONE) {
                    out[e] = (TO)v;
                } else if constexpr (EPI == EPI_GRAD) {
                    const TA xp = X[e] - A[e] * (TA)vec[col];
                    out[e] = (TO)((TA)-2 * (xp - v));
                } else {
                    out[e] = (TO)(A[e] * (TA)vec[col] + v);
                }
            }
}

template <typename TM>
__global__ void pad_kernel(int m, int ld, const double *__restrict__ W,
                           bool strict_upper, TM *__restrict__ Wpad,
                           double *__restrict__ diag) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ld * ld) return;
    const int i = (int)(idx / ld), j = (int)(idx - (int64_t)i * ld);
    double v = 0.0;
    if (i < m && j < m && (!strict_upper || j > i)) v = W[(int64_t)i * m + j];
    Wpad[idx] = (TM)v;
    if (diag && i == 0) diag[j] = (j < m) ? W[(int64_t)j * m + j] : 0.0;
}

}  // namespace

size_t gram_workspace(int64_t n, int m) {
    int BM, T, nsplit;
    gram_shape(n, m, BM, T, nsplit);
    return (size_t)nsplit * m * m * sizeof(double);
}

template <typename TA, typename TM>
void gram(hipStream_t s, int64_t n, int m, const TA *A, const TA *B,
          const double *h, bool zero_diag, bool symmetric, double *partials,
          double *out, bool reduce) {
    const int ld = leading_dim(m);
    int BM, T, nsplit;
    gram_shape(n, m, BM, T, nsplit);
    if (h) symmetric = false;
    const int ntiles = symmetric ? T * (T + 1) / 2 : T * T;
    const int64_t rows = ((n + nsplit - 1) / nsplit + kGramKT - 1) / kGramKT * kGramKT;
    const int grid = ntiles * nsplit;   // multiple of 8
#define TM_GRAM(BMV, SH)                                                            \
    hipLaunchKernelGGL((gram_kernel<TA, TM, BMV, SH>), dim3(grid), dim3(kThreads), 0, s, \
                       n, m, ld, A, B, h, T, ntiles, symmetric, rows, partials)
    if (BM == 128) {
        if (h) TM_GRAM(128, true); else TM_GRAM(128, false);
    } else {
        if (h) TM_GRAM(64, true); else TM_GRAM(64, false);
    }
#undef TM_GRAM
    TM_HIP(hipGetLastError());
    if (!reduce) return;
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       s, m, nsplit, BM, symmetric, zero_diag, partials, out);
    TM_HIP(hipGetLastError());
}

template <typename TA, typename TM, typename TO>
void rot(hipStream_t s, int64_t n, int m, const TA *A, const TM *Wpad, int epi,
         const TA *X, const double *vec, TO *out) {
    const int ld = leading_dim(m);
    constexpr int BR = 64, BC = 64;
    const int nrb = (int)((n + BR - 1) / BR);
    const int ncb = (ld + BC - 1) / BC;
    int grid = nrb * ncb;
    grid = (grid + 7) / 8 * 8;
#define TM_ROT(E)                                                                      \
    hipLaunchKernelGGL((rot_kernel<TA, TM, TO, E, BR, BC>), dim3(grid), dim3(kThreads), \
                       0, s, n, m, ld, A, Wpad, X, vec, out, nrb, ncb)
    if (epi == EPI_NONE) TM_ROT(EPI_NONE);
    else if (epi == EPI_GRAD) TM_ROT(EPI_GRAD);
    else TM_ROT(EPI_TRMM);
#undef TM_ROT
    TM_HIP(hipGetLastError());
}

template <typename TM>
void pad_matrix(hipStream_t s, int m, const double *W, bool strict_upper,
                TM *Wpad, double *diag) {
    const int ld = leading_dim(m);
    const int64_t total = (int64_t)ld * ld;
    hipLaunchKernelGGL(pad_kernel<TM>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       m, ld, W, strict_upper, Wpad, diag);
    TM_HIP(hipGetLastError());
}

template void gram<double, double>(hipStream_t, int64_t, int, const double *, const double *, const double *, bool, bool, double *, double *, bool);
template void gram<float, float>(hipStream_t, int64_t, int, const float *, const float *, const double *, bool, bool, double *, double *, bool);
template void gram<double, float>(hipStream_t, int64_t, int, const double *, const double *, const double *, bool, bool, double *, double *, bool);
template void rot<double, double, double>(hipStream_t, int64_t, int, const double *, const double *, int, const double *, const double *, double *);
template void rot<float, float, float>(hipStream_t, int64_t, int, const float *, const float *, int, const float *, const double *, float *);
template void rot<double, float, float>(hipStream_t, int64_t, int, const double *, const float *, int, const double *, const double *, float *);
template void rot<double, float, double>(hipStream_t, int64_t, int, const double *, const float *, int, const double *, const double *, double *);
template void pad_matrix<double>(hipStream_t, int, const double *, bool, double *, double *);
template void pad_matrix<float>(hipStream_t, int, const double *, bool, float *, double *);

}  // namespace tmin
