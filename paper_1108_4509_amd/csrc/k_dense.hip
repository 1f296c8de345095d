// Dense m x m FP64 kernels of the iteration: the Cholesky factorization and
// triangular inverse of Fig. 4 (steps (2) and (3)), and the assembly of the
// m x m H of Eq. 9 from the pieces of Algorithm-2.
//
// The factorization is O(m^3) with m <= 1024, so it is latency-bound; it runs
// as one workgroup of 1024 lanes with the matrix in a device workspace
// (resident in L2) and the current panel staged in LDS.
#include "tm_common.h"

#include <cmath>

namespace tmin {
namespace {

constexpr int kDenseThreads = 1024;
constexpr int NBMAX = 32;
constexpr int kStage = 17920;   // doubles of LDS staging (140 KiB)

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

// Factor the nb x nb diagonal block D = L_kk L_kk^T (lower, in LDS) in place
// and build Dinv = L_kk^{-1}, one element per lane of the workgroup
// (requires NB * NB <= blockDim).  Returns false on a bad pivot.
template <int NB>
__device__ bool block_chol_inv(int nb, double (*D)[NB + 1], double (*Dinv)[NB + 1],
                               const double *Sdiag) {
    const int t = threadIdx.x;
    const int i = t / NB, j = t % NB;
    const bool mine = t < NB * NB && i < nb && j < nb;
    bool ok = true;
    if (mine) Dinv[i][j] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        const double dkk = D[k][k];
        if (!(dkk > kPivotTol * fabs(Sdiag[k]))) ok = false;
        const double lik = mine ? D[i][k] : 0.0;
        const double ljk = mine ? D[j][k] : 0.0;
        __syncthreads();
        if (mine) {
            if (j > k && j <= i) D[i][j] -= lik * ljk / dkk;
            else if (j == k && i > k) D[i][k] = lik / sqrt(dkk);
            else if (i == k && j == k) D[k][k] = sqrt(dkk);
        }
        __syncthreads();
    }
    if (!ok) return false;
    // Dinv = L^{-1}: row k scaled by 1/l_kk, then eliminated from the rows below
    for (int k = 0; k < nb; ++k) {
        if (mine && i == k) Dinv[k][j] /= D[k][k];
        __syncthreads();
        if (mine && i > k) Dinv[i][j] -= D[i][k] * Dinv[k][j];
        __syncthreads();
    }
    return true;
}

// S = L L^T (L lower; S = R^T R with R = L^T) and Rinv = R^{-1} = L^{-T}.
// Blocked right-looking Cholesky with NB-wide panels: the diagonal block is
// factored and inverted in LDS by the whole workgroup, the panel
// L_ik = S_ik L_kk^{-T} and the trailing update S_ij -= L_ik L_jk^T run on FP64
// matrix cores (16 x 16 blocks spread over the 16 waves) with the panel staged
// in LDS.  The inverse X = L^{-1} is then built block row by block row,
// X_i,0:i = -L_ii^{-1} (L_i,0:i X_0:i,0:i), again on matrix cores.
// work: L (m*m), X (m*m), T (NB*m) doubles.
template <int NB>
__global__ __launch_bounds__(kDenseThreads) void chol_inv_kernel(
    int m, const double *__restrict__ S, double *__restrict__ Rinv,
    double *__restrict__ work, int32_t *__restrict__ info) {
    __shared__ double stage[kStage];
    __shared__ double D[NB][NB + 1];
    __shared__ double Dinv[NB][NB + 1];
    __shared__ double Sd[NB];
    constexpr int PS = NB + 1;   // row stride of the staged panel
    double *L = work;
    double *X = work + (size_t)m * m;
    double *T = X + (size_t)m * m;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int nwaves = kDenseThreads / 64;
    for (int64_t e = tid; e < (int64_t)m * m; e += kDenseThreads) {
        L[e] = S[e];
        X[e] = 0.0;
    }
    __syncthreads();

    for (int kb = 0; kb < m; kb += NB) {
        const int nb = (m - kb < NB) ? (m - kb) : NB;
        if (tid < NB * NB) {
            const int i = tid / NB, j = tid % NB;
            D[i][j] = (i < nb && j <= i) ? L[(size_t)(kb + i) * m + kb + j] : 0.0;
        }
        if (tid < nb) Sd[tid] = S[(size_t)(kb + tid) * m + kb + tid];
        __syncthreads();
        if (!block_chol_inv<NB>(nb, D, Dinv, Sd)) {
            if (tid == 0) info[0] = kb + 1;
            return;   // uniform: every lane saw the same pivots
        }
        if (tid < NB * NB) {
            const int i = tid / NB, j = tid % NB;
            if (i < nb && j <= i) {
                L[(size_t)(kb + i) * m + kb + j] = D[i][j];
                X[(size_t)(kb + i) * m + kb + j] = Dinv[i][j];
            }
        }
        const int R = m - kb - nb;          // rows below the diagonal block
        // stage S_ik (R x nb), then the panel L_ik = S_ik Dinv^T on matrix cores
        for (int e = tid; e < R * NB; e += kDenseThreads) {
            const int r = e / NB, c = e % NB;
            stage[r * PS + c] = (c < nb) ? L[(size_t)(kb + nb + r) * m + kb + c] : 0.0;
        }
        __syncthreads();
        const int nbr = (R + 15) / 16;
        // each wave computes whole 16-row strips of the panel (all NB columns);
        // at most kStrips strips per wave (m / 16 / 16 for the largest m)
        constexpr int kStrips = (NB == 32) ? 2 : 4;
        d4 pacc[kStrips][NB / 16];
#pragma unroll
        for (int sidx = 0; sidx < kStrips; ++sidx) {
            const int bi = wave + sidx * nwaves;
            if (bi >= nbr) break;
            const int ra = bi * 16 + (lane & 15);
#pragma unroll
            for (int bj = 0; bj < NB / 16; ++bj) {
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int t0 = 0; t0 < nb; t0 += 4) {
                    const int k = t0 + (lane >> 4);
                    const double a = (ra < R) ? stage[ra * PS + k] : 0.0;
                    const double b = Dinv[bj * 16 + (lane & 15)][k];   // B[k][j] = Dinv[j][k]
                    acc = mfma64(a, b, acc);
                }
                pacc[sidx][bj] = acc;
            }
        }
        __syncthreads();   // all reads of the staged S_ik done
#pragma unroll
        for (int sidx = 0; sidx < kStrips; ++sidx) {
            const int bi = wave + sidx * nwaves;
            if (bi >= nbr) break;
#pragma unroll
            for (int bj = 0; bj < NB / 16; ++bj) {
                const d4 acc = pacc[sidx][bj];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = bi * 16 + mfma64_row(lane, r), c = bj * 16 + (lane & 15);
                    if (i < R && c < nb) {
                        stage[i * PS + c] = acc[r];
                        L[(size_t)(kb + nb + i) * m + kb + c] = acc[r];
                    }
                }
            }
        }
        __syncthreads();
        // trailing update of the lower triangle (disjoint from the panel columns)
        const int npairs = nbr * (nbr + 1) / 2;
        for (int p = wave; p < npairs; p += nwaves) {
            int bi, bj;
            lower_pair(p, bi, bj);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = bi * 16 + (lane & 15), rb = bj * 16 + (lane & 15);
            for (int t0 = 0; t0 < nb; t0 += 4) {
                const int k = t0 + (lane >> 4);
                const double a = (ra < R) ? stage[ra * PS + k] : 0.0;
                const double b = (rb < R) ? stage[rb * PS + k] : 0.0;
                acc = mfma64(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < R && j <= i) L[(size_t)(kb + nb + i) * m + kb + nb + j] -= acc[r];
            }
        }
        __syncthreads();
    }

    // inverse, block row ib: X_ib,0:ib = -Dinv_ib (L_ib,0:ib X_0:ib,0:ib)
    for (int ib = NB; ib < m; ib += NB) {
        const int nb = (m - ib < NB) ? (m - ib) : NB;
        const int SS = ib + 1;
        for (int e = tid; e < nb * ib; e += kDenseThreads) {
            const int r = e / ib, k = e - (e / ib) * ib;
            stage[r * SS + k] = L[(size_t)(ib + r) * m + k];
        }
        for (int e = tid; e < NB * NB; e += kDenseThreads) {
            const int r = e / NB, c = e % NB;
            Dinv[r][c] = (r < nb && c <= r) ? X[(size_t)(ib + r) * m + ib + c] : 0.0;
        }
        __syncthreads();
        const int nbi = (nb + 15) / 16, nbj = (ib + 15) / 16;
        for (int p = wave; p < nbi * nbj; p += nwaves) {
            const int bi = p / nbj, bj = p - (p / nbj) * nbj;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = bi * 16 + (lane & 15), jc = bj * 16 + (lane & 15);
            for (int k0 = (bj * 16) & ~3; k0 < ib; k0 += 4) {
                const int k = k0 + (lane >> 4);
                const double a = (ra < nb && k < ib) ? stage[ra * SS + k] : 0.0;
                const double b = (k < ib && jc < ib) ? X[(size_t)k * m + jc] : 0.0;
                acc = mfma64(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < nb && j < ib) T[(size_t)i * m + j] = acc[r];
            }
        }
        __syncthreads();
        // X_ib,0:ib = -Dinv (nb x nb) T (nb x ib) on matrix cores
        for (int p = wave; p < nbi * nbj; p += nwaves) {
            const int bi = p / nbj, bj = p - (p / nbj) * nbj;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = bi * 16 + (lane & 15), jc = bj * 16 + (lane & 15);
            for (int k0 = 0; k0 < nb; k0 += 4) {
                const int k = k0 + (lane >> 4);
                const double a = (ra < nb) ? Dinv[ra][k] : 0.0;
                const double b = (k < nb && jc < ib) ? T[(size_t)k * m + jc] : 0.0;
                acc = mfma64(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < nb && j < ib) X[(size_t)(ib + i) * m + j] = -acc[r];
            }
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)m * m; e += kDenseThreads) {
        const int i = (int)(e / m), j = (int)(e % m);
        Rinv[e] = (j >= i) ? X[(size_t)j * m + i] : 0.0;
    }
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
    return ((size_t)2 * m * m + (size_t)m * NBMAX) * sizeof(double);
}

void chol_inverse(hipStream_t s, int m, const double *S, double *Rinv,
                  double *work, int32_t *info) {
    TM_REQUIRE(m >= 1 && m <= 1024, TM_ENOTSUP, "Cholesky supports m <= 1024");
    // the staged panel (m x (NB+1) doubles) must fit the LDS staging area
    if (m <= 512)
        hipLaunchKernelGGL(chol_inv_kernel<32>, dim3(1), dim3(kDenseThreads), 0, s, m, S,
                           Rinv, work, info);
    else
        hipLaunchKernelGGL(chol_inv_kernel<16>, dim3(1), dim3(kDenseThreads), 0, s, m, S,
                           Rinv, work, info);
    TM_HIP(hipGetLastError());
}

void assemble_subspace_matrix(hipStream_t s, int m, const double *Hp,
                              const double *h, double *A) {
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, m, Hp, h, A);
    TM_HIP(hipGetLastError());
}

}  // namespace tmin
