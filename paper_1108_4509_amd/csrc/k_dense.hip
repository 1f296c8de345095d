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

// Factor the nb x nb diagonal block D = L_kk L_kk^T and build L_kk^{-1} at the
// same time, with the whole workgroup: Gaussian elimination without pivoting
// on the augmented NB x 2NB matrix [D | I], double-buffered in LDS so that one
// barrier per step suffices.  Afterwards the D half holds U = diag(d) L1^T and
// the I half holds L1^{-1} (L1 unit lower), so L = L1 diag(d)^{1/2} and
// L^{-1} = diag(d)^{-1/2} L1^{-1}.  Rows and columns at or beyond nb (last,
// partial panel) are padded with the identity.  Writes L_kk (lower), the
// diagonal block of X = L^{-1} (with zeros above its diagonal), the same block
// of Rinv = X^T (upper), and Dinv = L_kk^{-1} in LDS.  Returns false (the
// same on every lane) if a pivot is not clearly positive.
template <int NB>
__device__ bool diag_factor(int m, int kb, int nb, const double *__restrict__ src,
                            double *__restrict__ L, double *__restrict__ X,
                            double *__restrict__ Rinv, const double *Sd, double *buf,
                            double *piv, double (*Dinv)[NB + 1]) {
    constexpr int W2 = 2 * NB, RS = W2 + 1;
    double *A0 = buf, *A1 = buf + NB * RS;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * W2; e += kDenseThreads) {
        const int i = e / W2, c = e % W2;
        double v;
        if (c < NB) {
            v = (i == c) ? 1.0 : 0.0;
            if (i < nb && c < nb) {
                const int r = i > c ? i : c, q = i > c ? c : i;   // lower part
                v = src[(size_t)(kb + r) * m + kb + q];
            }
        } else {
            v = (i == c - NB) ? 1.0 : 0.0;
        }
        A0[i * RS + c] = v;
    }
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < NB; ++k) {
        const double *cur = (k & 1) ? A1 : A0;
        double *nxt = (k & 1) ? A0 : A1;
        const double d = cur[k * RS + k];
        if (!(d > kPivotTol * fabs(Sd[k]))) ok = false;
        if (tid == 0) piv[k] = d;
        const double inv = 1.0 / d;
        for (int e = tid; e < NB * W2; e += kDenseThreads) {
            const int i = e / W2, c = e % W2;
            double v = cur[i * RS + c];
            if (i > k) v -= cur[i * RS + k] * inv * cur[k * RS + c];
            nxt[i * RS + c] = v;
        }
        __syncthreads();
    }
    if (!ok) return false;
    const double *F = (NB & 1) ? A1 : A0;
    for (int e = tid; e < NB * NB; e += kDenseThreads) {
        const int i = e / NB, c = e % NB;
        if (i < nb && c < nb) {
            if (c <= i) L[(size_t)(kb + i) * m + kb + c] = F[c * RS + i] / sqrt(piv[c]);
            const double xv = F[i * RS + NB + c] / sqrt(piv[i]);   // 0 above the diagonal
            Dinv[i][c] = xv;
            X[(size_t)(kb + i) * m + kb + c] = xv;
            if (c <= i) Rinv[(size_t)(kb + c) * m + kb + i] = xv;
        } else {
            Dinv[i][c] = 0.0;
        }
    }
    return true;
}

// S = L L^T (L lower; S = R^T R with R = L^T) and Rinv = R^{-1} = L^{-T}
// (upper triangle only; the caller clears the rest).
// Blocked right-looking Cholesky with NB-wide panels: the diagonal block is
// factored and inverted by diag_factor, the panel L_ik = S_ik L_kk^{-T} and the
// trailing update S_ij -= L_ik L_jk^T run on FP64 matrix cores (16 x 16 blocks
// spread over the 16 waves) with the panel staged in LDS.  The first panel
// reads S directly, later ones the updated copy in L.  The inverse
// X = L^{-1} is then assembled by recursive doubling from the NB x NB diagonal
// inverses: for consecutive diagonal blocks A, C of size b,
//   X_CA = -X_C (L_CA X_A),
// all pairs of a level at once, b = NB, 2 NB, 4 NB, ...
// work: L (m*m), X (m*m), T (m*m) doubles.
template <int NB>
__global__ __launch_bounds__(kDenseThreads) void chol_inv_kernel(
    int m, const double *__restrict__ S, double *__restrict__ Rinv,
    double *__restrict__ work, int32_t *__restrict__ info) {
    __shared__ double stage[kStage];
    __shared__ double Dinv[NB][NB + 1];
    __shared__ double Sd[NB];
    __shared__ double piv[NB];
    constexpr int PS = NB + 1;   // row stride of the staged panel
    double *L = work;
    double *X = work + (size_t)m * m;
    double *T = X + (size_t)m * m;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int nwaves = kDenseThreads / 64;

    for (int kb = 0; kb < m; kb += NB) {
        const int nb = (m - kb < NB) ? (m - kb) : NB;
        const double *src = (kb == 0) ? S : L;
        if (tid < NB) Sd[tid] = (tid < nb) ? S[(size_t)(kb + tid) * m + kb + tid] : 1.0;
        __syncthreads();
        if (!diag_factor<NB>(m, kb, nb, src, L, X, Rinv, Sd, stage, piv, Dinv)) {
            if (tid == 0) info[0] = kb + 1;
            return;   // uniform: every lane saw the same pivots
        }
        __syncthreads();
        const int R = m - kb - nb;          // rows below the diagonal block
        // stage S_ik (R x nb), then the panel L_ik = S_ik Dinv^T on matrix cores
        for (int e = tid; e < R * NB; e += kDenseThreads) {
            const int r = e / NB, c = e % NB;
            stage[r * PS + c] = (c < nb) ? src[(size_t)(kb + nb + r) * m + kb + c] : 0.0;
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
                if (i < R && j <= i) {
                    const size_t g = (size_t)(kb + nb + i) * m + kb + nb + j;
                    L[g] = src[g] - acc[r];
                }
            }
        }
        __syncthreads();
    }

    // recursive doubling of the inverse: level with block size b; operands
    // are read from L2 eight k-steps at a time to keep loads in flight
    for (int b = NB; b < m; b *= 2) {
        const int nblk = (m + b - 1) / b;
        const int npair = nblk / 2;
        const int nbi = b / 16, nbj = b / 16;
        const int work1 = npair * nbi * nbj;
        // phase 1: T_q = L_CA X_A  (rows of C: up to b, columns of A: b)
        for (int p = wave; p < work1; p += nwaves) {
            const int q = p / (nbi * nbj), rem = p - q * (nbi * nbj);
            const int bi = rem / nbj, bj = rem - (rem / nbj) * nbj;
            const int cA = 2 * q * b, rC = cA + b;
            const int nrC = (m - rC < b) ? (m - rC) : b;
            if (bi * 16 >= nrC) continue;
            const int ra = rC + bi * 16 + (lane & 15);
            const int jc = cA + bj * 16 + (lane & 15);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = (bj * 16) & ~3; k0 < b; k0 += 32) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int kk = k0 + 4 * u;
                    const int k = cA + kk + (lane >> 4);
                    const bool in = kk < b;
                    av[u] = (in && ra < m) ? L[(size_t)ra * m + k] : 0.0;
                    bv[u] = in ? X[(size_t)k * m + jc] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = mfma64(av[u], bv[u], acc);
            }
            double *Tq = T + (size_t)q * b * b;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < nrC) Tq[(size_t)i * b + j] = acc[r];
            }
        }
        __syncthreads();
        // phase 2: X_CA = -X_C T_q (and Rinv_AC = X_CA^T)
        for (int p = wave; p < work1; p += nwaves) {
            const int q = p / (nbi * nbj), rem = p - q * (nbi * nbj);
            const int bi = rem / nbj, bj = rem - (rem / nbj) * nbj;
            const int cA = 2 * q * b, rC = cA + b;
            const int nrC = (m - rC < b) ? (m - rC) : b;
            if (bi * 16 >= nrC) continue;
            const int ra = rC + bi * 16 + (lane & 15);
            const int kmax = (bi * 16 + 16 < nrC) ? bi * 16 + 16 : nrC;
            const double *Tq = T + (size_t)q * b * b;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < kmax; k0 += 32) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k0 + 4 * u + (lane >> 4);
                    const bool in = k < kmax;
                    av[u] = (in && ra < m) ? X[(size_t)ra * m + rC + k] : 0.0;
                    bv[u] = in ? Tq[(size_t)k * b + bj * 16 + (lane & 15)] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = mfma64(av[u], bv[u], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (i < nrC) {
                    X[(size_t)(rC + i) * m + cA + j] = -acc[r];
                    Rinv[(size_t)(cA + j) * m + rC + i] = -acc[r];
                }
            }
        }
        __syncthreads();
    }
}

__global__ void zero_lower_kernel(int m, double *__restrict__ A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)m * m) return;
    const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
    if (j < i) A[idx] = 0.0;
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
    return (size_t)3 * m * m * sizeof(double);
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
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(zero_lower_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       m, Rinv);
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
