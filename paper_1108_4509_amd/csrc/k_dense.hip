// Dense m x m FP64 kernels of the iteration: the Cholesky factorization and
// triangular inverse of Fig. 4 (steps (2) and (3)), and the assembly of the
// m x m H of Eq. 9 from the pieces of Algorithm-2.
//
// The factorization is O(m^3) with m <= 1024, so it is latency-bound; it runs
// as one workgroup of 1024 lanes with the matrix in a device workspace
// (resident in L2) and the current panel staged in LDS.
#include "tm_common.h"

#include <algorithm>
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

// Factor the NB x NB diagonal block D = L_kk L_kk^T and invert it, by one
// wave, on the augmented NB x 2NB matrix [D | I] staged in LDS (aug, row
// stride 2NB + 1): lane c keeps column c in registers (rows a[0..NB)).
// Gaussian elimination without pivoting: at step k every lane reads the
// multipliers a_ik / a_kk of lane k's column by readlane and updates its own
// column, so no barrier and no memory round trip is needed.  Afterwards the D half holds U = diag(d) L1^T and
// the I half L1^{-1} (L1 unit lower), so L = L1 diag(d)^{1/2} and
// L^{-1} = diag(d)^{-1/2} L1^{-1}.  Results go back to LDS: L_kk^T into the
// D half of aug, L_kk^{-1} (zero above the diagonal) into Dinv, the pivots d
// into piv.  For NB = 16 the upper 32 lanes repeat the last column.
__device__ inline double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

template <int NB>
__device__ void diag_factor_wave(int lane, double *aug, double *piv, double (*Dinv)[NB + 1]) {
    constexpr int NC = 2 * NB, RS = 2 * NB + 1;
    const int c = lane < NC ? lane : NC - 1;
    double a[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) a[i] = aug[i * RS + c];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        // the multipliers a_ik / a_kk come from lane k by readlane
        const double dk = readlane_f64(a[k], k);
        if (lane == 0) piv[k] = dk;
        // a_ic -= a_ik (a_kc / a_kk): one scaling per lane, one FMA per row
        const double rk = a[k] * (1.0 / dk);
#pragma unroll
        for (int i = k + 1; i < NB; ++i) a[i] = fma(-readlane_f64(a[i], k), rk, a[i]);
    }
    if (lane < NB) {
        // lane i: row i of L, L_iq = U_qi / sqrt(d_q) for q <= i, stored transposed
#pragma unroll
        for (int q = 0; q < NB; ++q) aug[q * RS + lane] = (q <= lane) ? a[q] / sqrt(piv[q]) : 0.0;
    } else if (lane < NC) {
        // lane NB + col: column col of X = diag(d)^{-1/2} L1^{-1}
        const int col = lane - NB;
#pragma unroll
        for (int i = 0; i < NB; ++i) Dinv[i][col] = (i >= col) ? a[i] / sqrt(piv[i]) : 0.0;
    }
}

// S = L L^T (L lower; S = R^T R with R = L^T) and Rinv = R^{-1} = L^{-T}
// (upper triangle only; the caller clears the rest), in one right-looking
// sweep over NB-wide panels that also carries the block forward substitution
// L X = I:
//   1. the diagonal block is factored and inverted by one wave (Dinv = L_kk^{-1});
//   2. the panel's rows of the inverse are finished, X_k = Dinv W_k, where W
//      holds I minus the updates of the earlier panels;
//   3. the panel L_ik = S_ik Dinv^T;
//   4. the trailing matrix S_ij -= L_ik L_jk^T (lower tiles) and the rows of W
//      below, W_i -= L_ik X_k, both on FP64 matrix cores with L_ik and X_k
//      staged in LDS.
// W lives in the X workspace (rows below the panel), so each entry of X is
// written once as final.  work: L (m*m), X (m*m) doubles.
template <int NB>
__global__ __launch_bounds__(kDenseThreads) void chol_inv_kernel(
    int m, const double *__restrict__ S, double *__restrict__ Rinv,
    double *__restrict__ work, int32_t *__restrict__ info) {
    __shared__ double stage[kStage];
    __shared__ double Dinv[NB][NB + 1];
    __shared__ double piv[NB];
    __shared__ double Sd[NB];
    __shared__ int ok_flag;
    constexpr int PS = NB + 1;   // row stride of the staged panel
    double *L = work;
    double *X = work + (size_t)m * m;
    constexpr int nwaves = kDenseThreads / 64;

    for (int kb = 0; kb < m; kb += NB) {
        // the lane index is made opaque per panel so that the many per-lane
        // offsets of the unrolled loops are not hoisted out of the panel loop
        // (their live ranges would exceed the register file)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wave = tid >> 6;
        const int nb = (m - kb < NB) ? (m - kb) : NB;
        const double *src = (kb == 0) ? S : L;
        const int R = m - kb - nb;          // rows below the diagonal block
        const int kw = kb + nb;             // columns of X_k and of the W update
        const int XSS = ((kw + 15) & ~15) + 1;
        double *XS = stage + kStage - NB * XSS;   // X_k (NB x kw), after the panel
        // (1) diagonal block: stage [D | I] (identity-padded beyond nb),
        // factor and invert it with one wave, then publish L_kk, the
        // diagonal block of X and of Rinv
        {
            constexpr int RSA = 2 * NB + 1;
            constexpr int NA = NB * 2 * NB, UA = (NA + kDenseThreads - 1) / kDenseThreads;
            double v[UA];
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const int e = tid + u * kDenseThreads;
                const int i = e / (2 * NB), c = e - (e / (2 * NB)) * (2 * NB);
                v[u] = (i == c || i == c - NB) ? 1.0 : 0.0;
                if (e < NA && c < NB && i < nb && c < nb) {
                    const int r = i > c ? i : c, q = i > c ? c : i;   // lower part
                    v[u] = src[(size_t)(kb + r) * m + kb + q];
                }
            }
            const double sd = (tid < nb) ? S[(size_t)(kb + tid) * m + kb + tid] : 1.0;
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const int e = tid + u * kDenseThreads;
                if (e < NA) stage[(e / (2 * NB)) * RSA + e % (2 * NB)] = v[u];
            }
            if (tid < NB) Sd[tid] = sd;
            __syncthreads();
            if (wave == 0) {
                diag_factor_wave<NB>(lane, stage, piv, Dinv);
                if (lane == 0) {
                    int ok = 1;
                    for (int k = 0; k < nb; ++k)
                        if (!(piv[k] > kPivotTol * fabs(Sd[k]))) ok = 0;
                    ok_flag = ok;
                }
            }
            __syncthreads();
            if (!ok_flag) {
                if (tid == 0) info[0] = kb + 1;
                return;   // uniform
            }
            for (int e = tid; e < NB * NB; e += kDenseThreads) {
                const int i = e / NB, c = e - (e / NB) * NB;
                if (i < nb && c < nb) {
                    if (c <= i) L[(size_t)(kb + i) * m + kb + c] = stage[c * RSA + i];
                    const double xv = Dinv[i][c];
                    X[(size_t)(kb + i) * m + kb + c] = xv;
                    if (c <= i) Rinv[(size_t)(kb + c) * m + kb + i] = xv;
                } else {
                    Dinv[i][c] = 0.0;
                }
            }
            __syncthreads();   // stage is reused below; Dinv padding visible
        }
        // (2) X_k = Dinv W_k on the columns left of the block; the block itself
        // is Dinv.  Stage X_k (zero rows beyond nb) for the W update.
        {
            // one wave per 16-column tile of W_k, all NB rows: the tile is
            // read completely before it is overwritten in place
            const int nbj = kb / 16;
            for (int bj = wave; bj < nbj; bj += nwaves) {
                const int jc = bj * 16 + (lane & 15);
                d4 acc[NB / 16];
#pragma unroll
                for (int bi = 0; bi < NB / 16; ++bi) acc[bi] = d4{0.0, 0.0, 0.0, 0.0};
                double bv[NB / 4];   // all loads in flight before the products
#pragma unroll
                for (int u = 0; u < NB / 4; ++u) {
                    const int t = 4 * u + (lane >> 4);
                    bv[u] = (t < nb) ? X[(size_t)(kb + t) * m + jc] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < NB / 4; ++u)
#pragma unroll
                    for (int bi = 0; bi < NB / 16; ++bi)
                        acc[bi] = mfma64(Dinv[bi * 16 + (lane & 15)][4 * u + (lane >> 4)], bv[u], acc[bi]);
#pragma unroll
                for (int bi = 0; bi < NB / 16; ++bi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = bi * 16 + mfma64_row(lane, r);
                        XS[i * XSS + jc] = (i < nb) ? acc[bi][r] : 0.0;
                        if (i < nb) {
                            X[(size_t)(kb + i) * m + jc] = acc[bi][r];
                            Rinv[(size_t)jc * m + kb + i] = acc[bi][r];
                        }
                    }
            }
            for (int e = tid; e < NB * NB; e += kDenseThreads) {
                const int i = e / NB, c = e - (e / NB) * NB;
                if (kb + c < XSS - 1) XS[i * XSS + kb + c] = Dinv[i][c];
            }
        }
        // (3) stage S_ik (R x nb), then the panel L_ik = S_ik Dinv^T
        for (int e0 = tid; e0 < R * NB; e0 += 8 * kDenseThreads) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kDenseThreads, r = e / NB, c = e % NB;
                v[u] = (e < R * NB && c < nb) ? src[(size_t)(kb + nb + r) * m + kb + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kDenseThreads;
                if (e < R * NB) stage[(e / NB) * PS + e % NB] = v[u];
            }
        }
        __syncthreads();
        const int nbr = (R + 15) / 16;
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
        // (4) trailing update of the lower triangle (disjoint from the panel
        // columns) and of the W rows below the panel
        const int npairs = nbr * (nbr + 1) / 2;
        const int ncw = (kw + 15) / 16;
        const int nwork = npairs + nbr * ncw;
        for (int p = wave; p < nwork; p += nwaves) {
            const bool sym = p < npairs;
            int bi, bj;
            if (sym) {
                lower_pair(p, bi, bj);
            } else {
                const int q = p - npairs;
                bi = q / ncw;
                bj = q - bi * ncw;
            }
            // old values first, so their latency overlaps the products
            double old[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                double v = 0.0;
                if (sym) {
                    if (i < R && j <= i) v = src[(size_t)(kb + nb + i) * m + kb + nb + j];
                } else {
                    // columns of this panel were never updated: W = I there (0 off the diagonal)
                    if (i < R && j < kb) v = X[(size_t)(kb + nb + i) * m + j];
                }
                old[r] = v;
            }
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = bi * 16 + (lane & 15), rb = bj * 16 + (lane & 15);
            for (int t0 = 0; t0 < nb; t0 += 4) {
                const int k = t0 + (lane >> 4);
                const double a = (ra < R) ? stage[ra * PS + k] : 0.0;
                double b;
                if (sym) b = (rb < R) ? stage[rb * PS + k] : 0.0;
                else b = (rb < kw) ? XS[k * XSS + rb] : 0.0;
                acc = mfma64(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + mfma64_row(lane, r), j = bj * 16 + (lane & 15);
                if (sym) {
                    if (i < R && j <= i) L[(size_t)(kb + nb + i) * m + kb + nb + j] = old[r] - acc[r];
                } else {
                    if (i < R && j < kw) X[(size_t)(kb + nb + i) * m + j] = old[r] - acc[r];
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
    return (size_t)2 * m * m * sizeof(double);
}

void chol_inverse(hipStream_t s, int m, const double *S, double *Rinv,
                  double *work, int32_t *info) {
    TM_REQUIRE(m >= 1 && m <= 1024, TM_ENOTSUP, "Cholesky supports m <= 1024");
    // the staged panel (R x (NB+1)) and X_k (NB x (kb+nb) rounded to 16, +1)
    // must fit the LDS staging area together, for every panel
    {
        const int NB = m <= 512 ? 32 : 16;
        for (int kb = 0; kb < m; kb += NB) {
            const int nb = std::min(NB, m - kb), R = m - kb - nb;
            const int XSS = ((kb + nb + 15) & ~15) + 1;
            TM_REQUIRE((size_t)R * (NB + 1) + (size_t)NB * XSS <= (size_t)kStage, TM_ENOTSUP,
                       "Cholesky staging exceeds LDS");
        }
    }
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
