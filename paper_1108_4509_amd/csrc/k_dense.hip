// Dense m x m FP64 kernels of the iteration: the Cholesky factorization and
// triangular inverse of Fig. 4 (steps (2) and (3)), and the symmetric
// eigensolve that diagonalizes the m x m H (Eq. 9) for the Rayleigh-Ritz step
// and the occasional subspace rotation.
//
// These are O(m^3) with m <= ~1024, so they are latency-bound; each runs as one
// workgroup of 1024 lanes with the matrix in a device workspace (resident in
// L2) and 16-wide blocks cached in LDS.
#include "tm_common.h"

#include <cmath>

namespace tmin {
namespace {

constexpr int kDenseThreads = 1024;
constexpr int NB = 16;

// Factor the nb x nb diagonal block D (lower, in LDS) in place and write its
// inverse (lower) to Dinv.  Runs on one wave; returns false on a bad pivot.
// A pivot below kPivotTol times the original diagonal entry counts as a
// breakdown: C^T C is then numerically singular (dependent columns of C).
constexpr double kPivotTol = 1e-14;

__device__ bool small_chol_inv(int nb, double (*D)[NB + 1], double (*Dinv)[NB + 1],
                               const double *Sdiag, int lane) {
    bool ok = true;
    for (int k = 0; k < nb; ++k) {
        const double d = D[k][k];
        if (!(d > kPivotTol * fabs(Sdiag[k]))) ok = false;
        const double r = sqrt(fmax(d, 0.0));
        __builtin_amdgcn_wave_barrier();
        if (lane > k && lane < nb) D[lane][k] /= r;
        if (lane == 0) D[k][k] = r;
        __builtin_amdgcn_wave_barrier();
        // trailing update inside the block: lanes own rows
        if (lane > k && lane < nb)
            for (int j = k + 1; j <= lane; ++j) D[lane][j] -= D[lane][k] * D[j][k];
        __builtin_amdgcn_wave_barrier();
    }
    if (!ok) return false;
    // inverse of the lower-triangular D, row by row: lane owns column c
    for (int i = 0; i < nb; ++i) {
        if (lane < nb) {
            const int c = lane;
            double v;
            if (c > i) {
                v = 0.0;
            } else if (c == i) {
                v = 1.0 / D[i][i];
            } else {
                double s = 0.0;
                for (int k = c; k < i; ++k) s += D[i][k] * Dinv[k][c];
                v = -s / D[i][i];
            }
            Dinv[i][c] = v;
        }
        __builtin_amdgcn_wave_barrier();
    }
    return true;
}

// S = L L^T (L lower, S = R^T R with R = L^T); Rinv = L^{-T}.
// work: m*m doubles (L), work + m*m: m*m doubles (L^{-1}), + m*NB (panel).
__global__ __launch_bounds__(kDenseThreads) void chol_inv_kernel(
    int m, const double *__restrict__ S, double *__restrict__ Rinv,
    double *__restrict__ work, int32_t *__restrict__ info) {
    __shared__ double D[NB][NB + 1];
    __shared__ double Dinv[NB][NB + 1];
    __shared__ double Sd[NB];
    __shared__ int bad;
    double *L = work;
    double *X = work + (size_t)m * m;         // L^{-1}
    double *panel = X + (size_t)m * m;        // m x NB
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nthr = blockDim.x;
    if (tid == 0) bad = 0;
    for (int64_t e = tid; e < (int64_t)m * m; e += nthr) {
        L[e] = S[e];
        X[e] = 0.0;
    }
    __syncthreads();

    // ---- blocked right-looking Cholesky
    for (int kb = 0; kb < m; kb += NB) {
        const int nb = (m - kb < NB) ? (m - kb) : NB;
        if (tid < 64) {
            for (int e = lane; e < NB * NB; e += 64) {
                const int i = e / NB, j = e % NB;
                D[i][j] = (i < nb && j <= i) ? L[(size_t)(kb + i) * m + kb + j] : 0.0;
                Dinv[i][j] = 0.0;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < nb) Sd[lane] = S[(size_t)(kb + lane) * m + kb + lane];
            __builtin_amdgcn_wave_barrier();
            const bool ok = small_chol_inv(nb, D, Dinv, Sd, lane);
            if (!ok && lane == 0) bad = kb + 1;
            for (int e = lane; e < nb * nb; e += 64) {
                const int i = e / nb, j = e % nb;
                if (j <= i) {
                    L[(size_t)(kb + i) * m + kb + j] = D[i][j];
                    X[(size_t)(kb + i) * m + kb + j] = Dinv[i][j];
                }
            }
        }
        __syncthreads();
        if (bad) break;
        // panel: L_ik = S_ik L_kk^{-T}, rows i >= kb + nb
        const int rows = m - kb - nb;
        for (int e = tid; e < rows * nb; e += nthr) {
            const int i = kb + nb + e / nb, c = e % nb;
            double s = 0.0;
            for (int t = 0; t <= c; ++t) s += L[(size_t)i * m + kb + t] * Dinv[c][t];
            panel[(size_t)i * NB + c] = s;
        }
        __syncthreads();
        for (int e = tid; e < rows * nb; e += nthr) {
            const int i = kb + nb + e / nb, c = e % nb;
            L[(size_t)i * m + kb + c] = panel[(size_t)i * NB + c];
        }
        __syncthreads();
        // trailing update of the lower triangle: S_ij -= L_ik L_jk^T
        for (int64_t e = tid; e < (int64_t)rows * rows; e += nthr) {
            const int i = kb + nb + (int)(e / rows);
            const int j = kb + nb + (int)(e % rows);
            if (j > i) continue;
            double s = 0.0;
            for (int t = 0; t < nb; ++t)
                s += L[(size_t)i * m + kb + t] * L[(size_t)j * m + kb + t];
            L[(size_t)i * m + j] -= s;
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) info[0] = bad;
        return;
    }

    // ---- blocked inverse X = L^{-1}: diagonal blocks are already in X.
    // Block row ib: X_ib,: = -Dinv_ib * sum_{k < ib} L_ib,k X_k,:
    for (int ib = NB; ib < m; ib += NB) {
        const int nb = (m - ib < NB) ? (m - ib) : NB;
        // T = L[ib:ib+nb, 0:ib] X[0:ib, 0:ib] into panel (nb x ib, row-major)
        for (int e = tid; e < nb * ib; e += nthr) {
            const int r = e / ib, c = e % ib;
            double s = 0.0;
            for (int k = c; k < ib; ++k) s += L[(size_t)(ib + r) * m + k] * X[(size_t)k * m + c];
            panel[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < nb * ib; e += nthr) {
            const int r = e / ib, c = e % ib;
            double s = 0.0;
            for (int t = 0; t <= r; ++t)
                s += X[(size_t)(ib + r) * m + ib + t] * panel[(size_t)t * ib + c];
            X[(size_t)(ib + r) * m + c] = -s;
        }
        __syncthreads();
    }
    // Rinv = X^T (upper triangular)
    for (int64_t e = tid; e < (int64_t)m * m; e += nthr) {
        const int i = (int)(e / m), j = (int)(e % m);
        Rinv[e] = (j >= i) ? X[(size_t)j * m + i] : 0.0;
    }
}

// -------------------------------------------------------------- Jacobi
// Parallel cyclic Jacobi with round-robin ("circle") pair ordering: in each
// step the M/2 disjoint pairs (p, q) are rotated at once.  A <- J^T A J is
// applied as independent 2 x 2 block updates; V <- V J.  M = m rounded up to
// even; index m (when m is odd) is a dummy that never rotates.
__device__ inline int rr_index(int pos, int step, int M) {
    if (pos == 0) return 0;
    return 1 + (pos - 1 + step) % (M - 1);
}

__global__ __launch_bounds__(kDenseThreads) void jacobi_kernel(
    int m, const double *__restrict__ Ain, double *__restrict__ U,
    double *__restrict__ w, double *__restrict__ work, int32_t *__restrict__ info,
    int max_sweeps) {
    __shared__ double cs_c[512], cs_s[512];
    __shared__ int pp[512], qq[512];
    __shared__ double red[kDenseThreads];
    __shared__ int stop;
    double *A = work;
    double *V = work + (size_t)m * m;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int M = (m + 1) & ~1;
    const int half = M / 2;
    double fro2 = 0.0;
    for (int64_t e = tid; e < (int64_t)m * m; e += nthr) {
        const double a = Ain[e];
        A[e] = a;
        fro2 += a * a;
        const int i = (int)(e / m), j = (int)(e % m);
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    red[tid] = fro2;
    __syncthreads();
    for (int k = kDenseThreads / 2; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    const double anorm = sqrt(red[0]);
    __syncthreads();
    if (tid == 0) stop = 0;
    double prev_off = 1e300;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // off-diagonal norm
        double o = 0.0;
        for (int64_t e = tid; e < (int64_t)m * m; e += nthr) {
            const int i = (int)(e / m), j = (int)(e % m);
            if (i != j) o += A[e] * A[e];
        }
        red[tid] = o;
        __syncthreads();
        for (int k = kDenseThreads / 2; k > 0; k >>= 1) {
            if (tid < k) red[tid] += red[tid + k];
            __syncthreads();
        }
        if (tid == 0) {
            const double off = sqrt(red[0]);
            if (off <= 1e-15 * anorm || m < 2) stop = 1;
            else if (sweep >= 3 && off > 0.5 * prev_off && off <= 1e-12 * anorm) stop = 1;
            prev_off = off;
        }
        __syncthreads();
        if (stop) break;
        for (int step = 0; step < M - 1; ++step) {
            if (tid < half) {
                int p = rr_index(tid, step, M), q = rr_index(M - 1 - tid, step, M);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[(size_t)p * m + q];
                    if (apq != 0.0) {
                        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                                      : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                pp[tid] = p;
                qq[tid] = q;
                cs_c[tid] = c;
                cs_s[tid] = s;
            }
            __syncthreads();
            // A <- J^T A J on 2 x 2 blocks (pair a rows, pair b columns)
            for (int64_t e = tid; e < (int64_t)half * half; e += nthr) {
                const int a = (int)(e / half), b = (int)(e % half);
                const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
                const double ca = cs_c[a], sa = cs_s[a], cb = cs_c[b], sb = cs_s[b];
                const bool qa_ok = qa < m, qb_ok = qb < m;
                const double x00 = A[(size_t)pa * m + pb];
                const double x01 = qb_ok ? A[(size_t)pa * m + qb] : 0.0;
                const double x10 = qa_ok ? A[(size_t)qa * m + pb] : 0.0;
                const double x11 = (qa_ok && qb_ok) ? A[(size_t)qa * m + qb] : 0.0;
                // columns: B = X J_b
                const double b00 = cb * x00 - sb * x01, b01 = sb * x00 + cb * x01;
                const double b10 = cb * x10 - sb * x11, b11 = sb * x10 + cb * x11;
                // rows: J_a^T B
                double y00 = ca * b00 - sa * b10, y01 = ca * b01 - sa * b11;
                double y10 = sa * b00 + ca * b10, y11 = sa * b01 + ca * b11;
                if (a == b) { y01 = 0.0; y10 = 0.0; }
                A[(size_t)pa * m + pb] = y00;
                if (qb_ok) A[(size_t)pa * m + qb] = y01;
                if (qa_ok) A[(size_t)qa * m + pb] = y10;
                if (qa_ok && qb_ok) A[(size_t)qa * m + qb] = y11;
            }
            // V <- V J
            for (int64_t e = tid; e < (int64_t)m * half; e += nthr) {
                const int k = (int)(e / half), b = (int)(e % half);
                const int pb = pp[b], qb = qq[b];
                if (qb >= m) continue;
                const double cb = cs_c[b], sb = cs_s[b];
                const double vp = V[(size_t)k * m + pb], vq = V[(size_t)k * m + qb];
                V[(size_t)k * m + pb] = cb * vp - sb * vq;
                V[(size_t)k * m + qb] = sb * vp + cb * vq;
            }
            __syncthreads();
        }
    }
    // sort ascending by rank (ties broken by index) and scatter
    for (int i = tid; i < m; i += nthr) {
        const double wi = A[(size_t)i * m + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double wj = A[(size_t)j * m + j];
            rank += (wj < wi) || (wj == wi && j < i);
        }
        w[rank] = wi;
        for (int k = 0; k < m; ++k) U[(size_t)k * m + rank] = V[(size_t)k * m + i];
    }
    if (tid == 0) info[0] = sweep;
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
    return ((size_t)2 * m * m + (size_t)m * NB) * sizeof(double);
}

void chol_inverse(hipStream_t s, int m, const double *S, double *Rinv,
                  double *work, int32_t *info) {
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kDenseThreads), 0, s, m, S,
                       Rinv, work, info);
    TM_HIP(hipGetLastError());
}

size_t jacobi_workspace(int m) { return (size_t)2 * m * m * sizeof(double); }

void jacobi_eig(hipStream_t s, int m, const double *A, double *U, double *w,
                double *work, int32_t *info) {
    TM_REQUIRE(m <= 1024, TM_ENOTSUP, "eigensolver supports m <= 1024");
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kDenseThreads), 0, s, m, A, U,
                       w, work, info, 40);
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
