// Sparse product X = H C (Fig. 2, step (1)) for row-major N x ld blocks.
//
// HBM-bound: every row of C is gathered by its neighbours' rows, so the
// kernels keep each XCD on one contiguous slab of rows (neighbour rows then
// hit that XCD's L2) and move 16-byte vectors per lane along the m columns.
#include "tm_common.h"

namespace tmin {
namespace {

template <typename T> struct Vec;
template <> struct Vec<double> { using type = double2; static constexpr int W = 2; };
template <> struct Vec<float> { using type = float4; static constexpr int W = 4; };

__device__ inline double2 fma_v(double a, double2 c, double2 acc) {
    acc.x = fma(a, c.x, acc.x);
    acc.y = fma(a, c.y, acc.y);
    return acc;
}
__device__ inline float4 fma_v(float a, float4 c, float4 acc) {
    acc.x = fmaf(a, c.x, acc.x);
    acc.y = fmaf(a, c.y, acc.y);
    acc.z = fmaf(a, c.z, acc.z);
    acc.w = fmaf(a, c.w, acc.w);
    return acc;
}
template <typename V> __device__ inline V zero_v();
template <> __device__ inline double2 zero_v<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ inline float4 zero_v<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// Launch geometry shared by both kernels: a workgroup of 256 lanes holds
// `rpb` rows at once with `tpr` lanes per row (each lane loops over the
// row's vectors with stride tpr).  Workgroup b runs on XCD b % 8; it is given
// the contiguous row range of logical slab (b % 8) * (grid / 8) + b / 8.
struct Geometry {
    int tpr, rpb;
    int64_t rows_per_block;
    int grid;
};

Geometry geometry(int64_t n, int ldv) {
    Geometry g;
    g.tpr = ldv < 256 ? ldv : 256;
    g.rpb = 256 / g.tpr;
    int64_t blocks = (n + g.rpb * 4 - 1) / (g.rpb * 4);  // ~4 row passes per block
    if (blocks > 8192) blocks = 8192;
    blocks = (blocks + 7) / 8 * 8;
    g.rows_per_block = (n + blocks - 1) / blocks;
    g.grid = (int)((n + g.rows_per_block - 1) / g.rows_per_block);
    g.grid = (g.grid + 7) / 8 * 8;
    return g;
}

__device__ inline int64_t logical_block(int grid) {
    const int b = blockIdx.x;
    return (int64_t)(b & 7) * (grid >> 3) + (b >> 3);
}

template <typename T>
__global__ __launch_bounds__(256) void spmm_csr_kernel(
    int64_t n, int ldv, int tpr, int rpb, int64_t rows_per_block,
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, const typename Vec<T>::type *__restrict__ C,
    typename Vec<T>::type *__restrict__ X) {
    using V = typename Vec<T>::type;
    const int t = threadIdx.x;
    const int rr = t / tpr;
    const int lane = t - rr * tpr;
    if (rr >= rpb) return;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    for (int64_t r = r_begin + rr; r < r_end; r += rpb) {
        const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
        for (int cv = lane; cv < ldv; cv += tpr) {
            V acc = zero_v<V>();
            for (int64_t k = k0; k < k1; ++k)
                acc = fma_v(val[k], C[(int64_t)col[k] * ldv + cv], acc);
            X[r * ldv + cv] = acc;
        }
    }
}

// Neighbour index along one axis with periodic wrap or Dirichlet cut-off.
__device__ inline bool neighbour(int coord, int off, int extent, int periodic,
                                 int &out) {
    int c = coord + off;
    if (periodic) {
        c %= extent;
        if (c < 0) c += extent;
    } else if (c < 0 || c >= extent) {
        return false;
    }
    out = c;
    return true;
}

template <typename T, int ORDER, int NDIM>
__global__ __launch_bounds__(256) void spmm_stencil_kernel(
    int64_t n, int ldv, int tpr, int rpb, int64_t rows_per_block,
    StencilDev H, const T *__restrict__ V,
    const typename Vec<T>::type *__restrict__ C,
    typename Vec<T>::type *__restrict__ X) {
    using Vv = typename Vec<T>::type;
    const int t = threadIdx.x;
    const int rr = t / tpr;
    const int lane = t - rr * tpr;
    if (rr >= rpb) return;
    const T c0 = (T)H.c0, c1 = (T)H.c1, c2 = (T)H.c2;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    const int ext[3] = {H.nx, H.ny, H.nz};
    const int64_t stride[3] = {1, (int64_t)H.nx, (int64_t)H.nx * H.ny};
    for (int64_t r = r_begin + rr; r < r_end; r += rpb) {
        int crd[3];
        crd[0] = (int)(r % H.nx);
        crd[1] = (int)((r / H.nx) % H.ny);
        crd[2] = NDIM == 3 ? (int)(r / ((int64_t)H.nx * H.ny)) : 0;
        const T diag = c0 + (V ? V[r] : (T)0);
        for (int cv = lane; cv < ldv; cv += tpr) {
            Vv acc = fma_v(diag, C[r * ldv + cv], zero_v<Vv>());
#pragma unroll
            for (int ax = 0; ax < NDIM; ++ax) {
#pragma unroll
                for (int o = -ORDER / 2; o <= ORDER / 2; ++o) {
                    if (o == 0) continue;
                    int c;
                    if (!neighbour(crd[ax], o, ext[ax], H.periodic, c)) continue;
                    const int64_t nb = r + (int64_t)(c - crd[ax]) * stride[ax];
                    const T coef = (o == 1 || o == -1) ? c1 : c2;
                    acc = fma_v(coef, C[nb * ldv + cv], acc);
                }
            }
            X[r * ldv + cv] = acc;
        }
    }
}

}  // namespace

template <typename T>
void spmm_csr(hipStream_t s, const CsrDev &H, int ld, const T *C, T *X) {
    const int ldv = ld / Vec<T>::W;
    Geometry g = geometry(H.n, ldv);
    const T *val;
    if constexpr (sizeof(T) == 8) val = H.val64; else val = H.val32;
    hipLaunchKernelGGL(spmm_csr_kernel<T>, dim3(g.grid), dim3(256), 0, s, H.n,
                       ldv, g.tpr, g.rpb, g.rows_per_block, H.rowptr, H.col, val,
                       reinterpret_cast<const typename Vec<T>::type *>(C),
                       reinterpret_cast<typename Vec<T>::type *>(X));
    TM_HIP(hipGetLastError());
}

template <typename T>
void spmm_stencil(hipStream_t s, const StencilDev &H, int64_t n, int ld,
                  const T *C, T *X) {
    const int ldv = ld / Vec<T>::W;
    Geometry g = geometry(n, ldv);
    const T *V;
    if constexpr (sizeof(T) == 8) V = H.V64; else V = H.V32;
    auto Cv = reinterpret_cast<const typename Vec<T>::type *>(C);
    auto Xv = reinterpret_cast<typename Vec<T>::type *>(X);
#define TM_STENCIL_LAUNCH(ORD, ND)                                                 \
    hipLaunchKernelGGL((spmm_stencil_kernel<T, ORD, ND>), dim3(g.grid), dim3(256), \
                       0, s, n, ldv, g.tpr, g.rpb, g.rows_per_block, H, V, Cv, Xv)
    if (H.ndim == 3 && H.order == 2) TM_STENCIL_LAUNCH(2, 3);
    else if (H.ndim == 3 && H.order == 4) TM_STENCIL_LAUNCH(4, 3);
    else if (H.ndim == 2 && H.order == 2) TM_STENCIL_LAUNCH(2, 2);
    else if (H.ndim == 2 && H.order == 4) TM_STENCIL_LAUNCH(4, 2);
    else throw Error{TM_EINVAL, "unsupported stencil"};
#undef TM_STENCIL_LAUNCH
    TM_HIP(hipGetLastError());
}

template void spmm_csr<double>(hipStream_t, const CsrDev &, int, const double *, double *);
template void spmm_csr<float>(hipStream_t, const CsrDev &, int, const float *, float *);
template void spmm_stencil<double>(hipStream_t, const StencilDev &, int64_t, int, const double *, double *);
template void spmm_stencil<float>(hipStream_t, const StencilDev &, int64_t, int, const float *, float *);

}  // namespace tmin
