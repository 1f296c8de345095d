// Sparse product X = H C (Fig. 2, step (1)) for row-major N x ld blocks, with
// optional column dot products of the input and output fused into the
// epilogue: h_j = c_j . x_j (Fig. 2, steps (2)-(3)) after X = HC, and
// p_j . p_j, p_j . y_j (the line step) after Y = HP.  The fusion saves a full
// pass over both blocks.
//
// HBM-bound: every row of C is gathered by its neighbours' rows, so the
// kernels keep each XCD on one contiguous slab of rows (neighbour rows then
// hit that XCD's L2) and move 16-byte vectors per lane along the m columns.
#include "tm_common.h"

namespace tmin {
namespace {

typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec;
template <> struct Vec<double> { using type = vd2; static constexpr int W = 2; };
template <> struct Vec<float> { using type = vf4; static constexpr int W = 4; };

constexpr int kMaxCv = 2;     // column vectors per lane (ld <= 1024)
constexpr int kGridCap = 1024;

// Launch geometry: a workgroup of 256 lanes holds `rpb` rows at once with
// `tpr` lanes per row (each lane loops over the row's vectors with stride
// tpr).  Workgroup b runs on XCD b % 8; it is given the contiguous row range
// of logical slab (b % 8) * (grid / 8) + b / 8.
struct Geometry {
    int tpr, rpb;
    int64_t rows_per_block;
    int grid;
};

Geometry geometry(int64_t n, int ldv) {
    Geometry g;
    g.tpr = ldv < 256 ? ldv : 256;
    g.rpb = 256 / g.tpr;
    int64_t blocks = (n + g.rpb - 1) / g.rpb;
    if (blocks > kGridCap) blocks = kGridCap;
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

template <typename V, typename T>
__device__ inline V fma_v(T a, V c, V acc) {
#pragma unroll
    for (int w = 0; w < Vec<T>::W; ++w) acc[w] = fma(a, c[w], acc[w]);
    return acc;
}

// Per-lane FP64 accumulators of the fused dots: [cv slot][dot][vector element]
template <typename T>
struct DotAcc {
    double v[kMaxCv][2][Vec<T>::W];
    __device__ void zero() {
#pragma unroll
        for (int q = 0; q < kMaxCv; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int w = 0; w < Vec<T>::W; ++w) v[q][p][w] = 0.0;
    }
    // dot 0: a . b, dot 1: a . a
    __device__ void add(int q, const typename Vec<T>::type &a, const typename Vec<T>::type &b,
                        int ndot) {
#pragma unroll
        for (int w = 0; w < Vec<T>::W; ++w) {
            const double x = (double)a[w], y = (double)b[w];
            v[q][0][w] += x * y;
            if (ndot > 1) v[q][1][w] += x * x;
        }
    }
};

// Fold the per-lane sums over the rows of the workgroup (fixed order) and
// write partials[(p * grid + lb) * ld + col].
template <typename T>
__device__ void flush_dots(const DotAcc<T> &acc, int ndot, int rr, int lane, int tpr, int rpb,
                           int ldv, int64_t lb, double *__restrict__ partials, double *red) {
    constexpr int W = Vec<T>::W;
    const int ld = ldv * W;
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        if (p >= ndot) break;
        if (rr < rpb) {
#pragma unroll
            for (int q = 0; q < kMaxCv; ++q) {
                const int cv = lane + q * tpr;
                if (cv < ldv)
#pragma unroll
                    for (int w = 0; w < W; ++w) red[rr * ld + cv * W + w] = acc.v[q][p][w];
            }
        }
        __syncthreads();
        for (int col = t; col < ld; col += 256) {
            double s = 0.0;
            for (int g = 0; g < rpb; ++g) s += red[g * ld + col];
            partials[((int64_t)p * gridDim.x + lb) * ld + col] = s;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void spmm_csr_kernel(
    int64_t n, int ldv, int tpr, int rpb, int64_t rows_per_block,
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, const typename Vec<T>::type *__restrict__ C,
    typename Vec<T>::type *__restrict__ X, int ndot, double *__restrict__ partials) {
    using V = typename Vec<T>::type;
    __shared__ double red[1024];
    const int t = threadIdx.x;
    const int rr = t / tpr;
    const int lane = t - rr * tpr;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    DotAcc<T> dacc;
    dacc.zero();
    if (rr < rpb) {
        for (int64_t r = r_begin + rr; r < r_end; r += rpb) {
            const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
#pragma unroll
            for (int q = 0; q < kMaxCv; ++q) {
                const int cv = lane + q * tpr;
                if (cv >= ldv) break;
                V acc = V(0);
                for (int64_t k = k0; k < k1; ++k)
                    acc = fma_v<V, T>(val[k], C[(int64_t)col[k] * ldv + cv], acc);
                X[r * ldv + cv] = acc;
                if (ndot > 0) dacc.add(q, C[r * ldv + cv], acc, ndot);
            }
        }
    }
    if (ndot > 0) flush_dots<T>(dacc, ndot, rr, lane, tpr, rpb, ldv, lb, partials, red);
}

// Neighbour index along one axis with periodic wrap or Dirichlet cut-off.
__device__ inline bool neighbour(int coord, int off, int extent, int periodic, int &out) {
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
    int64_t n, int ldv, int tpr, int rpb, int64_t rows_per_block, StencilDev H,
    const T *__restrict__ Vpot, const typename Vec<T>::type *__restrict__ C,
    typename Vec<T>::type *__restrict__ X, int ndot, double *__restrict__ partials) {
    using V = typename Vec<T>::type;
    __shared__ double red[1024];
    const int t = threadIdx.x;
    const int rr = t / tpr;
    const int lane = t - rr * tpr;
    const T c0 = (T)H.c0, c1 = (T)H.c1, c2 = (T)H.c2;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    const int ext[3] = {H.nx, H.ny, H.nz};
    const int64_t stride[3] = {1, (int64_t)H.nx, (int64_t)H.nx * H.ny};
    DotAcc<T> dacc;
    dacc.zero();
    if (rr < rpb) {
        for (int64_t r = r_begin + rr; r < r_end; r += rpb) {
            int crd[3];
            crd[0] = (int)(r % H.nx);
            crd[1] = (int)((r / H.nx) % H.ny);
            crd[2] = NDIM == 3 ? (int)(r / ((int64_t)H.nx * H.ny)) : 0;
            const T diag = c0 + (Vpot ? Vpot[r] : (T)0);
            int64_t nb[3][4];
            bool has[3][4];
#pragma unroll
            for (int ax = 0; ax < NDIM; ++ax) {
                int s = 0;
#pragma unroll
                for (int o = -ORDER / 2; o <= ORDER / 2; ++o) {
                    if (o == 0) continue;
                    int c;
                    has[ax][s] = neighbour(crd[ax], o, ext[ax], H.periodic, c);
                    nb[ax][s] = r + (int64_t)(c - crd[ax]) * stride[ax];
                    ++s;
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxCv; ++q) {
                const int cv = lane + q * tpr;
                if (cv >= ldv) break;
                const V center = C[r * ldv + cv];
                V acc = fma_v<V, T>(diag, center, V(0));
#pragma unroll
                for (int ax = 0; ax < NDIM; ++ax) {
                    int s = 0;
#pragma unroll
                    for (int o = -ORDER / 2; o <= ORDER / 2; ++o) {
                        if (o == 0) continue;
                        const T coef = (o == 1 || o == -1) ? c1 : c2;
                        if (has[ax][s]) acc = fma_v<V, T>(coef, C[nb[ax][s] * ldv + cv], acc);
                        ++s;
                    }
                }
                X[r * ldv + cv] = acc;
                if (ndot > 0) dacc.add(q, center, acc, ndot);
            }
        }
    }
    if (ndot > 0) flush_dots<T>(dacc, ndot, rr, lane, tpr, rpb, ldv, lb, partials, red);
}

// Wide blocks (at least 64 vectors per row): one wave per row at a time, so
// the row index, its CSR range, column indices and values are wave-uniform
// and come through the scalar cache; each lane owns NCV vectors of the row.
// The four waves of a workgroup walk interleaved rows of its slab.
template <typename T, int NCV>
__device__ void flush_wave_dots(const double (&ds)[NCV][2][Vec<T>::W], int ndot, int wave, int lane,
                                int64_t lb, double *__restrict__ partials, double *red) {
    constexpr int W = Vec<T>::W;
    constexpr int ld = NCV * 64 * W;
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        if (p >= ndot) break;
#pragma unroll
        for (int q = 0; q < NCV; ++q)
#pragma unroll
            for (int w = 0; w < W; ++w) red[wave * ld + (lane + 64 * q) * W + w] = ds[q][p][w];
        __syncthreads();
        for (int col = t; col < ld; col += 256) {
            const double sum = ((red[col] + red[ld + col]) + red[2 * ld + col]) + red[3 * ld + col];
            partials[((int64_t)p * gridDim.x + lb) * ld + col] = sum;
        }
        __syncthreads();
    }
}

template <typename T, int NCV>
__global__ __launch_bounds__(256) void spmm_csr_wave_kernel(
    int64_t n, int64_t rows_per_block, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const T *__restrict__ val,
    const typename Vec<T>::type *__restrict__ C, typename Vec<T>::type *__restrict__ X,
    int ndot, double *__restrict__ partials) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::W;
    constexpr int ldv = NCV * 64;
    __shared__ double red[4 * ldv * W];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    double ds[NCV][2][W];
#pragma unroll
    for (int q = 0; q < NCV; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) ds[q][p][w] = 0.0;
    for (int64_t r = r_begin + wave; r < r_end; r += 4) {
        const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
        V acc[NCV];
#pragma unroll
        for (int q = 0; q < NCV; ++q) acc[q] = V(0);
        // U nonzeros at a time keep U * NCV vector loads in flight
        constexpr int U = NCV >= 4 ? 1 : 4;
        int64_t k = k0;
        for (; k + U <= k1; k += U) {
            V v[U][NCV];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const V *src = C + (int64_t)col[k + u] * ldv + lane;
#pragma unroll
                for (int q = 0; q < NCV; ++q) v[u][q] = src[64 * q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NCV; ++q) acc[q] = fma_v<V, T>(val[k + u], v[u][q], acc[q]);
        }
        for (; k < k1; ++k) {
            const V *src = C + (int64_t)col[k] * ldv + lane;
#pragma unroll
            for (int q = 0; q < NCV; ++q) acc[q] = fma_v<V, T>(val[k], src[64 * q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < NCV; ++q) X[r * ldv + lane + 64 * q] = acc[q];
        if (ndot > 0) {
#pragma unroll
            for (int q = 0; q < NCV; ++q) {
                const V c = C[r * ldv + lane + 64 * q];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ds[q][0][w] += (double)c[w] * (double)acc[q][w];
                    if (ndot > 1) ds[q][1][w] += (double)c[w] * (double)c[w];
                }
            }
        }
    }
    if (ndot > 0) flush_wave_dots<T, NCV>(ds, ndot, wave, lane, lb, partials, red);
}

template <typename T, int NCV, int ORDER, int NDIM>
__global__ __launch_bounds__(256) void spmm_stencil_wave_kernel(
    int64_t n, int64_t rows_per_block, StencilDev H, const T *__restrict__ Vpot,
    const typename Vec<T>::type *__restrict__ C, typename Vec<T>::type *__restrict__ X,
    int ndot, double *__restrict__ partials) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::W;
    constexpr int ldv = NCV * 64;
    __shared__ double red[4 * ldv * W];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T c0 = (T)H.c0, c1 = (T)H.c1, c2 = (T)H.c2;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t r_begin = lb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    const int ext[3] = {H.nx, H.ny, H.nz};
    const int64_t stride[3] = {1, (int64_t)H.nx, (int64_t)H.nx * H.ny};
    double ds[NCV][2][W];
#pragma unroll
    for (int q = 0; q < NCV; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) ds[q][p][w] = 0.0;
    for (int64_t r = r_begin + wave; r < r_end; r += 4) {
        int crd[3];
        crd[0] = (int)(r % H.nx);
        crd[1] = (int)((r / H.nx) % H.ny);
        crd[2] = NDIM == 3 ? (int)(r / ((int64_t)H.nx * H.ny)) : 0;
        const T diag = c0 + (Vpot ? Vpot[r] : (T)0);
        V center[NCV], acc[NCV];
#pragma unroll
        for (int q = 0; q < NCV; ++q) {
            center[q] = C[r * ldv + lane + 64 * q];
            acc[q] = fma_v<V, T>(diag, center[q], V(0));
        }
#pragma unroll
        for (int ax = 0; ax < NDIM; ++ax) {
#pragma unroll
            for (int o = -ORDER / 2; o <= ORDER / 2; ++o) {
                if (o == 0) continue;
                int c;
                if (!neighbour(crd[ax], o, ext[ax], H.periodic, c)) continue;
                const int64_t nb = r + (int64_t)(c - crd[ax]) * stride[ax];
                const T coef = (o == 1 || o == -1) ? c1 : c2;
#pragma unroll
                for (int q = 0; q < NCV; ++q)
                    acc[q] = fma_v<V, T>(coef, C[nb * ldv + lane + 64 * q], acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < NCV; ++q) {
            X[r * ldv + lane + 64 * q] = acc[q];
            if (ndot > 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ds[q][0][w] += (double)center[q][w] * (double)acc[q][w];
                    if (ndot > 1) ds[q][1][w] += (double)center[q][w] * (double)center[q][w];
                }
            }
        }
    }
    if (ndot > 0) flush_wave_dots<T, NCV>(ds, ndot, wave, lane, lb, partials, red);
}

// ---------------------------------------------------------------- slab kernels
// For wide blocks the rows are cut into 512-byte column slabs (64 FP64 or
// 128 FP32 columns, one 8-byte element per lane) and the slabs are handed to
// the XCDs so that each XCD sweeps one contiguous (slab, row range) with all
// of its waves side by side: wave w of the XCD takes rows r0 + w,
// r0 + w + wpx, ...  The rows in flight on an XCD then form a narrow moving
// window, and a neighbour row needed again one grid plane later (the z +- 1
// couplings of a 3-D stencil, 2304 rows apart at 48^3) is 2304 x 512 B =
// 1.2 MB back in the stream: still in the XCD's 4 MB L2.  With whole rows
// (2 KB in FP64) that distance is 4.7 MB and the re-reads go to memory.
// Workgroup b runs on XCD b % 8.  Fused column dots are reduced over the 4
// waves in a fixed order and written per workgroup:
// partials[(p * nprow + part * bpx + b / 8) * ld + col].
template <typename T> struct SlabE;
template <> struct SlabE<double> { using type = double; static constexpr int W = 1; };
template <> struct SlabE<float> { using type = vf2; static constexpr int W = 2; };

template <typename T>
__device__ inline double slab_elem(const typename SlabE<T>::type &v, int w) {
    if constexpr (SlabE<T>::W == 1) return (double)v; else return (double)v[w];
}

struct SlabMap {
    int s;          // slab
    int64_t r0, r1; // row range
    int prow;       // partial-sum row of this workgroup
};

// slab and row range of the j-th pass of this workgroup
__device__ inline SlabMap slab_map(int64_t n, int nslab, int j) {
    const int xcd = blockIdx.x & 7, bpx = gridDim.x >> 3, bx = blockIdx.x >> 3;
    SlabMap mp;
    if (nslab >= 8) {
        mp.s = xcd * (nslab >> 3) + j;
        mp.r0 = 0;
        mp.r1 = n;
        mp.prow = bx;
    } else {
        const int xps = 8 / nslab, part = xcd % xps;
        mp.s = xcd / xps;
        mp.r0 = n * part / xps;
        mp.r1 = n * (part + 1) / xps;
        mp.prow = part * bpx + bx;
    }
    return mp;
}

template <typename T>
__device__ void slab_flush_dots(const double (&d)[2][SlabE<T>::W], int ndot, int nprow, int ld,
                                const SlabMap &mp, double *__restrict__ partials,
                                double (*red)[4][128]) {
    constexpr int W = SlabE<T>::W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int w = 0; w < W; ++w) red[p][wave][lane * W + w] = d[p][w];
    __syncthreads();
    if (wave == 0) {
        for (int p = 0; p < ndot; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int e = lane * W + w;
                const double v = ((red[p][0][e] + red[p][1][e]) + red[p][2][e]) + red[p][3][e];
                partials[((int64_t)p * nprow + mp.prow) * ld + mp.s * 64 * W + e] = v;
            }
    }
    __syncthreads();
}

// RW consecutive rows per wave and step: the first eight nonzeros of all RW
// rows are gathered before any is consumed, so 8 RW loads are in flight.
template <typename T, int RW>
__global__ __launch_bounds__(256) void spmm_csr_slab_kernel(
    int64_t n, int ldE, int nslab, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const T *__restrict__ val,
    const typename SlabE<T>::type *__restrict__ C, typename SlabE<T>::type *__restrict__ X,
    int ndot, double *__restrict__ partials) {
    using E = typename SlabE<T>::type;
    constexpr int W = SlabE<T>::W;
    __shared__ double red[2][4][128];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpx = (gridDim.x >> 3) * 4;
    const int w = (blockIdx.x >> 3) * 4 + wave;
    const int npass = nslab >= 8 ? nslab >> 3 : 1;
    const int nprow = nslab >= 8 ? (gridDim.x >> 3) : (8 / nslab) * (gridDim.x >> 3);
    for (int j = 0; j < npass; ++j) {
        const SlabMap mp = slab_map(n, nslab, j);
        const E *Cs = C + mp.s * 64 + lane;
        E *Xs = X + mp.s * 64 + lane;
        double d[2][W];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < W; ++q) d[p][q] = 0.0;
        for (int64_t rb = mp.r0 + (int64_t)w * RW; rb < mp.r1; rb += (int64_t)wpx * RW) {
            int64_t k0[RW], k1[RW];
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                const bool in = rb + t < mp.r1;
                k0[t] = in ? rowptr[rb + t] : 0;
                k1[t] = in ? rowptr[rb + t + 1] : 0;
            }
            E v[RW][8];
            T a[RW][8];
#pragma unroll
            for (int t = 0; t < RW; ++t)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in = k0[t] + u < k1[t];
                    a[t][u] = in ? val[k0[t] + u] : T(0);
                    v[t][u] = in ? Cs[(int64_t)col[k0[t] + u] * ldE] : E(0);
                }
#pragma unroll
            for (int t = 0; t < RW; ++t) {
                if (rb + t >= mp.r1) break;
                E acc = E(0);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = a[t][u] * v[t][u] + acc;
                for (int64_t k = k0[t] + 8; k < k1[t]; ++k) acc = val[k] * Cs[(int64_t)col[k] * ldE] + acc;
                const int64_t r = rb + t;
                Xs[r * ldE] = acc;
                if (ndot > 0) {
                    const E c = Cs[r * ldE];
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const double cq = slab_elem<T>(c, q);
                        d[0][q] += cq * slab_elem<T>(acc, q);
                        if (ndot > 1) d[1][q] += cq * cq;
                    }
                }
            }
        }
        if (ndot > 0) slab_flush_dots<T>(d, ndot, nprow, ldE * W, mp, partials, red);
    }
}

template <typename T, int ORDER, int NDIM>
__global__ __launch_bounds__(256) void spmm_stencil_slab_kernel(
    int64_t n, int ldE, int nslab, StencilDev H, const T *__restrict__ Vpot,
    const typename SlabE<T>::type *__restrict__ C, typename SlabE<T>::type *__restrict__ X,
    int ndot, double *__restrict__ partials) {
    using E = typename SlabE<T>::type;
    constexpr int W = SlabE<T>::W;
    __shared__ double red[2][4][128];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpx = (gridDim.x >> 3) * 4;
    const int w = (blockIdx.x >> 3) * 4 + wave;
    const int npass = nslab >= 8 ? nslab >> 3 : 1;
    const int nprow = nslab >= 8 ? (gridDim.x >> 3) : (8 / nslab) * (gridDim.x >> 3);
    const T c0 = (T)H.c0, c1 = (T)H.c1, c2 = (T)H.c2;
    const int ext[3] = {H.nx, H.ny, H.nz};
    const int64_t stride[3] = {1, (int64_t)H.nx, (int64_t)H.nx * H.ny};
    for (int j = 0; j < npass; ++j) {
        const SlabMap mp = slab_map(n, nslab, j);
        const E *Cs = C + mp.s * 64 + lane;
        E *Xs = X + mp.s * 64 + lane;
        double d[2][W];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < W; ++q) d[p][q] = 0.0;
        for (int64_t r = mp.r0 + w; r < mp.r1; r += wpx) {
            int crd[3];
            crd[0] = (int)(r % H.nx);
            crd[1] = (int)((r / H.nx) % H.ny);
            crd[2] = NDIM == 3 ? (int)(r / ((int64_t)H.nx * H.ny)) : 0;
            const T diag = c0 + (Vpot ? Vpot[r] : T(0));
            const E center = Cs[r * ldE];
            E acc = diag * center;
#pragma unroll
            for (int ax = 0; ax < NDIM; ++ax) {
#pragma unroll
                for (int o = -ORDER / 2; o <= ORDER / 2; ++o) {
                    if (o == 0) continue;
                    int c;
                    if (!neighbour(crd[ax], o, ext[ax], H.periodic, c)) continue;
                    const int64_t nb = r + (int64_t)(c - crd[ax]) * stride[ax];
                    const T coef = (o == 1 || o == -1) ? c1 : c2;
                    acc = coef * Cs[nb * ldE] + acc;
                }
            }
            Xs[r * ldE] = acc;
            if (ndot > 0) {
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const double cq = slab_elem<T>(center, q);
                    d[0][q] += cq * slab_elem<T>(acc, q);
                    if (ndot > 1) d[1][q] += cq * cq;
                }
            }
        }
        if (ndot > 0) slab_flush_dots<T>(d, ndot, nprow, ldE * W, mp, partials, red);
    }
}

// Slab launch: returns nslab, or 0 when the block does not cut into a power
// of two of 512-byte slabs.
template <typename T>
int slab_count(int ld) {
    constexpr int cols = 64 * SlabE<T>::W;
    if (ld % cols != 0) return 0;
    const int ns = ld / cols;
    if (ns < 1 || (ns & (ns - 1)) != 0 || ns > 64) return 0;
    return ns;
}

constexpr int kSlabGrid = 1024;   // 128 workgroups (512 waves) per XCD
constexpr int kSlabRows = 4;      // consecutive rows per wave step (CSR)

// partial rows written by a slab launch
inline int slab_partial_rows(int nslab) {
    return nslab >= 8 ? kSlabGrid / 8 : (8 / nslab) * (kSlabGrid / 8);
}

// grid for the wave kernels: ~kGridCap workgroups of 4 waves, multiple of 8
Geometry wave_geometry(int64_t n) {
    Geometry g;
    g.tpr = 64;
    g.rpb = 4;
    int64_t blocks = (n + 3) / 4;
    if (blocks > kGridCap) blocks = kGridCap;
    blocks = (blocks + 7) / 8 * 8;
    g.rows_per_block = (n + blocks - 1) / blocks;
    g.grid = (int)((n + g.rows_per_block - 1) / g.rows_per_block);
    g.grid = (g.grid + 7) / 8 * 8;
    return g;
}

}  // namespace

size_t spmm_partials_workspace(int ld) { return (size_t)2 * (kGridCap + 8) * ld * sizeof(double); }

template <typename T>
int spmm_csr(hipStream_t s, const CsrDev &H, int ld, const T *C, T *X, int ndot,
             double *partials) {
    const int ldv = ld / Vec<T>::W;
    TM_REQUIRE(ldv <= kMaxCv * 256, TM_ENOTSUP, "block too wide for the SpMM kernel");
    Geometry g = geometry(H.n, ldv);
    const T *val;
    if constexpr (sizeof(T) == 8) val = H.val64; else val = H.val32;
    if (const int ns = slab_count<T>(ld); ns > 0 && H.n >= 64 * kSlabGrid) {
        using E = typename SlabE<T>::type;
        hipLaunchKernelGGL((spmm_csr_slab_kernel<T, kSlabRows>), dim3(kSlabGrid), dim3(256), 0, s, H.n,
                           ld / SlabE<T>::W, ns, H.rowptr, H.col, val,
                           reinterpret_cast<const E *>(C), reinterpret_cast<E *>(X), ndot, partials);
        TM_HIP(hipGetLastError());
        return slab_partial_rows(ns);
    }
    auto Cv = reinterpret_cast<const typename Vec<T>::type *>(C);
    auto Xv = reinterpret_cast<typename Vec<T>::type *>(X);
    if (ldv % 64 == 0 && ldv <= 512) {
        Geometry w = wave_geometry(H.n);
#define TM_CSR_WAVE(NCV)                                                                   \
    hipLaunchKernelGGL((spmm_csr_wave_kernel<T, NCV>), dim3(w.grid), dim3(256), 0, s, H.n, \
                       w.rows_per_block, H.rowptr, H.col, val, Cv, Xv, ndot, partials)
        switch (ldv / 64) {
        case 1: TM_CSR_WAVE(1); break;
        case 2: TM_CSR_WAVE(2); break;
        case 4: TM_CSR_WAVE(4); break;
        case 8: TM_CSR_WAVE(8); break;
        default: goto generic;
        }
#undef TM_CSR_WAVE
        TM_HIP(hipGetLastError());
        return w.grid;
    }
generic:
    hipLaunchKernelGGL(spmm_csr_kernel<T>, dim3(g.grid), dim3(256), 0, s, H.n, ldv, g.tpr, g.rpb,
                       g.rows_per_block, H.rowptr, H.col, val, Cv, Xv, ndot, partials);
    TM_HIP(hipGetLastError());
    return g.grid;
}

template <typename T>
int spmm_stencil(hipStream_t s, const StencilDev &H, int64_t n, int ld, const T *C, T *X,
                 int ndot, double *partials) {
    const int ldv = ld / Vec<T>::W;
    TM_REQUIRE(ldv <= kMaxCv * 256, TM_ENOTSUP, "block too wide for the SpMM kernel");
    Geometry g = geometry(n, ldv);
    const T *Vp;
    if constexpr (sizeof(T) == 8) Vp = H.V64; else Vp = H.V32;
    if (const int ns = slab_count<T>(ld); ns > 0 && n >= 64 * kSlabGrid) {
        using E = typename SlabE<T>::type;
        const E *Ce = reinterpret_cast<const E *>(C);
        E *Xe = reinterpret_cast<E *>(X);
        const int ldE = ld / SlabE<T>::W;
#define TM_SLAB(ORD, ND)                                                                     \
    hipLaunchKernelGGL((spmm_stencil_slab_kernel<T, ORD, ND>), dim3(kSlabGrid), dim3(256), 0, s, \
                       n, ldE, ns, H, Vp, Ce, Xe, ndot, partials)
        if (H.ndim == 3 && H.order == 2) TM_SLAB(2, 3);
        else if (H.ndim == 3 && H.order == 4) TM_SLAB(4, 3);
        else if (H.ndim == 2 && H.order == 2) TM_SLAB(2, 2);
        else TM_SLAB(4, 2);
#undef TM_SLAB
        TM_HIP(hipGetLastError());
        return slab_partial_rows(ns);
    }
    auto Cv = reinterpret_cast<const typename Vec<T>::type *>(C);
    auto Xv = reinterpret_cast<typename Vec<T>::type *>(X);
    const int ncv = ldv / 64;
    if (ldv % 64 == 0 && (ncv == 1 || ncv == 2 || ncv == 4 || ncv == 8)) {
        Geometry w = wave_geometry(n);
#define TM_STW(NCV, ORD, ND)                                                                 \
    hipLaunchKernelGGL((spmm_stencil_wave_kernel<T, NCV, ORD, ND>), dim3(w.grid), dim3(256), 0, \
                       s, n, w.rows_per_block, H, Vp, Cv, Xv, ndot, partials)
#define TM_STW_ORD(NCV)                                                                      \
    if (H.ndim == 3 && H.order == 2) TM_STW(NCV, 2, 3);                                      \
    else if (H.ndim == 3 && H.order == 4) TM_STW(NCV, 4, 3);                                 \
    else if (H.ndim == 2 && H.order == 2) TM_STW(NCV, 2, 2);                                 \
    else TM_STW(NCV, 4, 2);
        switch (ncv) {
        case 1: TM_STW_ORD(1); break;
        case 2: TM_STW_ORD(2); break;
        case 4: TM_STW_ORD(4); break;
        default: TM_STW_ORD(8); break;
        }
#undef TM_STW_ORD
#undef TM_STW
        TM_HIP(hipGetLastError());
        return w.grid;
    }
#define TM_STENCIL_LAUNCH(ORD, ND)                                                         \
    hipLaunchKernelGGL((spmm_stencil_kernel<T, ORD, ND>), dim3(g.grid), dim3(256), 0, s, n, \
                       ldv, g.tpr, g.rpb, g.rows_per_block, H, Vp, Cv, Xv, ndot, partials)
    if (H.ndim == 3 && H.order == 2) TM_STENCIL_LAUNCH(2, 3);
    else if (H.ndim == 3 && H.order == 4) TM_STENCIL_LAUNCH(4, 3);
    else if (H.ndim == 2 && H.order == 2) TM_STENCIL_LAUNCH(2, 2);
    else if (H.ndim == 2 && H.order == 4) TM_STENCIL_LAUNCH(4, 2);
    else throw Error{TM_EINVAL, "unsupported stencil"};
#undef TM_STENCIL_LAUNCH
    TM_HIP(hipGetLastError());
    return g.grid;
}

template int spmm_csr<double>(hipStream_t, const CsrDev &, int, const double *, double *, int, double *);
template int spmm_csr<float>(hipStream_t, const CsrDev &, int, const float *, float *, int, double *);
template int spmm_stencil<double>(hipStream_t, const StencilDev &, int64_t, int, const double *, double *, int, double *);
template int spmm_stencil<float>(hipStream_t, const StencilDev &, int64_t, int, const float *, float *, int, double *);

}  // namespace tmin
