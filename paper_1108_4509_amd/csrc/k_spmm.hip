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

#include <algorithm>

namespace tmin {
namespace {

typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec;
template <> struct Vec<double> { using type = vd2; static constexpr int W = 2; };
template <> struct Vec<float> { using type = vf4; static constexpr int W = 4; };

constexpr int kMaxCv = 4;     // column vectors per lane of the generic kernels (ld <= 2048)
constexpr int kRedWords = 2048;   // LDS words of their dot fold: rpb * ld <= 2048
constexpr int kGridCap = 4096;   // 4 waves each: about 16 waves per CU

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
    __shared__ double red[kRedWords];
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
    __shared__ double red[kRedWords];
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

// UB nonzeros are gathered before any is consumed (UB * NCV vector loads in
// flight per lane); measured best: 8 for FP32 one-vector rows, 2 for two,
// 1 for four or more
template <typename T, int NCV, int UB = (NCV >= 4 ? 1 : (sizeof(T) == 4 && NCV == 1 ? 8 : (NCV == 2 && sizeof(T) == 4 ? 1 : 2)))>
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
        constexpr int U = UB;
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

// Column-chunked form: a chunk is 256 bytes of every row (16 lanes of
// 16-byte vectors; 4 rows per wave, 16 per workgroup pass), and the launch
// is chunk-major, so each XCD walks all rows of one chunk (or a contiguous
// part of them) in order.  The rows that neighbour the ones in flight then
// stay in that XCD's L2 even for stencil offsets of a whole grid plane.  The
// workgroup's row pointers, columns and values are staged in LDS first (two
// round trips for all its rows), and each lane group gathers two rows at a
// time.
constexpr int kChunkRows = 64;   // rows per workgroup
constexpr int kChunkMeta = 1024; // staged nonzeros per workgroup

template <typename T, int L, int UB, int RG>
__global__ __launch_bounds__(256) void spmm_csr_chunk_kernel(
    int64_t n, int rows_per_block, int nrb, int nchunks, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const T *__restrict__ val,
    const typename Vec<T>::type *__restrict__ C, typename Vec<T>::type *__restrict__ X,
    int ldv, int ndot, double *__restrict__ partials, SpmmEpi epi) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::W;
    constexpr int RPW = 64 / L, RPP = 4 * RPW;
    __shared__ double red[2][RPP][L * W];
    __shared__ int64_t rp[257];
    __shared__ int32_t cs[kChunkMeta];
    __shared__ T vs[kChunkMeta];
    const int64_t lb = logical_block(gridDim.x);
    if (lb >= (int64_t)nrb * nchunks) return;   // uniform
    const int chunk = (int)(lb / nrb), rb = (int)(lb - (int64_t)chunk * nrb);
    const int t = threadIdx.x, l = t % L, slot = t / L;
    const int cv = chunk * L + l;
    const int64_t r_begin = (int64_t)rb * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n) r_end = n;
    const int nr = (int)(r_end - r_begin);   // <= 256
    for (int i = t; i <= nr; i += 256) rp[i] = rowptr[r_begin + i];
    __syncthreads();
    const int64_t e0 = rp[0];
    const int ne = (int)(rp[nr] - e0);
    const bool staged = ne <= kChunkMeta;   // uniform
    if (staged) {
        for (int e = t; e < ne; e += 256) {
            cs[e] = col[e0 + e];
            vs[e] = val[e0 + e];
        }
    }
    __syncthreads();
    double ds[2][W];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int w = 0; w < W; ++w) ds[p][w] = 0.0;
    // batched operators: this lane's columns belong to problem grp, whose
    // diagonal term d_grp is added and whose affine coefficients apply
    const int grp = epi.dld > 0 ? cv * W / epi.dld : 0;
    const T *Dg = epi.D ? reinterpret_cast<const T *>(epi.D) + (int64_t)grp * n : nullptr;
    const T ea = (T)(epi.gab ? epi.gab[2 * grp] : epi.a);
    const T eb = (T)(epi.gab ? epi.gab[2 * grp + 1] : epi.b);
    const V *E = reinterpret_cast<const V *>(epi.E);
    const bool own = epi.affine || ndot > 0 || Dg;   // the epilogue reads the row's own c
    // c, e: the row's own vectors of C and E (loaded ahead by the caller)
    auto finish = [&](int64_t r, V acc, V c, V e) {
        if (own) {
            if (Dg) {
                const T dr = Dg[r];
#pragma unroll
                for (int w = 0; w < W; ++w) acc[w] = fma(dr, c[w], acc[w]);
            }
            if (epi.affine) {
#pragma unroll
                for (int w = 0; w < W; ++w) acc[w] = fma(eb, acc[w], ea * c[w]);
            }
            if (ndot > 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ds[0][w] += (double)c[w] * (double)acc[w];
                    if (ndot == 2) ds[1][w] += (double)c[w] * (double)c[w];
                    if (ndot == 3) ds[1][w] += (double)e[w] * (double)acc[w];
                }
            }
        }
        X[r * ldv + cv] = acc;
    };
    if (staged) {
        // RG rows per lane group at a time (rows i, i + RPP, ...), UB
        // nonzeros of each per batch, all gathers in flight together; slots
        // past a row's end read entry 0 with weight zero
        for (int i = slot; i < nr; i += RG * RPP) {
            int s0[RG], s1[RG];
            V acc[RG], cown[RG], eown[RG];
            int len = 0;
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int ig = i + g * RPP;
                const bool has = ig < nr;
                s0[g] = has ? (int)(rp[ig] - e0) : 0;
                s1[g] = has ? (int)(rp[ig + 1] - e0) : 0;
                len = max(len, s1[g] - s0[g]);
                acc[g] = V(0);
                // the epilogue's own rows of C and E are loaded with the
                // first gathers, not after them
                const int64_t rr = r_begin + (has ? ig : 0);
                cown[g] = own ? C[rr * ldv + cv] : V(0);
                eown[g] = ndot == 3 ? E[rr * ldv + cv] : V(0);
            }
            for (int o = 0; o < len; o += UB) {
                V v[RG][UB];
                T x[RG][UB];
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int u = 0; u < UB; ++u) {
                        const int q = s0[g] + o + u;
                        const bool in = q < s1[g];
                        v[g][u] = C[(int64_t)cs[in ? q : 0] * ldv + cv];
                        x[g][u] = in ? vs[in ? q : 0] : T(0);
                    }
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int u = 0; u < UB; ++u) acc[g] = fma_v<V, T>(x[g][u], v[g][u], acc[g]);
            }
#pragma unroll
            for (int g = 0; g < RG; ++g)
                if (i + g * RPP < nr) finish(r_begin + i + g * RPP, acc[g], cown[g], eown[g]);
        }
    } else {
        for (int i = slot; i < nr; i += RPP) {
            V acc = V(0);
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
                acc = fma_v<V, T>(val[k], C[(int64_t)col[k] * ldv + cv], acc);
            const int64_t r = r_begin + i;
            finish(r, acc, own ? C[r * ldv + cv] : V(0), ndot == 3 ? E[r * ldv + cv] : V(0));
        }
    }
    if (ndot > 0) {
        // the RPP row slots meet in LDS; summed in slot order
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) red[p][slot][l * W + w] = ds[p][w];
        __syncthreads();
        const int ld = ldv * W;
        if (t < 2 * L * W) {
            const int p = t / (L * W), e = t - p * (L * W);
            if (p < (ndot == 3 ? 2 : ndot)) {
                double sum = 0.0;
                for (int g = 0; g < RPP; ++g) sum += red[p][g][e];
                partials[((int64_t)p * nrb + rb) * ld + chunk * L * W + e] = sum;
            }
        }
    }
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

// 3-D second-order (7-point) stencil, marching along z.  A workgroup owns a
// TX x TY tile of the xy plane, one 16-lane column chunk (16-byte vectors per
// lane) and a slab of ZS planes.  Each of its 16 point slots keeps the values
// of its NPT points at planes z-1, z, z+1 in registers, so every element of C
// is loaded once per slab (plus one plane at each slab end) instead of being
// gathered by its six neighbours; the in-plane neighbours come from the plane's
// tile and its one-point halo ring, staged in LDS.  Dirichlet boundaries read
// zeros outside the grid; periodic ones wrap (a ragged last tile holds the
// periodic images, so its active points see the right neighbours).  The fused
// column dots are summed per workgroup in FP64 and written as the partial row
// (zslab * nty + ty) * ntx + tx.
constexpr int kZL = 16;    // lanes per column chunk

template <typename T, int TX, int TY, int ZS, int NDOT>
__global__ __launch_bounds__(256) void spmm_stencil_zmarch_kernel(
    StencilDev H, int ldv, const T *__restrict__ Vpot, const typename Vec<T>::type *__restrict__ C,
    typename Vec<T>::type *__restrict__ X, int ntx, int nty, int nzs, int nch,
    double *__restrict__ partials, SpmmEpi epi) {
    constexpr int ndot = NDOT;
    using V = typename Vec<T>::type;
    const V *E = reinterpret_cast<const V *>(epi.E);
    constexpr int W = Vec<T>::W;
    constexpr int L = kZL, NS = 256 / L, NP = TX * TY, NPT = NP / NS;
    static_assert(NP % NS == 0, "tile");
    constexpr int HX = TX + 2, HY = TY + 2;
    __shared__ V tile[HY * HX * L];
    __shared__ double red[NDOT > 0 ? 2 : 1][NDOT > 0 ? NS : 1][NDOT > 0 ? L * W : 1];
    const int nx = H.nx, ny = H.ny, nz = H.nz;
    const bool per = H.periodic != 0;
    const int64_t lb = logical_block(gridDim.x);
    const int64_t nblk = (int64_t)ntx * nty * nzs;
    if (lb >= nblk * nch) return;   // uniform
    const int ch = (int)(lb / nblk);
    const int64_t cb = lb - (int64_t)ch * nblk;   // partial row of this workgroup
    const int tx = (int)(cb % ntx), ty = (int)((cb / ntx) % nty), zsb = (int)(cb / ((int64_t)ntx * nty));
    const int t = threadIdx.x, l = t % L, slot = t / L;
    const int cv = ch * L + l;
    const int x0 = tx * TX, y0 = ty * TY, z0 = zsb * ZS;
    const int z1 = min(z0 + ZS, nz);
    const int64_t plane = (int64_t)nx * ny;
    const T c0 = (T)H.c0, c1 = (T)H.c1;
    auto wrap = [](int c, int e) {
        c %= e;
        return c < 0 ? c + e : c;
    };
    int px[NPT], py[NPT];
    bool act[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int p = slot + k * NS;
        px[k] = x0 + p % TX;
        py[k] = y0 + p / TX;
        act[k] = px[k] < nx && py[k] < ny;
        if (per) {
            px[k] = wrap(px[k], nx);
            py[k] = wrap(py[k], ny);
        }
    }
    // value at (x, y, zz) of this lane's column vector; zero outside a
    // Dirichlet grid
    auto load = [&](int x, int y, int zz) -> V {
        if (per) {
            zz = wrap(zz, nz);
        } else if (zz < 0 || zz >= nz || x < 0 || x >= nx || y < 0 || y >= ny) {
            return V(0);
        }
        return C[((int64_t)zz * plane + (int64_t)y * nx + x) * ldv + cv];
    };
    V c[NPT][3];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        c[k][0] = load(px[k], py[k], z0 - 1);
        c[k][1] = load(px[k], py[k], z0);
    }
    double ds[2][W];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int w = 0; w < W; ++w) ds[p][w] = 0.0;
    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) c[k][2] = load(px[k], py[k], z + 1);
        __syncthreads();   // the previous plane's tile has been read
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = slot + k * NS;
            tile[((p / TX + 1) * HX + (p % TX + 1)) * L + l] = c[k][1];
        }
        // the halo ring: the two full rows, then the two side columns
        constexpr int NH = 2 * HX + 2 * TY;
        for (int h = slot; h < NH; h += NS) {
            int hx, hy;
            if (h < HX) { hy = 0; hx = h; }
            else if (h < 2 * HX) { hy = HY - 1; hx = h - HX; }
            else { const int g = h - 2 * HX; hy = 1 + g / 2; hx = (g & 1) ? HX - 1 : 0; }
            int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
            if (per) {
                gx = wrap(gx, nx);
                gy = wrap(gy, ny);
            }
            tile[(hy * HX + hx) * L + l] = load(gx, gy, z);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!act[k]) continue;
            const int p = slot + k * NS;
            const int lx = p % TX + 1, ly = p / TX + 1;
            const int64_t row = (int64_t)z * plane + (int64_t)py[k] * nx + px[k];
            const T dg = c0 + (Vpot ? Vpot[row] : (T)0);
            const V s1 = tile[(ly * HX + lx - 1) * L + l] + tile[(ly * HX + lx + 1) * L + l] +
                         tile[((ly - 1) * HX + lx) * L + l] + tile[((ly + 1) * HX + lx) * L + l] +
                         c[k][0] + c[k][2];
            const V ctr = c[k][1];
            V acc;
#pragma unroll
            for (int w = 0; w < W; ++w) acc[w] = fma(dg, ctr[w], c1 * s1[w]);
            if (epi.affine) {
                const T ea = (T)epi.a, eb = (T)epi.b;
#pragma unroll
                for (int w = 0; w < W; ++w) acc[w] = fma(eb, acc[w], ea * ctr[w]);
            }
            X[row * ldv + cv] = acc;
            if constexpr (NDOT > 0) {
                V e = V(0);
                if constexpr (NDOT == 3) e = E[row * ldv + cv];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    ds[0][w] += (double)ctr[w] * (double)acc[w];
                    if (NDOT == 2) ds[1][w] += (double)ctr[w] * (double)ctr[w];
                    if (NDOT == 3) ds[1][w] += (double)e[w] * (double)acc[w];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            c[k][0] = c[k][1];
            c[k][1] = c[k][2];
        }
    }
    if constexpr (NDOT > 0) {
        // the point slots meet in LDS and are summed in slot order
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int w = 0; w < W; ++w) red[p][slot][l * W + w] = ds[p][w];
        __syncthreads();
        const int ld = ldv * W;
        if (t < 2 * L * W) {
            const int p = t / (L * W), e = t - p * (L * W);
            if (p < (ndot == 3 ? 2 : ndot)) {
                double sum = 0.0;
                for (int g = 0; g < NS; ++g) sum += red[p][g][e];
                partials[((int64_t)p * nblk + cb) * ld + ch * L * W + e] = sum;
            }
        }
    }
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

size_t spmm_partials_workspace(int64_t n, int ld) {
    // the wave kernels write one partial row per workgroup (at most
    // kGridCap + 8), the chunked kernel one per 64-row block
    const int64_t nrb = (n + kChunkRows - 1) / kChunkRows;
    return (size_t)2 * std::max<int64_t>(kGridCap + 8, nrb) * ld * sizeof(double);
}

bool spmm_fast_path(bool stencil, const StencilDev &st, int ld, bool f64) {
    const int ldv = ld / (f64 ? 2 : 4);
    if (!stencil) return ldv % 16 == 0;
    return st.ndim == 3 && st.order == 2 && ldv % kZL == 0 && st.nx >= 3 && st.ny >= 3 && st.nz >= 3;
}

template <typename T>
int spmm_csr(hipStream_t s, const CsrDev &H, int ld, const T *C, T *X, int ndot,
             double *partials, const SpmmEpi &epi) {
    const int ldv = ld / Vec<T>::W;
    const T *val;
    if constexpr (sizeof(T) == 8) val = H.val64; else val = H.val32;
    auto Cv = reinterpret_cast<const typename Vec<T>::type *>(C);
    auto Xv = reinterpret_cast<typename Vec<T>::type *>(X);
    // chunk width and in-flight gathers: 256-byte chunks (16 lanes of 16-byte
    // vectors) with 4 rows per lane group in flight, one nonzero of each per
    // batch, for FP32 and FP64 rows.  Measured (HIP events, 20 launches): at
    // 48^3, m = 256, FP64 147 us against 149 us with 512-byte chunks and 8
    // rows; at 64^3 13-point, m = 512, 944 against 1028 us (the +-2 plane
    // window of a 512-byte chunk no longer fits one XCD's L2); 128-byte
    // chunks, 8 nonzeros per batch or 2 rows per group were slower at both
    // sizes.  Once the epilogue's own row is loaded with the first gathers
    // (121 registers), one nonzero per batch beats two: 48^3 FP64 134 against
    // 144 us, FP32 52 either way; 64^3 13-point FP64 920 against 945, FP32
    // 463 against 471 us
    if (ldv % 16 == 0) {
        const int nchunks = ldv / 16;
        const int64_t rpb = kChunkRows;
        const int64_t nrb64 = (H.n + rpb - 1) / rpb;
        TM_REQUIRE(nrb64 * nchunks < ((int64_t)1 << 31), TM_ENOTSUP, "matrix too large for the SpMM grid");
        const int nrb = (int)nrb64;
        int64_t grid = (int64_t)nchunks * nrb;
        grid = (grid + 7) / 8 * 8;
        hipLaunchKernelGGL((spmm_csr_chunk_kernel<T, 16, 1, 4>), dim3((unsigned)grid), dim3(256), 0, s,
                           H.n, (int)rpb, nrb, nchunks, H.rowptr, H.col, val, Cv, Xv, ldv, ndot,
                           partials, epi);
        TM_HIP(hipGetLastError());
        return nrb;
    }
    TM_REQUIRE(!epi.affine && ndot < 3 && !epi.D, TM_ENOTSUP,
               "SpMM epilogue needs the column-chunked kernel");
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
    TM_REQUIRE(ldv <= kMaxCv * 256, TM_ENOTSUP, "block too wide for the SpMM kernel");
    Geometry g = geometry(H.n, ldv);
    hipLaunchKernelGGL(spmm_csr_kernel<T>, dim3(g.grid), dim3(256), 0, s, H.n, ldv, g.tpr, g.rpb,
                       g.rows_per_block, H.rowptr, H.col, val, Cv, Xv, ndot, partials);
    TM_HIP(hipGetLastError());
    return g.grid;
}

template <typename T>
int spmm_stencil(hipStream_t s, const StencilDev &H, int64_t n, int ld, const T *C, T *X,
                 int ndot, double *partials, const SpmmEpi &epi) {
    const int ldv = ld / Vec<T>::W;
    const T *Vp;
    if constexpr (sizeof(T) == 8) Vp = H.V64; else Vp = H.V32;
    auto Cv = reinterpret_cast<const typename Vec<T>::type *>(C);
    auto Xv = reinterpret_cast<typename Vec<T>::type *>(X);
    if (H.ndim == 3 && H.order == 2 && ldv % kZL == 0 && H.nx >= 3 && H.ny >= 3 && H.nz >= 3) {
        // tiles measured at 48^3 and 100^3 (m = 256, 1024): FP64 8 x 8 x 8
        // (107 us, 3.8 ms), FP32 4 x 4 x 16 (42 us at 48^3)
        constexpr int TX = sizeof(T) == 8 ? 8 : 4, TY = TX, ZS = sizeof(T) == 8 ? 8 : 16;
        const int ntx = (H.nx + TX - 1) / TX, nty = (H.ny + TY - 1) / TY, nzs = (H.nz + ZS - 1) / ZS;
        const int nch = ldv / kZL;
        const int64_t nblk = (int64_t)ntx * nty * nzs;
        int64_t grid = nblk * nch;
        grid = (grid + 7) / 8 * 8;
        TM_REQUIRE(grid < ((int64_t)1 << 31), TM_ENOTSUP, "grid too large for the stencil SpMM");
#define TM_ZM(ND)                                                                                \
    hipLaunchKernelGGL((spmm_stencil_zmarch_kernel<T, TX, TY, ZS, ND>), dim3((unsigned)grid), dim3(256), 0, \
                       s, H, ldv, Vp, Cv, Xv, ntx, nty, nzs, nch, partials, epi)
        if (ndot == 0) TM_ZM(0);
        else if (ndot == 1) TM_ZM(1);
        else if (ndot == 2) TM_ZM(2);
        else TM_ZM(3);
#undef TM_ZM
        TM_HIP(hipGetLastError());
        return (int)nblk;
    }
    TM_REQUIRE(!epi.affine && ndot < 3, TM_ENOTSUP, "SpMM epilogue needs the 3-D 7-point stencil kernel");
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
    TM_REQUIRE(ldv <= kMaxCv * 256, TM_ENOTSUP, "block too wide for the SpMM kernel");
    Geometry g = geometry(n, ldv);
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

template int spmm_csr<double>(hipStream_t, const CsrDev &, int, const double *, double *, int, double *, const SpmmEpi &);
template int spmm_csr<float>(hipStream_t, const CsrDev &, int, const float *, float *, int, double *, const SpmmEpi &);
template int spmm_stencil<double>(hipStream_t, const StencilDev &, int64_t, int, const double *, double *, int, double *, const SpmmEpi &);
template int spmm_stencil<float>(hipStream_t, const StencilDev &, int64_t, int, const float *, float *, int, double *, const SpmmEpi &);

}  // namespace tmin
