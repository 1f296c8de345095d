// O(mN) block kernels: column dot products, the CG vector updates of Fig. 1,
// precision conversions, and the single-workgroup CG controller that decides
// gamma (Eq. 8), restarts, alpha and convergence without a host round trip.
#include "tm_common.h"

#include <cmath>

namespace tmin {
namespace {

constexpr int kDotThreads = 256;

// Column-dot partial sums.  grid.x = row chunks, grid.y = 256-column slabs.
// Within a slab of width w, 256 / w rows are visited at once; the per-row
// partial sums are folded in LDS in a fixed order.
template <typename T>
__global__ __launch_bounds__(kDotThreads) void coldots_kernel(
    int64_t n, int ld, int64_t rows_per_chunk, DotArgs<T> args,
    double *__restrict__ partials) {
    __shared__ double red[4][kDotThreads];
    const int slab0 = blockIdx.y * kDotThreads;
    int w = ld - slab0;
    if (w > kDotThreads) w = kDotThreads;
    const int ri = kDotThreads / w;
    const int t = threadIdx.x;
    const int ro = t / w;
    const int j = slab0 + (t - ro * w);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
    int64_t r1 = r0 + rows_per_chunk;
    if (r1 > n) r1 = n;
    if (ro < ri) {
        const double scj = (args.kind == 1) ? args.sc[j] : 0.0;
        for (int64_t r = r0 + ro; r < r1; r += ri) {
            const int64_t e = r * ld + j;
            const double wr = args.w ? args.w[r] : 1.0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if (p >= args.nprod) break;
                const double a = (double)args.a[p][e];
                const double b = (double)args.b[p][e];
                double v;
                if (args.kind == 1) {
                    const double d = a - scj * b;
                    v = d * d;
                } else {
                    v = a * b;
                }
                if (args.weighted[p]) v *= wr;
                acc[p] += v;
            }
        }
    }
    for (int p = 0; p < 4; ++p) red[p][t] = acc[p];
    __syncthreads();
    if (t < w) {
        for (int p = 0; p < args.nprod; ++p) {
            double s = 0.0;
            for (int q = 0; q < ri; ++q) s += red[p][q * w + t];
            partials[((int64_t)p * gridDim.x + blockIdx.x) * ld + slab0 + t] = s;
        }
    }
}

// Sum of per-chunk partial rows, partials[(p * nchunk + c) * ld + j] over c,
// for each product p and column j.  A workgroup takes 8 columns; its 128 lane
// groups stride over the chunks (loads unrolled to keep many in flight), then
// the group sums are combined by a fixed pairwise tree.
__global__ __launch_bounds__(1024) void coldots_reduce_kernel(
    int nchunk, int ld, const double *__restrict__ partials, double *__restrict__ out) {
    constexpr int CW = 8, NG = 1024 / CW;
    __shared__ double red[NG][CW + 1];
    const int p = blockIdx.x;
    const int t = threadIdx.x;
    const int c = t % CW, g = t / CW;
    const int j = blockIdx.y * CW + c;
    double s = 0.0;
    if (j < ld) {
        const double *base = partials + (int64_t)p * nchunk * ld + j;
#pragma unroll 8
        for (int q = g; q < nchunk; q += NG) s += base[(int64_t)q * ld];
    }
    red[g][c] = s;
    __syncthreads();
    for (int w = NG / 2; w >= 1; w >>= 1) {
        if (g < w) red[g][c] += red[g + w][c];
        __syncthreads();
    }
    if (g == 0 && j < ld) out[(int64_t)p * ld + j] = red[0][c];
}

int dot_chunks(int64_t n) {
    int64_t c = n / 128;
    if (c < 1) c = 1;
    if (c > 1024) c = 1024;
    return (int)c;
}

template <typename TG, typename TP>
__global__ void p_update_kernel(int64_t count, int ld, int ldg, const TG *__restrict__ G,
                                const double *__restrict__ M,
                                const CgState *__restrict__ st,
                                TP *__restrict__ P) {
    // 16-byte vectors of the block (count and ld are multiples of 32), the
    // same arithmetic per element as a scalar loop
    static_assert(sizeof(TG) == sizeof(TP), "G and P share a precision");
    constexpr int W = 16 / sizeof(TP);
    typedef TG VG __attribute__((ext_vector_type(W)));
    typedef TP VP __attribute__((ext_vector_type(W)));
    const int64_t nv = count / W;
    const double gamma0 = st->gamma;
    const bool grouped = ldg < ld;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        // gamma of the vector's column group (one group unless batched)
        const double gamma = grouped ? st[(int)((v * W) % ld) / ldg].gamma : gamma0;
        const VG g = reinterpret_cast<const VG *>(G)[v];
        const double mw = M ? M[(v * W) / ld] : 1.0;   // one row per vector
        VP out;
        if (gamma != 0.0) {
            const VP pv = reinterpret_cast<const VP *>(P)[v];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double z = (double)g[w];
                if (M) z *= mw;
                out[w] = (TP)(z + gamma * (double)pv[w]);
            }
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double z = (double)g[w];
                if (M) z *= mw;
                out[w] = (TP)z;
            }
        }
        reinterpret_cast<VP *>(P)[v] = out;
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32 x 32 -> 64-bit products
// mixed with the key, the key advanced by the Weyl increments between rounds.
__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Standard normal entries of an n x ld block (columns >= m zero): entry
// e = r * m + j is member e % 2 of the Box-Muller pair made from the Philox
// output for counter (e / 2, 0, 0, 0).
// Writes columns col0 .. col0 + width - 1 of an n x ld block; entry (r, j)
// of the problem (j < m) lands in column col0 + j.
__global__ void random_block_kernel(int64_t n, int m, int width, int ld, int col0, uint32_t k0,
                                    uint32_t k1, double *__restrict__ out) {
    const int64_t total = n * width;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / width;
        const int j = (int)(idx - r * width);
        double v = 0.0;
        if (j < m) {
            const uint64_t e = (uint64_t)r * (uint64_t)m + (uint64_t)j;
            const uint64_t k = e >> 1;
            uint32_t c[4] = {(uint32_t)k, (uint32_t)(k >> 32), 0u, 0u};
            philox4x32_10(c, k0, k1);
            const uint64_t a = (((uint64_t)c[1] << 32) | c[0]) >> 11;
            const uint64_t b = (((uint64_t)c[3] << 32) | c[2]) >> 11;
            const double u1 = (double)(a + 1) * 0x1.0p-53;   // (0, 1]
            const double u2 = (double)b * 0x1.0p-53;         // [0, 1)
            const double rad = sqrt(-2.0 * log(u1));
            const double th = 6.283185307179586476925286766559 * u2;
            v = (e & 1) ? rad * sin(th) : rad * cos(th);
        }
        out[r * ld + col0 + j] = v;
    }
}

// Chebyshev iteration for (H - sigma) z = g from z = 0, applied to a block
// in the block's own precision (the polynomial preconditioner of Eq. 18):
// start d = g / theta, z = d; step k: r <- r - (H d - sigma d),
// d <- c_dd d + c_r r, z <- z + d.  16-byte vectors (count is a multiple of
// 32), arithmetic in T.
template <typename T>
__global__ void cheb_init_kernel(int64_t count, const T *__restrict__ g, T inv_theta,
                                 T *__restrict__ d, T *__restrict__ z) {
    constexpr int W = 16 / sizeof(T);
    typedef T VT __attribute__((ext_vector_type(W)));
    const int64_t nv = count / W;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const VT x = reinterpret_cast<const VT *>(g)[v];
        VT o;
#pragma unroll
        for (int w = 0; w < W; ++w) o[w] = x[w] * inv_theta;
        reinterpret_cast<VT *>(d)[v] = o;
        reinterpret_cast<VT *>(z)[v] = o;
    }
}

template <typename T>
__global__ void cheb_step_kernel(int64_t count, const T *__restrict__ t, const T *r_in, T *r_out,
                                 T *__restrict__ d, T *__restrict__ z, T sigma, T c_dd, T c_r) {
    constexpr int W = 16 / sizeof(T);
    typedef T VT __attribute__((ext_vector_type(W)));
    const int64_t nv = count / W;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const VT tv = reinterpret_cast<const VT *>(t)[v];
        const VT rv = reinterpret_cast<const VT *>(r_in)[v];
        const VT dv = reinterpret_cast<const VT *>(d)[v];
        const VT zv = reinterpret_cast<const VT *>(z)[v];
        VT ro, dn, zo;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            ro[w] = rv[w] - (tv[w] - sigma * dv[w]);
            dn[w] = c_dd * dv[w] + c_r * ro[w];
            zo[w] = zv[w] + dn[w];
        }
        reinterpret_cast<VT *>(r_out)[v] = ro;
        reinterpret_cast<VT *>(d)[v] = dn;
        reinterpret_cast<VT *>(z)[v] = zo;
    }
}

// Cn = C + alpha P with alpha from the controller (Fig. 1's update), for
// the generalized problem, whose S-Gram cannot form it on the fly.
template <typename TP>
__global__ void update_block_kernel(int64_t count, const double *__restrict__ C,
                                    const TP *__restrict__ P, const CgState *__restrict__ st,
                                    double *__restrict__ Cn) {
    const double alpha = st->alpha;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        Cn[e] = C[e] + alpha * (double)P[e];
}

// Xs = X - Z diag(h) (Fig. 2 step (5) in the S metric: Z = S C).
__global__ void shift_block_kernel(int64_t count, int ld, const double *__restrict__ X,
                                   const double *__restrict__ Z, const double *__restrict__ h,
                                   double *__restrict__ Xs) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        Xs[e] = X[e] - Z[e] * h[e % ld];
}

// out[j] = v[j] for j < m, 0 for m <= j < ld.
__global__ void pad_vector_kernel(int m, int ld, const double *__restrict__ v,
                                  double *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ld) out[j] = j < m ? v[j] : 0.0;
}

// Diagonal preconditioner of Eq. 18: M_ii = 1 / (H_ii - sigma).
__global__ void jacobi_precond_kernel(int64_t n, const double *__restrict__ diag, double sigma,
                                      double *__restrict__ M) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        M[i] = 1.0 / (diag[i] - sigma);
}

template <typename TI, typename TO>
__global__ void convert_kernel(int64_t count, const TI *__restrict__ in,
                               TO *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (TO)in[e];
}

int elem_grid(int64_t count) {
    int64_t g = (count + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

// Fixed-order sum of v[0..m) by one workgroup of 256 lanes.
__device__ double block_sum(const double *v, int m, double *red) {
    const int t = threadIdx.x;
    double s = 0.0;
    for (int j = t; j < m; j += 256) s += v[j];
    red[t] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) red[t] += red[t + k];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_max(const double *v, int m, double *red) {
    const int t = threadIdx.x;
    double s = 0.0;
    for (int j = t; j < m; j += 256) s = fmax(s, v[j]);
    red[t] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) red[t] = fmax(red[t], red[t + k]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Controller, part 1 (after the gradient): energy, residual norm,
// convergence and phase-switch tests, restart decision and Polak-Ribiere gamma.
// dots rows: 0 gg = tr(G^T G), 1 gz = tr(G^T Z), 2 tr(G_prev^T Z), 3 tr(P_prev^T G).
__global__ __launch_bounds__(256) void control_gamma_kernel(
    int m, int ld, int ldg, const double *__restrict__ h, const double *__restrict__ dots,
    CgState *st, double *history) {
    __shared__ double red[256];
    // group blockIdx.x of a batched solve: its columns start at g * ldg
    const int g = blockIdx.x;
    h += (int64_t)g * ldg;
    dots += (int64_t)g * ldg;
    st += g;
    const double E = block_sum(h, m, red);
    const double gg = block_sum(dots, m, red);
    const double gz = block_sum(dots + ld, m, red);
    const double gpz = block_sum(dots + 2 * ld, m, red);
    const double ppg = block_sum(dots + 3 * ld, m, red);
    if (threadIdx.x != 0) return;
    const double rho = 0.5 * sqrt(gg);
    st->E = E;
    st->rho = rho;
    const bool finite = isfinite(E) && isfinite(rho);
    if (!finite) st->nan_seen = 1;
    const bool active = !st->done && !st->phase_end;
    if (active) {
        if (history && st->it < st->history_len) {
            history[2 * st->it] = E;
            history[2 * st->it + 1] = rho;
        }
        st->it += 1;
    }
    if (active && (rho <= st->tol || !finite)) st->done = 1;
    if (active && !st->done && st->phase_gate) {
        if (rho <= st->switch_tol) st->phase_end = 1;
        if (st->stall_window > 0) {
            if (st->window_it == 0) st->E_window = E;
            st->window_it += 1;
            if (st->window_it > st->stall_window) {
                if (st->E_window - E < st->stall_tol * fabs(E)) st->phase_end = 1;
                st->window_it = 0;
            }
        }
    }
    if (st->done || st->phase_end) {
        st->gamma = 0.0;
        st->pg = 0.0;
        return;
    }
    bool restart = st->force_restart || !st->have_prev;
    if (st->have_prev && E > st->E_prev + st->rise_tol * fabs(st->E_prev)) restart = true;
    double gamma = 0.0;
    if (!restart) gamma = (gz - gpz) / st->gz_prev;
    double pg = gz;
    if (gamma != 0.0) pg += gamma * ppg;
    if (!(pg > 0.0) || !isfinite(gamma) || !isfinite(pg)) {  // not a descent direction
        gamma = 0.0;
        pg = gz;
    }
    if (gamma == 0.0) st->restarts += 1;
    st->gamma = gamma;
    st->pg = pg;
    st->E_prev = E;
    st->gz_prev = gz;
    st->have_prev = 1;
    st->force_restart = 0;
}

// Controller, part 2 (after Y = HP): step length from the second-order model
// curvature = 2 sum_j (p_j.y_j - h_j p_j.p_j), capped at 1 / max_j |p_j|.
// dots2 rows: 0 p_j.y_j, 1 p_j.p_j.
__global__ __launch_bounds__(256) void control_alpha_kernel(
    int m, int ld, int ldg, const double *__restrict__ h, const double *__restrict__ dots2,
    CgState *st) {
    __shared__ double red[256];
    const int g = blockIdx.x;
    h += (int64_t)g * ldg;
    dots2 += (int64_t)g * ldg;
    st += g;
    const double ppmax = block_max(dots2 + ld, m, red);
    // curvature terms, summed in a fixed order
    double local = 0.0;
    for (int j = threadIdx.x; j < m; j += 256)
        local += dots2[j] - h[j] * dots2[ld + j];
    red[threadIdx.x] = local;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (st->done || st->phase_end) {
        st->alpha = 0.0;
        return;
    }
    const double curv = 2.0 * red[0];
    const double cap = ppmax > 0.0 ? 1.0 / sqrt(ppmax) : 0.0;
    double alpha = cap;
    if (curv > 0.0) alpha = fmin(st->pg / curv, cap);
    if (!isfinite(alpha)) alpha = 0.0;
    st->alpha = alpha;
}

__global__ void sum_vector_kernel(int m, const double *v, double *out) {
    __shared__ double red[256];
    const double s = block_sum(v, m, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

size_t coldots_workspace(int64_t n, int ld) {
    return (size_t)4 * dot_chunks(n) * ld * sizeof(double);
}

template <typename T>
void coldots(hipStream_t s, int64_t n, int ld, const DotArgs<T> &args,
             double *partials, double *out) {
    const int nchunk = dot_chunks(n);
    const int64_t rows = (n + nchunk - 1) / nchunk;
    const int nslab = (ld + kDotThreads - 1) / kDotThreads;
    hipLaunchKernelGGL(coldots_kernel<T>, dim3(nchunk, nslab), dim3(kDotThreads), 0,
                       s, n, ld, rows, args, partials);
    reduce_partials(s, args.nprod, nchunk, ld, partials, out);
    TM_HIP(hipGetLastError());
}

void reduce_partials(hipStream_t s, int nprod, int nchunk, int ld, const double *partials,
                     double *out) {
    hipLaunchKernelGGL(coldots_reduce_kernel, dim3(nprod, (ld + 7) / 8), dim3(1024), 0, s,
                       nchunk, ld, partials, out);
    TM_HIP(hipGetLastError());
}

template <typename TG, typename TP>
void p_update(hipStream_t s, int64_t n, int ld, const TG *G, const double *M,
              const CgState *st, TP *P, int ldg) {
    const int64_t count = n * ld;
    hipLaunchKernelGGL((p_update_kernel<TG, TP>), dim3(elem_grid(count)), dim3(256),
                       0, s, count, ld, ldg > 0 ? ldg : ld, G, M, st, P);
    TM_HIP(hipGetLastError());
}

template <typename TI, typename TO>
void convert_block(hipStream_t s, int64_t count, const TI *in, TO *out) {
    hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3(elem_grid(count)), dim3(256),
                       0, s, count, in, out);
    TM_HIP(hipGetLastError());
}

void random_block(hipStream_t s, int64_t n, int m, uint64_t seed, double *out, int width,
                  int ld_out, int col0) {
    if (width <= 0) {
        width = ld_out = leading_dim(m);
        col0 = 0;
    }
    TM_REQUIRE(m <= width && col0 >= 0 && col0 + width <= ld_out, TM_EINVAL, "random block layout");
    hipLaunchKernelGGL(random_block_kernel, dim3(elem_grid(n * width)), dim3(256), 0, s, n, m, width,
                       ld_out, col0, (uint32_t)seed, (uint32_t)(seed >> 32), out);
    TM_HIP(hipGetLastError());
}

template <typename T>
void cheb_init(hipStream_t s, int64_t count, const T *g, double inv_theta, T *d, T *z) {
    hipLaunchKernelGGL((cheb_init_kernel<T>), dim3(elem_grid(count)), dim3(256), 0, s, count, g,
                       (T)inv_theta, d, z);
    TM_HIP(hipGetLastError());
}
template <typename T>
void cheb_step(hipStream_t s, int64_t count, const T *t, const T *r_in, T *r_out, T *d, T *z,
               double sigma, double c_dd, double c_r) {
    hipLaunchKernelGGL((cheb_step_kernel<T>), dim3(elem_grid(count)), dim3(256), 0, s, count, t, r_in,
                       r_out, d, z, (T)sigma, (T)c_dd, (T)c_r);
    TM_HIP(hipGetLastError());
}
template void cheb_init<double>(hipStream_t, int64_t, const double *, double, double *, double *);
template void cheb_init<float>(hipStream_t, int64_t, const float *, double, float *, float *);
template void cheb_step<double>(hipStream_t, int64_t, const double *, const double *, double *, double *,
                                double *, double, double, double);
template void cheb_step<float>(hipStream_t, int64_t, const float *, const float *, float *, float *,
                               float *, double, double, double);

template <typename TP>
void update_block(hipStream_t s, int64_t count, const double *C, const TP *P, const CgState *st,
                  double *Cn) {
    hipLaunchKernelGGL((update_block_kernel<TP>), dim3(elem_grid(count)), dim3(256), 0, s, count, C,
                       P, st, Cn);
    TM_HIP(hipGetLastError());
}
template void update_block<double>(hipStream_t, int64_t, const double *, const double *,
                                   const CgState *, double *);
template void update_block<float>(hipStream_t, int64_t, const double *, const float *,
                                  const CgState *, double *);

void shift_block(hipStream_t s, int64_t n, int ld, const double *X, const double *Z,
                 const double *h, double *Xs) {
    const int64_t count = n * ld;
    hipLaunchKernelGGL(shift_block_kernel, dim3(elem_grid(count)), dim3(256), 0, s, count, ld, X, Z,
                       h, Xs);
    TM_HIP(hipGetLastError());
}

void pad_vector(hipStream_t s, int m, int ld, const double *v, double *out) {
    hipLaunchKernelGGL(pad_vector_kernel, dim3((ld + 255) / 256), dim3(256), 0, s, m, ld, v, out);
    TM_HIP(hipGetLastError());
}

void jacobi_preconditioner(hipStream_t s, int64_t n, const double *diag, double sigma,
                           double *M) {
    hipLaunchKernelGGL(jacobi_precond_kernel, dim3(elem_grid(n)), dim3(256), 0, s, n, diag,
                       sigma, M);
    TM_HIP(hipGetLastError());
}

void cg_control_gamma(hipStream_t s, int m, int ld, const double *h,
                      const double *dots, CgState *st, double *history, int ngroups, int ldg) {
    hipLaunchKernelGGL(control_gamma_kernel, dim3(ngroups), dim3(256), 0, s, m, ld, ldg, h,
                       dots, st, history);
    TM_HIP(hipGetLastError());
}

void cg_control_alpha(hipStream_t s, int m, int ld, const double *h,
                      const double *dots2, CgState *st, int ngroups, int ldg) {
    hipLaunchKernelGGL(control_alpha_kernel, dim3(ngroups), dim3(256), 0, s, m, ld, ldg, h,
                       dots2, st);
    TM_HIP(hipGetLastError());
}

void sum_vector(hipStream_t s, int m, const double *v, double *out) {
    hipLaunchKernelGGL(sum_vector_kernel, dim3(1), dim3(256), 0, s, m, v, out);
    TM_HIP(hipGetLastError());
}

template void coldots<double>(hipStream_t, int64_t, int, const DotArgs<double> &, double *, double *);
template void coldots<float>(hipStream_t, int64_t, int, const DotArgs<float> &, double *, double *);
template void p_update<double, double>(hipStream_t, int64_t, int, const double *, const double *, const CgState *, double *, int);
template void p_update<float, float>(hipStream_t, int64_t, int, const float *, const double *, const CgState *, float *, int);
template void convert_block<double, float>(hipStream_t, int64_t, const double *, float *);
template void convert_block<float, double>(hipStream_t, int64_t, const float *, double *);

}  // namespace tmin
