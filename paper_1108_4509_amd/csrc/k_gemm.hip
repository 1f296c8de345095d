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
//   trmm_lds_kernel : the triangular product of Eq. 13 at ld = 256 with R'
//          held in LDS and C streamed once (see there).
//
// Operands are staged through LDS by 256-lane workgroups (2 x 2 waves); each
// wave owns a (B/2) x (B/2) output patch made of 16 x 16 MFMA blocks.  Matrix
// core precision TM is FP64 or FP32; loads may convert from FP64 storage
// (the MP2 policy keeps C in FP64 but runs steps (6) and (7) in FP32).
// Workgroup b runs on XCD b % 8, so the launch maps consecutive logical tiles
// to one XCD: row chunks of the tall operand stay in that XCD's L2.
#include "tm_common.h"

#include <type_traits>

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
// threads of a Gram workgroup: 8 waves as 2 x 4, each a 64 x 32 patch of a
// 128-wide tile (4 waves as 2 x 2 leave 2 per SIMD at the FP64 accumulator
// budget; 8 halve each wave's accumulators and staging).  The all-FP64
// shifted and updating products keep 4 waves: at 8 they exceed the
// 128-register budget of 4 waves per SIMD and spill.
template <typename TA, typename TM, bool SHIFT, bool UPD, typename TP>
constexpr int gram_threads() {
    return (sizeof(TA) == 8 && sizeof(TM) == 8 && (SHIFT || (UPD && sizeof(TP) == 8))) ? 256 : 512;
}
constexpr int kPad = 16;   // LDS row padding (elements) against bank conflicts

// 16-byte vector of T for global loads (clang vector types: element access
// with a constant index stays in registers)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = vf4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = vd2; static constexpr int W = 2; };

template <typename T>
__device__ inline typename Vec16<T>::type vzero() {
    return typename Vec16<T>::type(0);
}

template <typename T>
__device__ inline T velem(const typename Vec16<T>::type &v, int i) {
    return v[i];
}

// Inputs of the gradient traces fused into the EPI_GRAD epilogue
// (partials == nullptr: no fusion); see rot() in tm_common.h.
template <typename TO>
struct GradDots {
    const TO *Gp = nullptr;   // null: trace 2 (g_prev . M g) is not formed (reads 0)
    const TO *Pp = nullptr;
    const double *M = nullptr;
    double *partials = nullptr;
    const void *Xs = nullptr;   // EPI_GRADX: X' in the matrix-core precision
};

// rows of A and B per LDS stage: the FP32 instruction is twice as fast, so
// it gets twice the rows per synchronization
template <typename TM> constexpr int stage_rows() { return sizeof(TM) == 4 ? 32 : 16; }

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

// Which 16 x 16 blocks of a 128 x 128 tile a wave accumulates on a diagonal
// tile of a symmetric product.  The strictly lower 64 x 64 quarter (block
// rows 4-7, block columns 0-3) is the mirror of the upper one and is not
// formed; the other 48 blocks, taken column by column (columns 0-3: rows
// 0-3; columns 4-7: rows 0-7), are dealt in runs of 48 / waves.
// diag_block(nw, w, k) = 8 * (block row) + (block column) of the k-th block
// of wave w out of nw.
__host__ __device__ constexpr int diag_block(int nw, int w, int k) {
    const int q = w * (48 / nw) + k;
    return q < 16 ? 8 * (q % 4) + q / 4 : 8 * ((q - 16) % 8) + 4 + (q - 16) / 8;
}
__host__ __device__ constexpr unsigned diag_rows(int nw, int w) {
    unsigned r = 0;
    for (int k = 0; k < 48 / nw; ++k) r |= 1u << (diag_block(nw, w, k) / 8);
    return r;
}
__host__ __device__ constexpr unsigned diag_cols(int nw, int w) {
    unsigned c = 0;
    for (int k = 0; k < 48 / nw; ++k) c |= 1u << (diag_block(nw, w, k) % 8);
    return c;
}
constexpr bool diag_plan_ok(int nw) {
    // every block of the upper part exactly once, none of the lower quarter
    int seen[64] = {};
    for (int w = 0; w < nw; ++w)
        for (int k = 0; k < 48 / nw; ++k) ++seen[diag_block(nw, w, k)];
    for (int b = 0; b < 64; ++b)
        if (seen[b] != ((b / 8 >= 4 && b % 8 < 4) ? 0 : 1)) return false;
    return true;
}
static_assert(diag_plan_ok(4) && diag_plan_ok(8), "diagonal-tile block plan");
template <int V> struct IntC { static constexpr int value = V; };

// The update C_next = C + alpha P fused into S = C_next^T C_next (Fig. 1's
// step C + alpha P, then Fig. 4 step (1)): both operands are formed from C
// and P while they are staged, and the workgroups on the diagonal tiles store
// C_next (each element once).
template <typename TA, typename TP>
struct GramUpd {
    const TP *P = nullptr;
    const CgState *st = nullptr;
    TA *Cn = nullptr;
    int ldg = 0;   // batched solves: column j takes the alpha of st[j / ldg]
};

// One workgroup: a BM x BM tile of A^T B' over a chunk of rows.  Each lane
// loads 16-byte vectors from a fixed column group (so h is read once), the
// LDS stage is double-buffered, one barrier per stage.
template <typename TA, typename TM, int BM, bool SHIFT, bool UPD = false, typename TP = TA, int NT = kThreads>
__global__ __launch_bounds__(NT, NT / 128) void gram_kernel(
    int64_t n, int m, int ld, const TA *__restrict__ A, const TA *__restrict__ B,
    const double *__restrict__ h, int T, int ntiles, bool symmetric,
    int64_t rows_per_split, double *__restrict__ partials, GramUpd<TA, TP> up,
    TM *__restrict__ xout, int tg, int nwork) {
    constexpr int KT = stage_rows<TM>();
    constexpr int NW = NT / 64;             // waves: 2 x (NW / 2)
    constexpr int WM = BM / 2;              // rows of a wave's patch
    constexpr int WN = BM / (NW / 2);       // columns of a wave's patch
    constexpr int NBR = WM / 16, NBC = WN / 16;
    constexpr int VW = Vec16<TA>::W;
    constexpr int VPR = BM / VW;            // vectors per tile row
    constexpr int RPP = NT / VPR;           // tile rows per load pass
    constexpr int PASSES = KT / RPP;
    static_assert(KT % RPP == 0, "stage rows must be a multiple of rows per pass");
    using V = typename Vec16<TA>::type;
    using Acc = typename Mfma<TM>::acc_t;

    __shared__ TM As[2][KT][BM + kPad];
    __shared__ TM Bs[2][KT][BM + kPad];

    const int logical = xcd_logical(gridDim.x);
    if (logical >= nwork) return;   // uniform: the grid is rounded up to a multiple of 8
    const int split = logical / ntiles;
    const int tile = logical - split * ntiles;
    int ti, tj;
    if (tg > 0) {
        // block-diagonal result (batched solves): only the tiles of the
        // diagonal tg x tg tile blocks, each holding whole problems
        const int per = symmetric ? tg * (tg + 1) / 2 : tg * tg;
        const int grp = tile / per, r = tile - grp * per;
        if (symmetric) upper_tile(r, tg, ti, tj);
        else { ti = r / tg; tj = r - ti * tg; }
        ti += grp * tg;
        tj += grp * tg;
    } else if (symmetric) {
        upper_tile(tile, T, ti, tj);
    } else {
        ti = tile / T;
        tj = tile - ti * T;
    }
    const int i0 = ti * BM, j0 = tj * BM;
    const int64_t k_begin = (int64_t)split * rows_per_split;
    int64_t k_end = k_begin + rows_per_split;
    if (k_end > n) k_end = n;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave / (NW / 2), wj = wave % (NW / 2);
    const int cv = tid % VPR, rbase = tid / VPR;
    const int ci = i0 + cv * VW, cj = j0 + cv * VW;
    const bool ci_ok = ci < ld, cj_ok = cj < ld;   // ld is a multiple of 32
    const bool same = (ti == tj);

    double hv[VW];
#pragma unroll
    for (int w = 0; w < VW; ++w) hv[w] = (SHIFT && cj_ok) ? h[cj + w] : 0.0;

    Acc acc[NBR][NBC];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    // loads are unconditional (rows past the chunk end read a valid row and
    // columns past ld column 0, both zeroed at the store) so that no select
    // on a loaded value forces the prefetch to complete early
    typedef TP PV __attribute__((ext_vector_type(VW)));
    typedef TM XV __attribute__((ext_vector_type(VW)));   // VW elements of X'
    V ra[PASSES], rb[PASSES], rx[SHIFT ? PASSES : 1];
    PV pa[UPD ? PASSES : 1], pb[UPD ? PASSES : 1];
    int64_t krow[(UPD || SHIFT) ? PASSES : 1];
    bool rv[PASSES];
    const int ci_c = ci_ok ? ci : 0, cj_c = cj_ok ? cj : 0;
    TA alpha = TA(0), alpha_b = TA(0);
    if constexpr (UPD) {
        alpha = (TA)up.st[up.ldg > 0 ? ci_c / up.ldg : 0].alpha;
        alpha_b = (TA)up.st[up.ldg > 0 ? cj_c / up.ldg : 0].alpha;
    }
    // the workgroups of tile row 0 (of the diagonal tiles when only the
    // diagonal blocks run) store X' = X - C diag(h) for their columns (each
    // element once), in the matrix-core precision
    const bool xstore = SHIFT && xout != nullptr && (tg > 0 ? ti == tj : ti == 0);
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < PASSES; ++q) {
            const int64_t k = k0 + rbase + q * RPP;
            rv[q] = k < k_end;
            const int64_t kk = rv[q] ? k : k_begin;
            ra[q] = *reinterpret_cast<const V *>(A + kk * ld + ci_c);
            if constexpr (UPD || SHIFT) krow[q] = kk;
            if constexpr (UPD) {
                pa[q] = *reinterpret_cast<const PV *>(up.P + kk * ld + ci_c);
                if (!same) {
                    rb[q] = *reinterpret_cast<const V *>(B + kk * ld + cj_c);
                    pb[q] = *reinterpret_cast<const PV *>(up.P + kk * ld + cj_c);
                }
            } else {
                rb[q] = *reinterpret_cast<const V *>(B + kk * ld + cj_c);
            }
            if constexpr (SHIFT)
                if (!same) rx[q] = *reinterpret_cast<const V *>(A + kk * ld + cj_c);
        }
    };
    auto store = [&](int buf) {
        if constexpr (UPD) {
            // C_next = C + alpha P for both operands; the diagonal tiles keep it
#pragma unroll
            for (int q = 0; q < PASSES; ++q) {
#pragma unroll
                for (int w = 0; w < VW; ++w) {
                    ra[q][w] = ra[q][w] + alpha * (TA)pa[q][w];
                    if (same) rb[q][w] = ra[q][w];
                    else rb[q][w] = rb[q][w] + alpha_b * (TA)pb[q][w];
                }
                if (same && rv[q] && ci_ok) *reinterpret_cast<V *>(up.Cn + krow[q] * ld + ci) = ra[q];
            }
        }
#pragma unroll
        for (int q = 0; q < PASSES; ++q) {
            const int row = rbase + q * RPP;
            const bool va = rv[q] && ci_ok, vb = rv[q] && cj_ok;
            XV xv;
#pragma unroll
            for (int w = 0; w < VW; ++w) {
                As[buf][row][cv * VW + w] = va ? (TM)velem<TA>(ra[q], w) : TM(0);
                if constexpr (SHIFT) {
                    const TA xa = same ? velem<TA>(ra[q], w) : velem<TA>(rx[q], w);
                    TM x;
                    if constexpr (sizeof(TA) == 4) x = fmaf(-xa, (float)hv[w], velem<TA>(rb[q], w));
                    else x = (TM)((double)velem<TA>(rb[q], w) - (double)xa * hv[w]);
                    Bs[buf][row][cv * VW + w] = vb ? x : TM(0);
                    xv[w] = x;
                } else {
                    Bs[buf][row][cv * VW + w] = vb ? (TM)velem<TA>(rb[q], w) : TM(0);
                }
            }
            if constexpr (SHIFT)
                if (xstore && vb) *reinterpret_cast<XV *>(xout + krow[q] * ld + cj) = xv;
        }
    };

    // plan 0: the wave's WM x WN patch; plans 1..NW: wave plan - 1 of a
    // diagonal tile of a symmetric product (BM = 128, see diag_block)
    constexpr int PER = 48 / NW;
    double *P = partials + (int64_t)split * m * m;
    auto run = [&](auto plan) {
        constexpr int PL = decltype(plan)::value;
        constexpr int DW = PL - 1;
        int buf = 0;
        if (k_begin < k_end) {
            load(k_begin);
            store(0);
        }
        __syncthreads();
        for (int64_t k0 = k_begin; k0 < k_end; k0 += KT) {
            const bool more = k0 + KT < k_end;
            if (more) load(k0 + KT);
#pragma unroll
            for (int kk = 0; kk < KT; kk += 4) {
                const int kr = kk + (lane >> 4);
                if constexpr (PL == 0) {
                    TM fa[NBR], fb[NBC];
#pragma unroll
                    for (int a = 0; a < NBR; ++a) fa[a] = As[buf][kr][wi * WM + a * 16 + (lane & 15)];
#pragma unroll
                    for (int b = 0; b < NBC; ++b) fb[b] = Bs[buf][kr][wj * WN + b * 16 + (lane & 15)];
#pragma unroll
                    for (int a = 0; a < NBR; ++a)
#pragma unroll
                        for (int b = 0; b < NBC; ++b) acc[a][b] = Mfma<TM>::op(fa[a], fb[b], acc[a][b]);
                } else {
                    TM fa[8], fb[8];
#pragma unroll
                    for (int a = 0; a < 8; ++a)
                        if ((diag_rows(NW, DW) >> a) & 1u) fa[a] = As[buf][kr][a * 16 + (lane & 15)];
#pragma unroll
                    for (int b = 0; b < 8; ++b)
                        if ((diag_cols(NW, DW) >> b) & 1u) fb[b] = Bs[buf][kr][b * 16 + (lane & 15)];
#pragma unroll
                    for (int k = 0; k < PER; ++k)
                        acc[k / NBC][k % NBC] = Mfma<TM>::op(fa[diag_block(NW, DW, k) / 8],
                                                             fb[diag_block(NW, DW, k) % 8], acc[k / NBC][k % NBC]);
                }
            }
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
            for (int b = 0; b < NBC; ++b) {
                if (PL != 0 && a * NBC + b >= PER) continue;
                const int bi = PL == 0 ? wi * NBR + a : diag_block(NW, DW, a * NBC + b) / 8;
                const int bj = PL == 0 ? wj * NBC + b : diag_block(NW, DW, a * NBC + b) % 8;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + bi * 16 + Mfma<TM>::row(lane, r);
                    const int j = j0 + bj * 16 + (lane & 15);
                    if (i < m && j < m) P[(int64_t)i * m + j] = (double)acc[a][b][r];
                }
            }
    };
    if constexpr (BM == 128) {
        if (symmetric && same) {
            switch (wave) {
            case 0: run(IntC<1>{}); break;
            case 1: run(IntC<2>{}); break;
            case 2: run(IntC<3>{}); break;
            case 3: run(IntC<4>{}); break;
            case 4: if constexpr (NW > 4) run(IntC<5>{}); break;
            case 5: if constexpr (NW > 4) run(IntC<6>{}); break;
            case 6: if constexpr (NW > 4) run(IntC<7>{}); break;
            default: if constexpr (NW > 4) run(IntC<8>{}); break;
            }
            return;
        }
    }
    run(IntC<0>{});
}

// Sum over the row-chunk partials in a fixed order: 64 elements per
// workgroup, four lane groups take every fourth chunk, then the four group
// sums are added in order.  A symmetric product has partials only in the
// upper 64 x 64 blocks (block row <= block column: the upper tiles, less the
// lower quarter of 128-wide diagonal tiles): the elements of a strictly upper
// block are read there (rows contiguous) and written to both (i, j) and
// (j, i); lower blocks read nothing.
// With pad the workgroups cover the ld x ld padded matrix instead and also
// store it in the matrix-core precision (zeros outside m x m, mirrored for a
// symmetric product): the operand of the rotation GEMM that follows.
constexpr int kSymBlk = 64;
__global__ __launch_bounds__(256) void gram_reduce_kernel(int m, int nsplit, bool symmetric,
                                                          bool zero_diag,
                                                          const double *__restrict__ partials,
                                                          double *__restrict__ out, int ld,
                                                          float *__restrict__ padf,
                                                          double *__restrict__ padd,
                                                          BatchCols bc) {
    constexpr int E = 64, G = 4;
    __shared__ double red[G][E];
    const int e = threadIdx.x % E, g = threadIdx.x / E;
    const bool pad = padf != nullptr || padd != nullptr;
    const int cols = pad ? ld : m;
    const int64_t idx = (int64_t)blockIdx.x * E + e;
    const int64_t mm = (int64_t)m * m;
    double s = 0.0;
    int i = 0, j = 0;
    bool inside = idx < (int64_t)cols * cols;
    if (inside) {
        i = (int)(idx / cols);
        j = (int)(idx - (int64_t)i * cols);
    }
    const bool in_m = inside && i < m && j < m;
    bool active = in_m;
    if (active && symmetric && (i / kSymBlk) > (j / kSymBlk)) active = false;
    const int64_t src = (int64_t)i * m + j;
    if (active) {
#pragma unroll 8
        for (int p = g; p < nsplit; p += G) s += partials[(int64_t)p * mm + src];
    }
    red[g][e] = s;
    __syncthreads();
    if (g != 0 || !inside) return;
    double v = 0.0;
    if (active) {
        v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        if (zero_diag && i == j) v = 0.0;
        if (bc.ldg > 0) {
            // block-diagonal form of a batched solve (mirror-symmetric)
            const int gi = i / bc.ldg, gj = j / bc.ldg;
            const bool pi = i - gi * bc.ldg >= bc.mg, pj = j - gj * bc.ldg >= bc.mg;
            if (gi != gj || pi || pj) v = (i == j && pi) ? bc.pad : 0.0;
        }
        out[src] = v;
        if (symmetric && (i / kSymBlk) < (j / kSymBlk)) out[(int64_t)j * m + i] = v;
    }
    if (pad) {
        // lower tiles of a symmetric product are written by their mirror
        if (in_m && !active) return;
        const int64_t pidx = (int64_t)i * ld + j;
        if (padf) padf[pidx] = (float)v;
        else padd[pidx] = v;
        if (active && symmetric && (i / kSymBlk) < (j / kSymBlk)) {
            const int64_t q = (int64_t)j * ld + i;
            if (padf) padf[q] = (float)v;
            else padd[q] = v;
        }
    }
}

// ---------------------------------------------------------------- BF16x3 Gram
// H' = A^T B' on BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) with each operand split into two BF16 terms, x = hi + lo,
// hi = bf16(x), lo = bf16(x - hi): A^T B ~ hi_a^T hi_b + hi_a^T lo_b +
// lo_a^T hi_b, the lo_a^T lo_b term (2^-16 relative) dropped.  The split
// operand carries 16 significant bits, so the product is accurate to about
// 2^-16 relative to sum |a||b| -- between BF16 (2^-8) and FP32 (2^-24).
// The k dimension of a Gram product is the row index N, so the LDS tiles are
// stored k-contiguous: element (k, c) of a 32-row stage sits at
// [k / 8][c][k % 8], and one 16-byte read gives an MFMA lane its eight k.
// Loader map: thread t handles column pair t % (BM/2) and rows 8 g .. 8 g + 7
// of the stage, g = t / (BM/2).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// x rounded once to the 8 significant bits of BF16, in FP64: Veltkamp's
// splitting (Dekker 1971) with the constant 2^45 + 1 keeps the leading
// 53 - 45 = 8 bits of x rounded to nearest.  The result converts to FP32 and
// then to BF16 exactly, so FP64 operands are not rounded twice (through FP32).
// The splitting needs each operation rounded on its own: no FMA contraction
// of t - x (x * c - x in one rounding would break it).
__device__ inline double round_bf16_bits(double x) {
#pragma clang fp contract(off)
    const double t = x * 35184372088833.0;   // 2^45 + 1
    return t - (t - x);
}

// Two-term BF16 operand: hi = x to 8 bits, lo = the rest to 8 bits.
__device__ inline void split_bf16(double x, __bf16 &hi, __bf16 &lo) {
    const double h = round_bf16_bits(x);
    hi = (__bf16)(float)h;
    lo = (__bf16)(float)round_bf16_bits(x - h);
}

template <typename TA, int BM, bool SHIFT>
__global__ __launch_bounds__(kThreads, 2) void gram_bf16x3_kernel(
    int64_t n, int m, int ld, const TA *__restrict__ A, const TA *__restrict__ B,
    const double *__restrict__ h, int T, int ntiles, int64_t rows_per_split,
    double *__restrict__ partials) {
    constexpr int CP = BM / 2;              // column pairs per tile row
    constexpr int NKG = kThreads / CP;      // 8-row groups per stage
    constexpr int KT = 8 * NKG;             // rows per stage
    constexpr int WM = BM / 2;
    constexpr int NB = WM / 16;
    using Acc = typename Mfma<float>::acc_t;
    using V2 = typename std::conditional<sizeof(TA) == 8, vd2, float __attribute__((ext_vector_type(2)))>::type;

    __shared__ bf16x8 Ah[2][NKG][BM + 1], Al[2][NKG][BM + 1];
    __shared__ bf16x8 Bh[2][NKG][BM + 1], Bl[2][NKG][BM + 1];

    const int logical = xcd_logical(gridDim.x);
    const int split = logical / ntiles;
    const int tile = logical - split * ntiles;
    const int ti = tile / T, tj = tile - (tile / T) * T;
    const int i0 = ti * BM, j0 = tj * BM;
    const int64_t k_begin = (int64_t)split * rows_per_split;
    int64_t k_end = k_begin + rows_per_split;
    if (k_end > n) k_end = n;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave >> 1, wj = wave & 1;
    const int cp = tid % CP, kg = tid / CP;
    const int ci = i0 + 2 * cp, cj = j0 + 2 * cp;
    const bool ci_ok = ci < ld, cj_ok = cj < ld;   // ld is a multiple of 32
    const bool same = (ti == tj);
    double hv[2] = {0.0, 0.0};
    if (SHIFT && cj_ok) {
        hv[0] = h[cj];
        hv[1] = h[cj + 1];
    }

    Acc acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    V2 ra[8], rb[8], rx[SHIFT ? 8 : 1];
    bool rv[8];
    const int ci_c = ci_ok ? ci : 0, cj_c = cj_ok ? cj : 0;
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t k = k0 + 8 * kg + r;
            rv[r] = k < k_end;
            const int64_t kk = rv[r] ? k : k_begin;
            ra[r] = *reinterpret_cast<const V2 *>(A + kk * ld + ci_c);
            rb[r] = *reinterpret_cast<const V2 *>(B + kk * ld + cj_c);
            if constexpr (SHIFT)
                if (!same) rx[r] = *reinterpret_cast<const V2 *>(A + kk * ld + cj_c);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            bf16x8 ah, al, bh, bl;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                __bf16 x, y;
                split_bf16((rv[r] && ci_ok) ? (double)ra[r][c] : 0.0, x, y);
                ah[r] = x;
                al[r] = y;
                double bv = (double)rb[r][c];
                if constexpr (SHIFT) bv -= (double)(same ? ra[r][c] : rx[r][c]) * hv[c];
                split_bf16((rv[r] && cj_ok) ? bv : 0.0, x, y);
                bh[r] = x;
                bl[r] = y;
            }
            Ah[buf][kg][2 * cp + c] = ah;
            Al[buf][kg][2 * cp + c] = al;
            Bh[buf][kg][2 * cp + c] = bh;
            Bl[buf][kg][2 * cp + c] = bl;
        }
    };

    int buf = 0;
    if (k_begin < k_end) {
        load(k_begin);
        store(0);
    }
    __syncthreads();
    for (int64_t k0 = k_begin; k0 < k_end; k0 += KT) {
        const bool more = k0 + KT < k_end;
        if (more) load(k0 + KT);
#pragma unroll
        for (int ks = 0; ks < NKG / 4; ++ks) {
            const int g = 4 * ks + (lane >> 4);
            bf16x8 fah[NB], fal[NB], fbh[NB], fbl[NB];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                fah[a] = Ah[buf][g][wi * WM + a * 16 + (lane & 15)];
                fal[a] = Al[buf][g][wi * WM + a * 16 + (lane & 15)];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                fbh[b] = Bh[buf][g][wj * WM + b * 16 + (lane & 15)];
                fbl[b] = Bl[buf][g][wj * WM + b * 16 + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[a], fbh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[a], fbl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[a], fbh[b], acc[a][b], 0, 0, 0);
                }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    double *P = partials + (int64_t)split * m * m;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi * WM + a * 16 + Mfma<float>::row(lane, r);
                const int j = j0 + wj * WM + b * 16 + (lane & 15);
                if (i < m && j < m) P[(int64_t)i * m + j] = (double)acc[a][b][r];
            }
}

int gram_tile(int ld) { return ld >= 256 ? 128 : 64; }

// Tiles of a Gram launch: all of them, or, for a block-diagonal result with
// ldg-wide diagonal blocks (a batched solve), the diagonal tg x tg blocks of
// BM tiles that hold whole problems (tg = 1 when problems tile BM, ldg / BM
// when BM tiles a problem; 0: no skipping, the other cases).
int gram_tg(int BM, int ldg) {
    if (ldg <= 0) return 0;
    if (BM % ldg == 0) return 1;
    if (ldg % BM == 0) return ldg / BM;
    return 0;
}
int gram_ntiles(int T, bool symmetric, int tg) {
    if (tg > 0) return (T + tg - 1) / tg * (symmetric ? tg * (tg + 1) / 2 : tg * tg);
    return symmetric ? T * (T + 1) / 2 : T * T;
}

void gram_shape(int64_t n, int m, bool symmetric, int &BM, int &T, int &nsplit,
                size_t ws_bytes = 0, int ldg = 0) {
    const int ld = leading_dim(m);
    BM = gram_tile(ld);
    T = (ld + BM - 1) / BM;
    // two workgroups per CU (512 over the 256 CUs, so that no CU runs more
    // row chunks than another), at most 256 MiB of FP64 partials (or the
    // caller's workspace, ws_bytes), and at least 128 rows per split; the
    // grid (tiles x splits) is a multiple of 8 for the XCD mapping
    const int ntiles = gram_ntiles(T, symmetric, gram_tg(BM, ldg));
    int64_t ns = 512 / ntiles;
    int64_t cap_bytes = (int64_t)256 << 20;
    if (ws_bytes > 0 && (int64_t)ws_bytes < cap_bytes) cap_bytes = (int64_t)ws_bytes;
    int64_t cap = cap_bytes / ((int64_t)m * m * 8);
    if (ns > cap) ns = cap;
    int64_t cap_rows = n / 128;
    if (ns > cap_rows) ns = cap_rows;
    while (ns > 1 && (ntiles * ns) % 8 != 0) --ns;
    if (ns < 1 || (ntiles * ns) % 8 != 0) {
        ns = 1;
        while ((ntiles * ns) % 8 != 0) ++ns;
    }
    nsplit = (int)ns;
}

// One workgroup: a BR x BC tile of A W (+ epilogue), K looped in LDS stages.
template <typename T> __device__ inline void load4(const T *p, T (&v)[4]);
template <> __device__ inline void load4<float>(const float *p, float (&v)[4]) {
    const vf4 x = *reinterpret_cast<const vf4 *>(p);
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}
template <> __device__ inline void load4<double>(const double *p, double (&v)[4]) {
    const vd2 x = *reinterpret_cast<const vd2 *>(p), y = *reinterpret_cast<const vd2 *>(p + 2);
    v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
}
template <typename T> __device__ inline void store4(T *p, const T (&v)[4]);
template <> __device__ inline void store4<float>(float *p, const float (&v)[4]) {
    vf4 x;
    x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
    *reinterpret_cast<vf4 *>(p) = x;
}
template <> __device__ inline void store4<double>(double *p, const double (&v)[4]) {
    vd2 x, y;
    x[0] = v[0]; x[1] = v[1]; y[0] = v[2]; y[1] = v[3];
    *reinterpret_cast<vd2 *>(p) = x;
    *reinterpret_cast<vd2 *>(p + 2) = y;
}

template <typename TM, int BR, int BC>
struct RotSmem {
    static constexpr int KT = stage_rows<TM>();
    static constexpr int stage_bytes =
        (2 * BR * (KT + 1) + 2 * KT * (BC + kPad)) * (int)sizeof(TM);
    // rows of the accumulator tile per epilogue pass (FP64 tiles go in halves)
    static constexpr int EH = (BR * (BC + 4) * (int)sizeof(TM) <= stage_bytes) ? BR : BR / 2;
    static constexpr int tile_bytes = EH * (BC + 4) * (int)sizeof(TM);
    static constexpr int red_bytes = (kThreads / (BC / 4)) * 4 * BC * 8;
    static constexpr int a = stage_bytes > tile_bytes ? stage_bytes : tile_bytes;
    static constexpr int bytes = a > red_bytes ? a : red_bytes;
};

// One workgroup: a BR x BC tile of A W (+ epilogue), K looped in LDS stages.
// The accumulators then go through LDS so that the epilogue reads X and A,
// and writes the result, as row-contiguous 4-element vectors.
template <typename TA, typename TM, typename TO, int EPI, int BR, int BC>
__global__ __launch_bounds__(kThreads, 2) void rot_kernel(
    int64_t n, int m, int ld, const TA *__restrict__ A, const TM *__restrict__ W,
    const TA *__restrict__ X, const double *__restrict__ vec, TO *__restrict__ out,
    int nrb, int ncb, GradDots<TO> gd, int wg) {
    using SM = RotSmem<TM, BR, BC>;
    constexpr int KT = SM::KT;
    constexpr int WR = BR / 2, WC = BC / 2;
    constexpr int NBR = WR / 16, NBC = WC / 16;
    constexpr int VA = Vec16<TA>::W, VM = Vec16<TM>::W;
    constexpr int APR = KT / VA;            // A vectors per tile row
    constexpr int ARPP = kThreads / APR;    // A rows per pass
    constexpr int PA = BR / ARPP;
    constexpr int WPR = BC / VM;            // W vectors per tile row
    constexpr int WRPP = kThreads / WPR;
    constexpr int PW = KT / WRPP;
    static_assert(BR % ARPP == 0 && KT % WRPP == 0, "tile shape");
    using VAt = typename Vec16<TA>::type;
    using VMt = typename Vec16<TM>::type;
    using Acc = typename Mfma<TM>::acc_t;

    __shared__ __align__(16) char smem[SM::bytes];
    typedef TM AsRow[KT + 1];
    typedef TM WsRow[BC + kPad];
    AsRow *As0 = reinterpret_cast<AsRow *>(smem);                 // [2][BR][KT + 1]
    WsRow *Ws0 = reinterpret_cast<WsRow *>(smem + 2 * BR * (KT + 1) * sizeof(TM));   // [2][KT][BC+pad]

    const int logical = xcd_logical(gridDim.x);
    if (logical >= nrb * ncb) return;
    const int rb = logical / ncb, cb = logical - (logical / ncb) * ncb;
    const int64_t r0 = (int64_t)rb * BR;
    const int c0 = cb * BC;
    int kend = ld;
    if (EPI == EPI_TRMM && c0 + BC < kend) kend = c0 + BC;   // W strictly upper
    // block-diagonal W (wg-wide diagonal blocks): the tile's columns see only
    // the rows of the blocks they fall in; the products left out are exact
    // zeros, so the sums are those of the full loop
    int kbeg = 0;
    if (wg > 0) {
        kbeg = c0 / wg * wg;
        kbeg -= kbeg % KT;
        const int ge = (c0 + BC + wg - 1) / wg * wg;
        if (ge < kend) kend = ge;
    }

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int acv = tid % APR, arow = tid / APR;
    const int wcv = tid % WPR, wrow = tid / WPR;
    const bool wc_ok = c0 + wcv * VM < ld;

    Acc acc[NBR][NBC];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    VAt ra[PA];
    VMt rw[PW];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int64_t r = r0 + arow + q * ARPP;
            ra[q] = (r < n) ? *reinterpret_cast<const VAt *>(A + r * ld + k0 + acv * VA) : vzero<TA>();
        }
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int k = k0 + wrow + q * WRPP;
            rw[q] = wc_ok ? *reinterpret_cast<const VMt *>(W + (int64_t)k * ld + c0 + wcv * VM)
                          : vzero<TM>();
        }
    };
    auto store = [&](int buf) {
        AsRow *As = As0 + buf * BR;
        WsRow *Ws = Ws0 + buf * KT;
#pragma unroll
        for (int q = 0; q < PA; ++q)
#pragma unroll
            for (int w = 0; w < VA; ++w)
                As[arow + q * ARPP][acv * VA + w] = (TM)velem<TA>(ra[q], w);
#pragma unroll
        for (int q = 0; q < PW; ++q)
#pragma unroll
            for (int w = 0; w < VM; ++w) Ws[wrow + q * WRPP][wcv * VM + w] = velem<TM>(rw[q], w);
    };

    int buf = 0;
    load(kbeg);
    store(0);
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += KT) {
        const bool more = k0 + KT < kend;
        if (more) load(k0 + KT);
        const AsRow *As = As0 + buf * BR;
        const WsRow *Ws = Ws0 + buf * KT;
#pragma unroll
        for (int kk = 0; kk < KT; kk += 4) {
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
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // ---- epilogue through LDS, EH rows at a time
    constexpr int EH = SM::EH;
    constexpr int TS = BC + 4;                 // tile row stride
    constexpr int CVN = BC / 4;                // 4-column vectors per row
    constexpr int RPT = kThreads / CVN;        // rows per pass
    TM *tile = reinterpret_cast<TM *>(smem);
    const int ecv = tid % CVN, erow = tid / CVN;
    const int ecol = c0 + 4 * ecv;
    const bool col_ok = ecol < ld;             // ld is a multiple of 32
    constexpr bool GRADLIKE = EPI == EPI_GRAD || EPI == EPI_GRADX;
    const bool fuse = GRADLIKE && gd.partials != nullptr;
    const TM *Xs = reinterpret_cast<const TM *>(gd.Xs);
    double vv[4] = {0.0, 0.0, 0.0, 0.0};
    if ((EPI == EPI_GRAD || EPI == EPI_TRMM) && col_ok) {
#pragma unroll
        for (int w = 0; w < 4; ++w) vv[w] = vec[ecol + w];
    }
    double dsum[GRADLIKE ? 4 : 1][4];
#pragma unroll
    for (int p = 0; p < (GRADLIKE ? 4 : 1); ++p)
#pragma unroll
        for (int w = 0; w < 4; ++w) dsum[p][w] = 0.0;

#pragma unroll
    for (int half = 0; half < BR / EH; ++half) {
        if (half > 0) __syncthreads();
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
            for (int b = 0; b < NBC; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rl = wr * WR + a * 16 + Mfma<TM>::row(lane, r) - half * EH;
                    if (rl >= 0 && rl < EH) tile[rl * TS + wc * WC + b * 16 + (lane & 15)] = acc[a][b][r];
                }
        __syncthreads();
        // EG rows per lane at a time: all their loads are issued before any
        // result is formed, so the round trips overlap
        constexpr int EG = (sizeof(TM) == 8 && GRADLIKE) ? 1 : 4;   // FP64 tiles: no room
        static_assert(EH % (RPT * EG) == 0, "epilogue row groups");
        for (int rl0 = erow; rl0 < EH; rl0 += RPT * EG) {
            TA xv[EG][4], av[EG][4];
            TM xs[EG][4];
            TO gp[EG][4], pp[EG][4];
            double wgt[EG];
            bool ok[EG];
#pragma unroll
            for (int g = 0; g < EG; ++g) {
                const int rl = rl0 + g * RPT;
                const int64_t row = r0 + half * EH + rl;
                ok[g] = row < n && col_ok;
                const int64_t e = (ok[g] ? row : r0) * ld + (col_ok ? ecol : c0);
                if constexpr (EPI == EPI_GRAD) load4<TA>(X + e, xv[g]);
                if constexpr (EPI == EPI_GRADX) load4<TM>(Xs + e, xs[g]);
                if constexpr (EPI == EPI_GRAD || EPI == EPI_TRMM) load4<TA>(A + e, av[g]);
                if (GRADLIKE && fuse) {
                    if (gd.Gp) {
                        load4<TO>(gd.Gp + e, gp[g]);
                    } else {
#pragma unroll
                        for (int w = 0; w < 4; ++w) gp[g][w] = TO(0);
                    }
                    load4<TO>(gd.Pp + e, pp[g]);
                    wgt[g] = gd.M ? gd.M[ok[g] ? row : r0] : 1.0;
                }
            }
#pragma unroll
            for (int g = 0; g < EG; ++g) {
                if (!ok[g]) continue;
                const int rl = rl0 + g * RPT;
                const int64_t e = (r0 + half * EH + rl) * ld + ecol;
                TA v[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) v[w] = (TA)tile[rl * TS + 4 * ecv + w];
                TO o[4];
                if constexpr (EPI == EPI_NONE) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) o[w] = (TO)v[w];
                } else if constexpr (GRADLIKE) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        if constexpr (EPI == EPI_GRAD)
                            o[w] = (TO)((TA)-2 * ((xv[g][w] - av[g][w] * (TA)vv[w]) - v[w]));
                        else
                            o[w] = (TO)((TA)-2 * ((TA)xs[g][w] - v[w]));
                    }
                    if (fuse) {
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            const double gg = (double)o[w];
                            dsum[0][w] += gg * gg;
                            dsum[1][w] += wgt[g] * gg * gg;
                            dsum[2][w] += wgt[g] * (double)gp[g][w] * gg;
                            dsum[3][w] += (double)pp[g][w] * gg;
                        }
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < 4; ++w) o[w] = (TO)(av[g][w] * (TA)vv[w] + v[w]);
                }
                store4<TO>(out + e, o);
            }
        }
    }

    if constexpr (GRADLIKE) {
        if (fuse) {
            // the RPT lanes of a column vector meet in LDS; fixed order
            __syncthreads();
            double *red = reinterpret_cast<double *>(smem);   // [RPT][4][BC]
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int w = 0; w < 4; ++w) red[(erow * 4 + p) * BC + 4 * ecv + w] = dsum[p][w];
            __syncthreads();
            for (int e2 = tid; e2 < 4 * BC; e2 += kThreads) {
                const int p = e2 / BC, cc = e2 - (e2 / BC) * BC;
                const int col = c0 + cc;
                if (col >= ld) continue;
                double sum = 0.0;
                for (int g = 0; g < RPT; ++g) sum += red[(g * 4 + p) * BC + cc];
                gd.partials[((int64_t)p * nrb + rb) * ld + col] = sum;
            }
        }
    }
}

// --------------------------------------------- TRMM with R' resident in LDS
// C D + C R' (Eq. 13) on FP32 matrix cores for ld = 16 NB: R' is strictly
// upper triangular, so its 16 x 16 blocks on and above the diagonal fit in
// LDS (136 blocks, 148 KB at NB = 16).  One workgroup of eight waves per CU
// loads them once; each wave then streams its own 16-row strips of C from
// HBM straight into matrix-core operands (no LDS staging of C, no barriers)
// and forms the full output width, so C is read once and the zero blocks
// below the diagonal are never multiplied.  Inside an instruction the k
// order is permuted so that a lane's four k come from one 16-byte load: in
// k block kb, step e, lane group g takes k = 16 kb + 4 g + e, and R' supplies
// the same k.  Stored block (kb, jb), kb <= jb, keeps element (r, c) at word
// (r / 4) * 68 + 4 c + r % 4, so a lane's four k of one column are one
// aligned 16-byte LDS read.
constexpr int kTriWaves = 8;
constexpr int kTriStride = 68;
constexpr int kTriBlock = 4 * kTriStride;
constexpr int kTriGrid = 256;

__host__ __device__ constexpr int tri_index(int NB, int kb, int jb) {
    return kb * NB - kb * (kb - 1) / 2 + (jb - kb);
}

// Four consecutive elements of C as raw 16-byte vectors (one for FP32, two
// for FP64), converted to FP32 only when used, so that a prefetch does not
// wait for its own load.
template <typename TA> struct Raw4 {
    static constexpr int NV = sizeof(TA) == 8 ? 2 : 1;
    typename Vec16<TA>::type v[NV];
    __device__ void fetch(const TA *p) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = *reinterpret_cast<const typename Vec16<TA>::type *>(p + 4 / NV * i);
    }
    __device__ void to_float(float (&a)[4]) const {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = (float)v[e / (4 / NV)][e % (4 / NV)];
    }
};

template <typename TA, int NB>
__global__ __launch_bounds__(kTriWaves * 64) void trmm_lds_kernel(
    int64_t n, int ld, const TA *__restrict__ A, const float *__restrict__ W,
    const double *__restrict__ d, TA *__restrict__ out, int64_t nstrips) {
    constexpr int NBLK = NB * (NB + 1) / 2;
    using Acc = Mfma<float>::acc_t;
    __shared__ __align__(16) float Wl[NBLK * kTriBlock];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = lane & 15, g = lane >> 4;

    for (int idx = tid; idx < NBLK * 64; idx += kTriWaves * 64) {
        const int blk = idx >> 6, q = idx & 63;
        int kb = 0, b = blk;
        while (b >= NB - kb) {
            b -= NB - kb;
            ++kb;
        }
        const int jb = kb + b, rr = q >> 2, cq = q & 3;
        const vf4 x = *reinterpret_cast<const vf4 *>(W + (int64_t)(kb * 16 + rr) * ld + jb * 16 + 4 * cq);
        float *dst = Wl + blk * kTriBlock + (rr >> 2) * kTriStride + 16 * cq + (rr & 3);
#pragma unroll
        for (int t = 0; t < 4; ++t) dst[4 * t] = x[t];
    }
    __syncthreads();

    // balanced contiguous strips: workgroup, then wave (waves w and w + 4
    // share a SIMD, so the extra strips go to waves 0, 1, 2, ... first)
    const int64_t s0 = (int64_t)blockIdx.x * nstrips / gridDim.x;
    const int64_t s1 = (int64_t)(blockIdx.x + 1) * nstrips / gridDim.x;
    const int64_t cnt = s1 - s0, base = cnt / kTriWaves, rem = cnt % kTriWaves;
    const int64_t my0 = s0 + wave * base + (wave < rem ? wave : rem);
    const int64_t my1 = my0 + base + (wave < rem ? 1 : 0);

    // C of k block 0 of the first strip; each k block prefetches the next
    // (the last one the next strip's first), rows clamped to n - 1
    auto a_row = [&](int64_t st) {
        const int64_t r = st * 16 + j;
        return A + (r < n ? r : n - 1) * ld + 4 * g;
    };
    Raw4<TA> an;
    if (my0 < my1) an.fetch(a_row(my0));
    for (int64_t st = my0; st < my1; ++st) {
        const int64_t row0 = st * 16;
        const TA *Ar = a_row(st);
        const TA *An = a_row(st + 1 < my1 ? st + 1 : st);
        // out = C D + C R': this lane holds rows row0 + 4 g + r of column
        // 16 jb + j.  Column block jb is complete after k block jb (R' is
        // upper triangular), so it is written right then, while the C it
        // re-reads for the FP64 term C D was just loaded by this wave.  A
        // full strip needs no row mask; the last, partial one clamps its
        // loads to row n - 1 and masks its stores.
        auto strip = [&](auto fullc) {
        constexpr bool FULL = decltype(fullc)::value != 0;
        int64_t rowc[4];
        bool ok[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + 4 * g + r;
            ok[r] = FULL || row < n;
            rowc[r] = ok[r] ? row : n - 1;
        }
        auto finish = [&](int jb, const Acc &c) {
            const int col = jb * 16 + j;
            const TA dc = (TA)d[col];
            TA av[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = A[rowc[r] * ld + col];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (FULL || ok[r]) out[rowc[r] * ld + col] = av[r] * dc + (TA)c[r];
        };
        Acc acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            float a[4];
            an.to_float(a);
            an.fetch(kb + 1 < NB ? Ar + (kb + 1) * 16 : An);
            // the prefetch is issued before this block's work, not sunk into it
            __builtin_amdgcn_sched_barrier(0);
            // column blocks in two halves: only half of R's operands live
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                constexpr int HB = NB / 2;
                float bw[HB][4];
#pragma unroll
                for (int q = 0; q < HB; ++q) {
                    const int jb = h * HB + q;
                    if (jb < kb) continue;
                    const vf4 x = *reinterpret_cast<const vf4 *>(Wl + tri_index(NB, kb, jb) * kTriBlock +
                                                                 g * kTriStride + 4 * j);
                    bw[q][0] = x[0]; bw[q][1] = x[1]; bw[q][2] = x[2]; bw[q][3] = x[3];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int q = 0; q < HB; ++q) {
                        const int jb = h * HB + q;
                        if (jb >= kb) acc[jb] = Mfma<float>::op(a[e], bw[q][e], acc[jb]);
                    }
            }
            finish(kb, acc[kb]);
            // one scheduling region per k block: the LDS reads of a block
            // interleave with its own matrix-core work and are not hoisted
            // across blocks (which would exceed the register budget)
            __builtin_amdgcn_sched_barrier(0);
        }
        };
        if (row0 + 16 <= n) strip(IntC<1>{});
        else strip(IntC<0>{});
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

size_t gram_partials_bytes(int64_t n, int m, bool symmetric, size_t ws_bytes) {
    int BM, T, ns;
    gram_shape(n, m, symmetric, BM, T, ns, ws_bytes);
    return (size_t)ns * m * m * sizeof(double);
}

// The launch of a Gram: its tiles (gram_tg, gram_ntiles) times the split
// count gram_shape gives for that many tiles.
static void gram_plan(int T, int BM, bool symmetric, int nsplit, BatchCols bc, int &tg, int &ntiles,
                      int &nwork, int &grid) {
    tg = gram_tg(BM, bc.ldg);
    ntiles = gram_ntiles(T, symmetric, tg);
    nwork = ntiles * nsplit;
    grid = (nwork + 7) / 8 * 8;
}

size_t gram_workspace(int64_t n, int m, int ldg) {
    // the largest split count of the full launches and, for a batch, of the
    // launches over its diagonal tile blocks (more splits for fewer tiles)
    int BM, T, ns, most = 0;
    for (int l : {0, ldg})
        for (bool sym : {false, true}) {
            gram_shape(n, m, sym, BM, T, ns, 0, l);
            most = std::max(most, ns);
        }
    return (size_t)most * m * m * sizeof(double);
}

template <typename TA, typename TM>
void gram(hipStream_t s, int64_t n, int m, const TA *A, const TA *B,
          const double *h, bool zero_diag, bool symmetric, double *partials,
          double *out, bool reduce, TM *xshift, TM *wpad, size_t ws_bytes, BatchCols bc) {
    const int ld = leading_dim(m);
    int BM, T, nsplit;
    gram_shape(n, m, symmetric, BM, T, nsplit, ws_bytes, bc.ldg);
    int tg, ntiles, nwork, grid;
    gram_plan(T, BM, symmetric, nsplit, bc, tg, ntiles, nwork, grid);
    constexpr int KT = stage_rows<TM>();
    const int64_t rows = ((n + nsplit - 1) / nsplit + KT - 1) / KT * KT;
#define TM_GRAM(BMV, SH)                                                            \
    hipLaunchKernelGGL((gram_kernel<TA, TM, BMV, SH, false, TA, gram_threads<TA, TM, SH, false, TA>()>), \
                       dim3(grid), dim3(gram_threads<TA, TM, SH, false, TA>()), 0, s,         \
                       n, m, ld, A, B, h, T, ntiles, symmetric, rows, partials, GramUpd<TA, TA>{}, \
                       xshift, tg, nwork)
    if (BM == 128) {
        if (h) TM_GRAM(128, true); else TM_GRAM(128, false);
    } else {
        if (h) TM_GRAM(64, true); else TM_GRAM(64, false);
    }
#undef TM_GRAM
    TM_HIP(hipGetLastError());
    if (!reduce) return;
    const int64_t total = (int64_t)m * m;
    float *padf = nullptr;
    double *padd = nullptr;
    if (wpad) {
        if constexpr (sizeof(TM) == 4) padf = reinterpret_cast<float *>(wpad);
        else padd = reinterpret_cast<double *>(wpad);
    }
    const int64_t cover = wpad ? (int64_t)ld * ld : total;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((cover + 63) / 64)), dim3(256), 0,
                       s, m, nsplit, symmetric, zero_diag, partials, out, ld, padf, padd, bc);
    TM_HIP(hipGetLastError());
}

template <typename TA, typename TM, typename TP>
void gram_update(hipStream_t s, int64_t n, int m, const TA *C, const TP *P, const CgState *st,
                 TA *Cn, double *partials, double *out, BatchCols bc) {
    const int ld = leading_dim(m);
    int BM, T, nsplit;
    gram_shape(n, m, true, BM, T, nsplit, 0, bc.ldg);
    int tg, ntiles, nwork, grid;
    gram_plan(T, BM, true, nsplit, bc, tg, ntiles, nwork, grid);
    constexpr int KT = stage_rows<TM>();
    const int64_t rows = ((n + nsplit - 1) / nsplit + KT - 1) / KT * KT;
    GramUpd<TA, TP> up;
    up.P = P;
    up.st = st;
    up.Cn = Cn;
    up.ldg = bc.ldg;
    if (BM == 128)
        hipLaunchKernelGGL((gram_kernel<TA, TM, 128, false, true, TP, gram_threads<TA, TM, false, true, TP>()>),
                           dim3(grid), dim3(gram_threads<TA, TM, false, true, TP>()), 0, s,
                           n, m, ld, C, C, nullptr, T, ntiles, true, rows, partials, up, nullptr, tg,
                           nwork);
    else
        hipLaunchKernelGGL((gram_kernel<TA, TM, 64, false, true, TP, gram_threads<TA, TM, false, true, TP>()>),
                           dim3(grid), dim3(gram_threads<TA, TM, false, true, TP>()), 0, s,
                           n, m, ld, C, C, nullptr, T, ntiles, true, rows, partials, up, nullptr, tg,
                           nwork);
    TM_HIP(hipGetLastError());
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 63) / 64)), dim3(256), 0,
                       s, m, nsplit, true, false, partials, out, ld, nullptr, nullptr, bc);
    TM_HIP(hipGetLastError());
}

template <typename TA>
void gram_bf16x3(hipStream_t s, int64_t n, int m, const TA *A, const TA *B, const double *h,
                 bool zero_diag, double *partials, double *out, bool reduce, float *wpad,
                 size_t ws_bytes) {
    const int ld = leading_dim(m);
    int BM, T, nsplit;
    gram_shape(n, m, false, BM, T, nsplit, ws_bytes);
    const int ntiles = T * T;
    const int KT = 8 * (kThreads / (BM / 2));
    const int64_t rows = ((n + nsplit - 1) / nsplit + KT - 1) / KT * KT;
    const int grid = ntiles * nsplit;   // multiple of 8
#define TM_GRAM16(BMV, SH)                                                                 \
    hipLaunchKernelGGL((gram_bf16x3_kernel<TA, BMV, SH>), dim3(grid), dim3(kThreads), 0, s, n, m, \
                       ld, A, B, h, T, ntiles, rows, partials)
    if (BM == 128) {
        if (h) TM_GRAM16(128, true); else TM_GRAM16(128, false);
    } else {
        if (h) TM_GRAM16(64, true); else TM_GRAM16(64, false);
    }
#undef TM_GRAM16
    TM_HIP(hipGetLastError());
    if (!reduce) return;
    const int64_t total = (int64_t)m * m;
    float *padf = nullptr;
    if (wpad) padf = wpad;
    const int64_t cover = wpad ? (int64_t)ld * ld : total;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((cover + 63) / 64)), dim3(256), 0,
                       s, m, nsplit, false, zero_diag, partials, out, ld, padf, nullptr, BatchCols());
    TM_HIP(hipGetLastError());
}

template <typename TA, typename TM, typename TO>
int rot(hipStream_t s, int64_t n, int m, const TA *A, const TM *Wpad, int epi,
        const TA *X, const double *vec, TO *out, const TO *Gp, const TO *Pp,
        const double *M, double *partials, const TM *Xs, int wg) {
    TM_REQUIRE(epi != EPI_GRADX || Xs != nullptr, TM_EINVAL, "EPI_GRADX needs X'");
    TM_REQUIRE(wg == 0 || (wg > 0 && wg % 16 == 0), TM_EINVAL, "diagonal blocks of W: 16-column multiples");
    const int ld = leading_dim(m);
    if constexpr (std::is_same<TM, float>::value && std::is_same<TA, TO>::value) {
        if (ld == 256 && epi == EPI_TRMM && wg == 0) {
            const int64_t nstrips = (n + 15) / 16;
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(kTriGrid, nstrips));
            hipLaunchKernelGGL((trmm_lds_kernel<TA, 16>), dim3(grid), dim3(kTriWaves * 64), 0, s, n, ld, A,
                               Wpad, vec, out, nstrips);
            TM_HIP(hipGetLastError());
            return grid;
        }
    }
    const int B = ld >= 256 ? 128 : 64;
    // row tile: 64 rows give about twice the workgroups of 128 (7 rounds of
    // 512 at N = 110592 instead of 3.4, so less idle tail); measured faster
    // for every variant, the refinement gradient included
    const int BR = 64;
    const int nrb = (int)((n + BR - 1) / BR);
    const int ncb = (ld + B - 1) / B;
    int grid = nrb * ncb;
    grid = (grid + 7) / 8 * 8;
    GradDots<TO> gd;
    gd.Gp = Gp;
    gd.Pp = Pp;
    gd.M = M;
    gd.partials = (epi == EPI_GRAD || epi == EPI_GRADX) ? partials : nullptr;
    gd.Xs = Xs;
#define TM_ROT(E, BRV, BCV)                                                                  \
    hipLaunchKernelGGL((rot_kernel<TA, TM, TO, E, BRV, BCV>), dim3(grid), dim3(kThreads),   \
                       0, s, n, m, ld, A, Wpad, X, vec, out, nrb, ncb, gd, wg)
    if (B == 128) {
        if (epi == EPI_NONE) TM_ROT(EPI_NONE, 64, 128);
        else if (epi == EPI_GRAD) TM_ROT(EPI_GRAD, 64, 128);
        else if (epi == EPI_GRADX) TM_ROT(EPI_GRADX, 64, 128);
        else TM_ROT(EPI_TRMM, 64, 128);
    } else {
        if (epi == EPI_NONE) TM_ROT(EPI_NONE, 64, 64);
        else if (epi == EPI_GRAD) TM_ROT(EPI_GRAD, 64, 64);
        else if (epi == EPI_GRADX) TM_ROT(EPI_GRADX, 64, 64);
        else TM_ROT(EPI_TRMM, 64, 64);
    }
#undef TM_ROT
    TM_HIP(hipGetLastError());
    return nrb;
}

size_t rot_partials_workspace(int64_t n, int m) {
    // the smallest row tile rot() launches
    const int ld = leading_dim(m);
    return (size_t)4 * ((n + 63) / 64) * ld * sizeof(double);
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

template void gram<double, double>(hipStream_t, int64_t, int, const double *, const double *, const double *, bool, bool, double *, double *, bool, double *, double *, size_t, BatchCols);
template void gram<float, float>(hipStream_t, int64_t, int, const float *, const float *, const double *, bool, bool, double *, double *, bool, float *, float *, size_t, BatchCols);
template void gram<double, float>(hipStream_t, int64_t, int, const double *, const double *, const double *, bool, bool, double *, double *, bool, float *, float *, size_t, BatchCols);
template void gram_update<double, double, double>(hipStream_t, int64_t, int, const double *, const double *, const CgState *, double *, double *, double *, BatchCols);
template void gram_update<double, double, float>(hipStream_t, int64_t, int, const double *, const float *, const CgState *, double *, double *, double *, BatchCols);
template void gram_update<float, float, float>(hipStream_t, int64_t, int, const float *, const float *, const CgState *, float *, double *, double *, BatchCols);
template void gram_bf16x3<float>(hipStream_t, int64_t, int, const float *, const float *, const double *, bool, double *, double *, bool, float *, size_t);
template void gram_bf16x3<double>(hipStream_t, int64_t, int, const double *, const double *, const double *, bool, double *, double *, bool, float *, size_t);
template int rot<double, double, double>(hipStream_t, int64_t, int, const double *, const double *, int, const double *, const double *, double *, const double *, const double *, const double *, double *, const double *, int);
template int rot<float, float, float>(hipStream_t, int64_t, int, const float *, const float *, int, const float *, const double *, float *, const float *, const float *, const double *, double *, const float *, int);
template int rot<double, float, float>(hipStream_t, int64_t, int, const double *, const float *, int, const double *, const double *, float *, const float *, const float *, const double *, double *, const float *, int);
template int rot<double, float, double>(hipStream_t, int64_t, int, const double *, const float *, int, const double *, const double *, double *, const double *, const double *, const double *, double *, const float *, int);
template int rot<double, double, float>(hipStream_t, int64_t, int, const double *, const double *, int, const double *, const double *, float *, const float *, const float *, const double *, double *, const double *, int);
template void pad_matrix<double>(hipStream_t, int, const double *, bool, double *, double *);
template void pad_matrix<float>(hipStream_t, int, const double *, bool, float *, double *);

}  // namespace tmin
