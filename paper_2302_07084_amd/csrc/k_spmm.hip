// Sparse x dense products on gfx950.
//
// spmm: Y = A X with A a CSR matrix with values (the sparsified NetMF matrix
// of the randomized SVD, Algorithm "Fast Randomized SVD") and X a row-major
// n x k dense block.  graph_spmm: out = a Z + b D^-1 A Z + c1 E1 + c2 E2
// (+ acc += cacc out) with A the value-free graph adjacency, the building
// block of the Chebyshev recurrence of section 4.3.
//
// Both are gather-bound: every nonzero pulls one k-wide row of the dense
// operand.  One wave owns one output row.  Its 64 lanes read the row's column
// ids and values in coalesced batches of 64 and broadcast them lane to lane.
// The k columns are split into a main part, k_main = a multiple of L * N
// columns with L the largest power of two (<= 64) such that L * N <= k, and a
// tail of the remaining k - k_main < L * N columns.  Each lane moves one
// 16-byte vector (N = 4 floats, 2 doubles or 8 bf16) per gathered row: the
// main part runs G = 64 / L nonzeros per load instruction on L lanes each,
// the tail (at most 16 columns, 32 for BF16) runs 16 nonzeros per
// instruction on 4 lanes each (8 nonzeros on 8 lanes for FP64), so no lane sits idle for most of a wide row (k = 138 floats would
// otherwise take one 64-lane load per nonzero with 29 lanes idle).  Tails
// wider than 4 vectors are handled by a second launch on the tail columns.
// Every load is a whole 16-byte vector inside the row's ld span: columns from
// k up to the next multiple of N are read and their sums discarded.
// Each lane group accumulates its nonzeros in row order (so U, the number of
// loads in flight, does not change the result); groups are combined by a
// butterfly over lane offsets L, 2L, ... before the epilogue writes the row.
// U is picked per matrix and width by timing (pick_variant).
#include "common.hpp"

namespace lne {

namespace {

template <class T> struct Vec;
template <> struct Vec<double> { static constexpr int N = 2; using A = double; };
template <> struct Vec<float> { static constexpr int N = 4; using A = float; };
template <> struct Vec<__bf16> { static constexpr int N = 8; using A = float; };

// one 16-byte vector of N elements, widened to the accumulation type
template <class XT, class AT, int N>
__device__ __forceinline__ void load_vec(const XT *__restrict__ p, AT v[N]) {
    static_assert(sizeof(XT) * N == 16, "16-byte vectors");
    const uint4 raw = *reinterpret_cast<const uint4 *>(p);
    const XT *e = reinterpret_cast<const XT *>(&raw);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = (AT)e[i];
}

template <class OT, class AT, int N>
__device__ __forceinline__ void store_row(OT *__restrict__ p, int c0, int k, const AT v[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (c0 + i < k) p[i] = (OT)v[i];
}

// Loads of the streamed sparse structure, optionally marked non-temporal so
// that the stream does not displace gathered rows from the caches.
template <bool NT, class T> __device__ __forceinline__ T stream_load(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// One batch of up to 64 nonzeros held one per lane (column cj, value vj):
// lane group grp (L lanes) adds v_t X[j_t, c0 : c0 + N) for its nonzeros t =
// grp, grp + G, ... in order.  `on` switches the lane's loads off (tail lanes
// past k); every lane takes part in the shuffles.
template <int L, int U, bool VALS, class XT, class AT>
__device__ __forceinline__ void gather_batch(const XT *__restrict__ X, int64_t ldx, int c0,
                                             bool on, int32_t cj, AT vj, int cnt, int grp,
                                             AT acc[Vec<XT>::N]) {
    constexpr int N = Vec<XT>::N;
    constexpr int G = 64 / L;
    for (int t0 = 0; t0 < cnt; t0 += U * G) {
        int32_t j[U];
        AT v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int t = t0 + grp + q * G;
            j[q] = __shfl(cj, t & 63);
            if constexpr (VALS) {
                const AT vq = __shfl(vj, t & 63);
                v[q] = t < cnt ? vq : (AT)0;
            }
        }
        AT x[U][N];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (on && t0 + grp + q * G < cnt)
                load_vec<XT, AT, N>(X + (int64_t)j[q] * ldx + c0, x[q]);
            else
#pragma unroll
                for (int i = 0; i < N; ++i) x[q][i] = 0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if constexpr (VALS) acc[i] += v[q] * x[q][i];
                else acc[i] += x[q][i];
            }
    }
}

template <int L, class AT, int N> __device__ __forceinline__ void fold_groups(AT acc[N]) {
#pragma unroll
    for (int off = L; off < 64; off <<= 1)
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
}

// lanes per gathered tail row: 16 columns for FP32 and FP64, 32 for BF16
__host__ __device__ constexpr int tail_lanes(int N) { return N == 2 ? 8 : 4; }

// L = lanes per gathered main-part vector row (power of two, <= 64); TL = the
// tail is present (tail_lanes(N) lanes per nonzero); U = loop steps in flight;
// NT = non-temporal structure loads; VT value type; XT operand type; OT
// output type.  Columns [0, k_main) are the main part, [k_main, k) the tail.
template <int L, bool TL, int U, bool NT, class VT, class XT, class OT>
__global__ void __launch_bounds__(256)
k_spmm(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
       const VT *__restrict__ val, int64_t n_rows, const XT *__restrict__ X, int64_t ldx,
       OT *__restrict__ Y, int64_t ldy, int k_main, int k) {
    constexpr int N = Vec<XT>::N;
    using AT = typename Vec<XT>::A;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n_rows) return;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, lc = lane % L;
    constexpr int TLn = tail_lanes(N);
    const int grpt = lane / TLn, lct = lane % TLn;
    const int ct = k_main + lct * N;
    const int64_t beg = rp[row], end = rp[row + 1];
    for (int cb = 0;; cb += L * N) {
        const bool main = cb < k_main;
        const bool tail = TL && cb + L * N >= k_main;   // with the last main chunk
        const int c0 = cb + lc * N;
        AT acc[N], acct[N];
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = acct[i] = 0;
        for (int64_t b0 = beg; b0 < end; b0 += 64) {
            const int64_t idx = b0 + lane;
            const int32_t cj = idx < end ? stream_load<NT>(col + idx) : 0;
            const AT vj = idx < end ? (AT)stream_load<NT>(val + idx) : (AT)0;
            const int cnt = (int)min((int64_t)64, end - b0);
            if (main) gather_batch<L, U, true, XT, AT>(X, ldx, c0, true, cj, vj, cnt, grp, acc);
            if (tail)
                gather_batch<TLn, U, true, XT, AT>(X, ldx, ct, ct < k, cj, vj, cnt, grpt,
                                                          acct);
        }
        if (main) {
            fold_groups<L, AT, N>(acc);
            if (grp == 0) store_row<OT, AT, N>(Y + row * ldy + c0, c0, k, acc);
        }
        if (tail) {
            fold_groups<TLn, AT, N>(acct);
            if (grpt == 0 && ct < k) store_row<OT, AT, N>(Y + row * ldy + ct, ct, k, acct);
        }
        if (cb + L * N >= k_main) break;
    }
}

// out = a z + b (inv acc) + c1 e1 + c2 e2 at columns [c0, c0 + N) of a row;
// accum += cacc out when accum is given, or with ainit accum = cinit e1 +
// cacc out (accum not read: the first term of a sum started in the same pass).
template <class T, int N>
__device__ __forceinline__ void graph_epilogue(int64_t o, int c0, int k, const T acc[N], T inv,
                                               const T *__restrict__ Z, T *__restrict__ out, T a,
                                               T b, const T *__restrict__ E1, T c1,
                                               const T *__restrict__ E2, T c2,
                                               T *__restrict__ accum, T cacc, int ainit,
                                               T cinit) {
    T z[N], e1[N], e2[N];
    load_vec<T, T, N>(Z + o, z);
    if (E1) load_vec<T, T, N>(E1 + o, e1);
    if (E2) load_vec<T, T, N>(E2 + o, e2);
    T r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        r[i] = a * z[i] + b * (inv * acc[i]);
        if (E1) r[i] += c1 * e1[i];
        if (E2) r[i] += c2 * e2[i];
    }
    store_row<T, T, N>(out + o, c0, k, r);
    if (accum) {
        T s[N];
        if (ainit) {
#pragma unroll
            for (int i = 0; i < N; ++i) s[i] = cinit * e1[i];
        } else {
            load_vec<T, T, N>(accum + o, s);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) s[i] += cacc * r[i];
        store_row<T, T, N>(accum + o, c0, k, s);
    }
}

// W: weighted graph, D^-1 A with arc weights wt and d_i = sum_j A_ij (summed
// here from the row's weights).
template <int L, bool TL, int U, bool NT, bool W, class T>
__global__ void __launch_bounds__(256)
k_graph_spmm(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
             const uint32_t *__restrict__ wt, int64_t n_rows,
             const T *__restrict__ Z, int64_t ld, int k_main, int k, T *__restrict__ out, T a,
             T b, const T *__restrict__ E1, T c1, const T *__restrict__ E2, T c2,
             T *__restrict__ accum, T cacc, int ainit, T cinit) {
    constexpr int N = Vec<T>::N;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n_rows) return;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, lc = lane % L;
    constexpr int TLn = tail_lanes(N);
    const int grpt = lane / TLn, lct = lane % TLn;
    const int ct = k_main + lct * N;
    const int64_t beg = rp[row], end = rp[row + 1];
    T inv = end > beg ? (T)1 / (T)(end - beg) : (T)0;
    for (int cb = 0;; cb += L * N) {
        const bool main = cb < k_main;
        const bool tail = TL && cb + L * N >= k_main;
        const int c0 = cb + lc * N;
        T acc[N], acct[N];
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = acct[i] = 0;
        uint64_t wsum = 0;
        for (int64_t b0 = beg; b0 < end; b0 += 64) {
            const int64_t idx = b0 + lane;
            const int32_t cj = idx < end ? stream_load<NT>(col + idx) : 0;
            const uint32_t wj = (W && idx < end) ? stream_load<NT>(wt + idx) : 0u;
            wsum += wj;
            const int cnt = (int)min((int64_t)64, end - b0);
            if (main) gather_batch<L, U, W, T, T>(Z, ld, c0, true, cj, (T)wj, cnt, grp, acc);
            if (tail)
                gather_batch<TLn, U, W, T, T>(Z, ld, ct, ct < k, cj, (T)wj, cnt, grpt, acct);
        }
        if (W) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
            inv = wsum ? (T)1 / (T)wsum : (T)0;
        }
        if (main) {
            fold_groups<L, T, N>(acc);
            if (grp == 0)
                graph_epilogue<T, N>(row * ld + c0, c0, k, acc, inv, Z, out, a, b, E1, c1, E2, c2,
                                     accum, cacc, ainit, cinit);
        }
        if (tail) {
            fold_groups<TLn, T, N>(acct);
            if (grpt == 0 && ct < k)
                graph_epilogue<T, N>(row * ld + ct, ct, k, acct, inv, Z, out, a, b, E1, c1, E2,
                                     c2, accum, cacc, ainit, cinit);
        }
        if (cb + L * N >= k_main) break;
    }
}

// Y = A Omega with a sparse-sign Omega: one wave per row; the wave's k-wide
// row accumulator sits in LDS, every lane takes one nonzero (column j,
// value v) of a 64-entry batch, loads Omega's row j (kSparseOmega signed
// columns, 16 bytes) and adds +-v to those columns with LDS atomics.
template <class VT, class AT, class OT>
__global__ void __launch_bounds__(256)
k_spmm_sparse_omega(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                    const VT *__restrict__ val, int64_t n_rows, const int16_t *__restrict__ om,
                    OT *__restrict__ Y, int64_t ldy, int k) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    AT *acc = reinterpret_cast<AT *>(lds_raw) + (threadIdx.x >> 6) * k;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    for (int c = lane; c < k; c += 64) acc[c] = (AT)0;
    __builtin_amdgcn_wave_barrier();
    if (row >= n_rows) return;
    const int64_t beg = rp[row], end = rp[row + 1];
    for (int64_t b0 = beg; b0 < end; b0 += 64) {
        const int64_t idx = b0 + lane;
        if (idx < end) {
            const int32_t j = col[idx];
            const AT v = (AT)val[idx];
            const uint4 raw = *reinterpret_cast<const uint4 *>(om + (int64_t)j * kSparseOmega);
            const int16_t *e = reinterpret_cast<const int16_t *>(&raw);
#pragma unroll
            for (int t = 0; t < kSparseOmega; ++t) {
                const int c = e[t] > 0 ? e[t] - 1 : -e[t] - 1;
                if ((unsigned)c < (unsigned)k) atomicAdd(&acc[c], e[t] > 0 ? v : -v);
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int c = lane; c < k; c += 64) Y[row * ldy + c] = (OT)acc[c];
}

// Streaming element-wise kernels over n x k row blocks: each wave walks rows
// (grid-stride), its lanes across the row's columns, so no per-element index
// division.
template <class XT, class YT>
__global__ void k_scale(const XT *__restrict__ x, int64_t ldx, YT *__restrict__ y, int64_t ldy,
                        int64_t n, int k, double alpha) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = w0; i < n; i += nw)
        for (int c = lane; c < k; c += 64) y[i * ldy + c] = (YT)(alpha * (double)x[i * ldx + c]);
}

template <class T>
__global__ void k_axpby(const T *__restrict__ x, const T *__restrict__ y, T *__restrict__ out,
                        int64_t n, int k, int64_t ld, T a, T b) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = w0; i < n; i += nw)
        for (int c = lane; c < k; c += 64) {
            const int64_t o = i * ld + c;
            out[o] = a * x[o] + b * y[o];
        }
}

// Blocks of the row-walking kernels: 4 waves each, one row per wave, at most
// 64 blocks per CU (the loop covers the remaining rows).
inline unsigned rows_grid(int64_t n) {
    const int64_t blocks = ceil_div(n, 4);   // 4 waves (256 threads) per block
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
}

// launch shapes: unroll depth 4 or 8, structure loads normal or non-temporal
constexpr int kSpmmVariants = 4;

// Column split of a k-wide operand with N-element vectors: L lanes per
// main-part vector row, main part [0, k_main), tail [k_main, k).
struct ColSplit {
    int L, k_main, tail;
};

ColSplit split_cols(int k, int N) {
    if (k < N) return {1, 0, k};
    int L = 1;
    while (L < 64 && 2 * L * N <= k) L <<= 1;
    const int k_main = k - k % (L * N);
    return {L, k_main, k - k_main};
}

// Runs fn(L-tag, tail-flag, k_main, k_launch) for each launch covering the
// columns [0, k) (one launch unless the tail is wider than tail_lanes vectors,
// whose columns then take launches of their own) with the operand pointers
// advanced by col0 columns.
template <class F> void for_each_launch(int k, int N, F &&fn) {
    int col0 = 0;
    while (col0 < k) {
        const ColSplit s = split_cols(k - col0, N);
        const bool fuse = s.tail > 0 && s.tail <= tail_lanes(N) * N;
        const int kk = (fuse || s.tail == 0) ? k - col0 : s.k_main;
        fn(col0, s.L, fuse, s.k_main, kk);
        col0 += kk;
    }
}

template <int L, bool TL, class VT, class XT, class OT>
void spmm_launch(lne_ctx *ctx, const lne_csr *A, const XT *X, int64_t ldx, OT *Y, int64_t ldy,
                 int k_main, int k, int variant) {
    const unsigned grid = grid_of(A->n_rows * 64, 256);
    const VT *val = (const VT *)A->val;
    Launch Lc(ctx, "spmm");
#define LNE_SV(UU, NTT)                                                                    \
    k_spmm<L, TL, UU, NTT, VT, XT, OT><<<grid, 256, 0, ctx->stream>>>(                    \
        A->row_ptr, A->col, val, A->n_rows, X, ldx, Y, ldy, k_main, k)
    switch (variant) {
        case 1: LNE_SV(8, false); break;
        case 2: LNE_SV(4, true); break;
        case 3: LNE_SV(8, true); break;
        default: LNE_SV(4, false); break;
    }
#undef LNE_SV
}

template <bool TL, class VT, class XT, class OT>
void spmm_launch_l(int L, lne_ctx *ctx, const lne_csr *A, const XT *X, int64_t ldx, OT *Y,
                   int64_t ldy, int k_main, int k, int v) {
    switch (L) {
#define LNE_SL(LL)                                                                          \
    case LL: spmm_launch<LL, TL, VT, XT, OT>(ctx, A, X, ldx, Y, ldy, k_main, k, v); break;
        LNE_SL(1) LNE_SL(2) LNE_SL(4) LNE_SL(8) LNE_SL(16) LNE_SL(32)
        default: spmm_launch<64, TL, VT, XT, OT>(ctx, A, X, ldx, Y, ldy, k_main, k, v);
#undef LNE_SL
    }
}

template <class VT, class XT, class OT>
lne_status spmm_t(lne_ctx *ctx, const lne_csr *A, const XT *X, int64_t ldx, OT *Y,
                  int64_t ldy, int k, int dtype) {
    const int N = Vec<XT>::N;
    const bool aligned = ((uintptr_t)X % 16 == 0) && (ldx % N == 0);
    if (!aligned) return fail(ctx, LNE_EINVAL, "spmm: X must be 16-byte aligned with ld %% %d == 0", N);
    auto run = [&](int v) -> lne_status {
        for_each_launch(k, N, [&](int c0, int L, bool tl, int k_main, int kk) {
            if (tl) spmm_launch_l<true, VT, XT, OT>(L, ctx, A, X + c0, ldx, Y + c0, ldy, k_main, kk, v);
            else spmm_launch_l<false, VT, XT, OT>(L, ctx, A, X + c0, ldx, Y + c0, ldy, k_main, kk, v);
        });
        return check_launch(ctx, "spmm");
    };
    int v = 0;
    const std::string key = shape_key("spmm", A->n_rows, A->nnz, k, dtype);
    LNE_TRY(pick_variant(ctx, key, kSpmmVariants, run, &v));
    return run(v);
}

template <int L, bool TL, class T>
void gspmm_launch(lne_ctx *ctx, const Graph *g, const T *Z, T *out, int64_t ld, int k_main,
                  int k, double a, double b, const T *E1, double c1, const T *E2, double c2,
                  T *acc, double cacc, int ainit, double cinit, int variant) {
    const unsigned grid = grid_of(g->n * 64, 256);
    Launch Lc(ctx, "graph_spmm");
#define LNE_GS(UU, NTT, WW)                                                                \
    k_graph_spmm<L, TL, UU, NTT, WW, T><<<grid, 256, 0, ctx->stream>>>(                   \
        g->row_ptr, g->col, g->weight, g->n, Z, ld, k_main, k, out, (T)a, (T)b, E1, (T)c1,  \
        E2, (T)c2, acc, (T)cacc, ainit, (T)cinit)
#define LNE_GV(WW)                                                                         \
    switch (variant) {                                                                     \
        case 1: LNE_GS(8, false, WW); break;                                               \
        case 2: LNE_GS(4, true, WW); break;                                                \
        case 3: LNE_GS(8, true, WW); break;                                                \
        default: LNE_GS(4, false, WW); break;                                              \
    }
    if (g->weight) {
        LNE_GV(true)
    } else {
        LNE_GV(false)
    }
#undef LNE_GV
#undef LNE_GS
}

template <bool TL, class T>
void gspmm_launch_l(int L, lne_ctx *ctx, const Graph *g, const T *Z, T *out, int64_t ld,
                    int k_main, int k, double a, double b, const T *E1, double c1, const T *E2,
                    double c2, T *acc, double cacc, int ainit, double cinit, int v) {
    switch (L) {
#define LNE_GL(LL)                                                                            \
    case LL:                                                                                  \
        gspmm_launch<LL, TL, T>(ctx, g, Z, out, ld, k_main, k, a, b, E1, c1, E2, c2, acc, cacc, \
                                ainit, cinit, v);                                             \
        break;
        LNE_GL(1) LNE_GL(2) LNE_GL(4) LNE_GL(8) LNE_GL(16) LNE_GL(32)
        default:
            gspmm_launch<64, TL, T>(ctx, g, Z, out, ld, k_main, k, a, b, E1, c1, E2, c2, acc,
                                    cacc, ainit, cinit, v);
#undef LNE_GL
    }
}

template <class T>
lne_status gspmm_t(lne_ctx *ctx, const Graph *g, const T *Z, T *out, int64_t ld, int k,
                   double a, double b, const T *E1, double c1, const T *E2, double c2,
                   T *acc, double cacc, int ainit, double cinit, int dtype) {
    const int N = Vec<T>::N;
    for (const T *q : {Z, (const T *)out, E1, E2, (const T *)acc})
        if ((uintptr_t)q % 16)
            return fail(ctx, LNE_EINVAL, "graph_spmm: operands must be 16-byte aligned");
    if (ld % N) return fail(ctx, LNE_EINVAL, "graph_spmm: ld must be a multiple of %d", N);
    auto at = [](auto *p, int c0) { return p ? p + c0 : p; };
    auto run = [&](int v) -> lne_status {
        for_each_launch(k, N, [&](int c0, int L, bool tl, int k_main, int kk) {
            if (tl)
                gspmm_launch_l<true, T>(L, ctx, g, Z + c0, out + c0, ld, k_main, kk, a, b,
                                        at(E1, c0), c1, at(E2, c0), c2, at(acc, c0), cacc, ainit,
                                        cinit, v);
            else
                gspmm_launch_l<false, T>(L, ctx, g, Z + c0, out + c0, ld, k_main, kk, a, b,
                                         at(E1, c0), c1, at(E2, c0), c2, at(acc, c0), cacc, ainit,
                                         cinit, v);
        });
        return check_launch(ctx, "graph_spmm");
    };
    int v = 0;
    const std::string key = shape_key("graph_spmm", g->n, g->n_arcs, k, dtype);
    // the tuning runs write `out` and add to `acc`: tune only calls without an
    // accumulator, whose output is recomputed by the final run
    if (!acc) LNE_TRY(pick_variant(ctx, key, kSpmmVariants, run, &v));
    else v = tuned_or(ctx, key, 0);
    return run(v);
}

}  // namespace

lne_status spmm(lne_ctx *ctx, const lne_csr *A, const void *X, int64_t ldx, void *Y,
                int64_t ldy, int32_t k, int32_t dtype) {
    lne_status s;
    if (dtype == LNE_F64) {
        if (A->val_type != LNE_F64) return fail(ctx, LNE_EINVAL, "spmm: F64 needs F64 values");
        s = spmm_t<double, double, double>(ctx, A, (const double *)X, ldx, (double *)Y, ldy, k,
                                           dtype);
    } else if (dtype == LNE_F32) {
        if (A->val_type != LNE_F32) return fail(ctx, LNE_EINVAL, "spmm: F32 needs F32 values");
        s = spmm_t<float, float, float>(ctx, A, (const float *)X, ldx, (float *)Y, ldy, k, dtype);
    } else if (dtype == LNE_BF16) {
        if (A->val_type != LNE_F32) return fail(ctx, LNE_EINVAL, "spmm: BF16 needs F32 values");
        s = spmm_t<float, __bf16, __bf16>(ctx, A, (const __bf16 *)X, ldx, (__bf16 *)Y, ldy, k,
                                          dtype);
    } else {
        return fail(ctx, LNE_EINVAL, "spmm: bad dtype");
    }
    return s;
}

lne_status graph_spmm(lne_ctx *ctx, const Graph *g, const void *Z, void *out, int64_t ld,
                      int32_t k, int32_t dtype, double a, double b, const void *E1, double c1,
                      const void *E2, double c2, void *acc, double cacc, bool acc_init,
                      double cinit) {
    if (acc_init && (!acc || !E1))
        return fail(ctx, LNE_EINVAL, "graph_spmm: starting acc from E1 needs both");
    lne_status s;
    if (dtype == LNE_F64)
        s = gspmm_t<double>(ctx, g, (const double *)Z, (double *)out, ld, k, a, b,
                            (const double *)E1, c1, (const double *)E2, c2, (double *)acc, cacc,
                            acc_init ? 1 : 0, cinit, dtype);
    else if (dtype == LNE_F32)
        s = gspmm_t<float>(ctx, g, (const float *)Z, (float *)out, ld, k, a, b,
                           (const float *)E1, c1, (const float *)E2, c2, (float *)acc, cacc,
                           acc_init ? 1 : 0, cinit, dtype);
    else
        return fail(ctx, LNE_EINVAL, "graph_spmm: bad dtype");
    return s;
}

lne_status spmm_sparse_omega(lne_ctx *ctx, const lne_csr *A, const int16_t *om, void *Y,
                             int64_t ldy, int32_t k, int32_t dtype) {
    if (k < 1 || k > 1024 || ldy < k || !om || !Y)
        return fail(ctx, LNE_EINVAL, "spmm_sparse_omega: bad arguments");
    const unsigned grid = grid_of(A->n_rows * 64, 256);
    {
        Launch L(ctx, "spmm_sparse_omega");
        if (dtype == LNE_F64) {
            if (A->val_type != LNE_F64) return fail(ctx, LNE_EINVAL, "F64 needs F64 values");
            k_spmm_sparse_omega<double, double, double>
                <<<grid, 256, 4 * k * sizeof(double), ctx->stream>>>(
                    A->row_ptr, A->col, (const double *)A->val, A->n_rows, om, (double *)Y, ldy,
                    k);
        } else if (dtype == LNE_F32) {
            if (A->val_type != LNE_F32) return fail(ctx, LNE_EINVAL, "F32 needs F32 values");
            k_spmm_sparse_omega<float, float, float><<<grid, 256, 4 * k * sizeof(float),
                                                       ctx->stream>>>(
                A->row_ptr, A->col, (const float *)A->val, A->n_rows, om, (float *)Y, ldy, k);
        } else if (dtype == LNE_BF16) {
            if (A->val_type != LNE_F32) return fail(ctx, LNE_EINVAL, "BF16 needs F32 values");
            k_spmm_sparse_omega<float, float, __bf16><<<grid, 256, 4 * k * sizeof(float),
                                                        ctx->stream>>>(
                A->row_ptr, A->col, (const float *)A->val, A->n_rows, om, (__bf16 *)Y, ldy, k);
        } else {
            return fail(ctx, LNE_EINVAL, "spmm_sparse_omega: bad dtype");
        }
    }
    return check_launch(ctx, "spmm_sparse_omega");
}

lne_status axpby(lne_ctx *ctx, const void *x, const void *y, void *out, int64_t n, int32_t k,
                 int64_t ld, int32_t dt, double a, double b) {
    if (n * k == 0) return LNE_OK;
    {
        Launch L(ctx, "axpby");
        const unsigned grid = rows_grid(n);
        if (dt == LNE_F64)
            k_axpby<double><<<grid, 256, 0, ctx->stream>>>((const double *)x, (const double *)y,
                                                           (double *)out, n, k, ld, a, b);
        else if (dt == LNE_F32)
            k_axpby<float><<<grid, 256, 0, ctx->stream>>>((const float *)x, (const float *)y,
                                                          (float *)out, n, k, ld, (float)a,
                                                          (float)b);
        else
            return fail(ctx, LNE_EINVAL, "axpby: bad dtype");
    }
    return check_launch(ctx, "axpby");
}

lne_status dense_scale(lne_ctx *ctx, const void *x, int32_t xt, int64_t ldx, void *y,
                       int32_t yt, int64_t ldy, int64_t n, int32_t k, double alpha) {
    if (n * k == 0) return LNE_OK;
    const unsigned grid = rows_grid(n);
    {
        Launch L(ctx, "dense_scale");
#define LNE_SC(XT, YT)                                                                    \
    k_scale<XT, YT><<<grid, 256, 0, ctx->stream>>>((const XT *)x, ldx, (YT *)y, ldy, n, k, \
                                                   alpha)
        if (xt == LNE_F64 && yt == LNE_F64) LNE_SC(double, double);
        else if (xt == LNE_F64 && yt == LNE_F32) LNE_SC(double, float);
        else if (xt == LNE_F32 && yt == LNE_F32) LNE_SC(float, float);
        else if (xt == LNE_F32 && yt == LNE_F64) LNE_SC(float, double);
        else if (xt == LNE_F32 && yt == LNE_BF16) LNE_SC(float, __bf16);
        else if (xt == LNE_BF16 && yt == LNE_F32) LNE_SC(__bf16, float);
        else return fail(ctx, LNE_EINVAL, "dense_scale: unsupported conversion");
#undef LNE_SC
    }
    return check_launch(ctx, "dense_scale");
}

}  // namespace lne
