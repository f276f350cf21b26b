// Link-prediction evaluation (the protocol of the very-large-graph runs in
// the experiments section, after PyTorch-BigGraph): held-out edges are ranked
// against corrupted edges by the inner product of their endpoints' embedding
// rows, and the ranks are summarised as mean rank, mean reciprocal rank,
// HITS@k and AUC.
//
// k_link_rank: one 256-thread block per held-out edge (u, v).  x_u is staged
// once in LDS as FP64; every lane scores its share of the K corrupted
// destinations w (and every lane scores v itself, so the positive score is
// computed by the same sequential FP64 loop as the negatives): lane-private
// FP64 sums over the d columns, the row read as 16-byte vectors.  The block
// counts negatives scoring above and equal to the positive.
// k_link_metrics: one block folds the per-edge counts into the four metrics
// in a fixed order (deterministic).
#include "common.hpp"

namespace lne {

namespace {

constexpr int kLinkThreads = 256;
constexpr int kLinkMaxD = 2048;

template <class T>
__device__ __forceinline__ double dot_row(const double *__restrict__ xu,
                                          const T *__restrict__ row, int d) {
    double s = 0.0;
    if constexpr (sizeof(T) == 4) {
        int c = 0;
        for (; c + 4 <= d; c += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(row + c);
            s += xu[c] * (double)v.x;
            s += xu[c + 1] * (double)v.y;
            s += xu[c + 2] * (double)v.z;
            s += xu[c + 3] * (double)v.w;
        }
        for (; c < d; ++c) s += xu[c] * (double)row[c];
    } else {
        int c = 0;
        for (; c + 2 <= d; c += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(row + c);
            s += xu[c] * v.x;
            s += xu[c + 1] * v.y;
        }
        for (; c < d; ++c) s += xu[c] * row[c];
    }
    return s;
}

template <class T>
__global__ void __launch_bounds__(kLinkThreads)
k_link_rank(const T *__restrict__ X, int64_t n, int64_t ldx, int d,
            const int32_t *__restrict__ pos, const int32_t *__restrict__ neg, int K,
            uint32_t *__restrict__ above, uint32_t *__restrict__ ties,
            unsigned long long *__restrict__ bad) {
    __shared__ double xu[kLinkMaxD];
    __shared__ uint32_t wa[kLinkThreads / 64], wt[kLinkThreads / 64];
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t u = pos[2 * e], v = pos[2 * e + 1];
    const bool ok = u >= 0 && u < n && v >= 0 && v < n;   // block-uniform
    if (!ok) {
        if (tid == 0) {
            atomicAdd(bad, 1ull);
            above[e] = 0;
            ties[e] = 0;
        }
        return;
    }
    for (int c = tid; c < d; c += kLinkThreads) xu[c] = (double)X[(int64_t)u * ldx + c];
    __syncthreads();
    const double sp = dot_row<T>(xu, X + (int64_t)v * ldx, d);
    uint32_t na = 0, nt = 0, nbad = 0;
    for (int j = tid; j < K; j += kLinkThreads) {
        const int32_t w = neg[e * K + j];
        if (w < 0 || w >= n) {
            ++nbad;
            continue;
        }
        const double s = dot_row<T>(xu, X + (int64_t)w * ldx, d);
        na += s > sp ? 1u : 0u;
        nt += s == sp ? 1u : 0u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        na += __shfl_xor(na, o, 64);
        nt += __shfl_xor(nt, o, 64);
        nbad += __shfl_xor(nbad, o, 64);
    }
    if (lane == 0) {
        wa[wv] = na;
        wt[wv] = nt;
        if (nbad) atomicAdd(bad, (unsigned long long)nbad);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t a = 0, t = 0;
        for (int i = 0; i < kLinkThreads / 64; ++i) {
            a += wa[i];
            t += wt[i];
        }
        above[e] = a;
        ties[e] = t;
    }
}

// metrics[0..3] = mean rank, mean reciprocal rank, HITS@k, AUC, with rank =
// 1 + above (ties counted in the positive's favour) and the per-edge AUC
// (K - above - ties / 2) / K.
__global__ void __launch_bounds__(1024)
k_link_metrics(const uint32_t *__restrict__ above, const uint32_t *__restrict__ ties, int64_t h,
               int K, int hits_k, double *__restrict__ metrics) {
    __shared__ double red[4][1024 / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = tid; e < h; e += 1024) {
        const double r = 1.0 + (double)above[e];
        s[0] += r;
        s[1] += 1.0 / r;
        s[2] += r <= (double)hits_k ? 1.0 : 0.0;
        s[3] += ((double)K - (double)above[e] - 0.5 * (double)ties[e]) / (double)K;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s[i] += __shfl_xor(s[i], o, 64);
        if (lane == 0) red[i][wv] = s[i];
    }
    __syncthreads();
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) t += red[tid][w];
        metrics[tid] = t / (double)h;
    }
}

}  // namespace

}  // namespace lne

using namespace lne;

extern "C" {

lne_status lne_link_rank(lne_ctx *ctx, const void *X, int64_t n, int32_t d, int64_t ldx,
                         int32_t dtype, const int32_t *pos, int64_t h, const int32_t *neg,
                         int32_t K, int32_t hits_k, uint32_t *above, uint32_t *ties,
                         double *metrics) {
    if (!ctx) return LNE_EINVAL;
    if (!X || !pos || !neg || !metrics || n < 1 || d < 1 || d > kLinkMaxD || ldx < d || h < 1 ||
        h > 0x7fffffff || K < 1 || hits_k < 1 || (dtype != LNE_F32 && dtype != LNE_F64))
        return fail(ctx, LNE_EINVAL, "link_rank: bad arguments");
    const int N = dtype == LNE_F32 ? 4 : 2;
    if ((uintptr_t)X % 16 || ldx % N)
        return fail(ctx, LNE_EINVAL, "link_rank: X rows must be 16-byte aligned");
    Buf ab(ctx), tb(ctx), bb(ctx);
    if (!above) {
        LNE_TRY(alloc(ctx, ab, sizeof(uint32_t) * (size_t)h));
        above = ab.as<uint32_t>();
    }
    if (!ties) {
        LNE_TRY(alloc(ctx, tb, sizeof(uint32_t) * (size_t)h));
        ties = tb.as<uint32_t>();
    }
    LNE_TRY(alloc(ctx, bb, sizeof(unsigned long long)));
    LNE_HIP(ctx, hipMemsetAsync(bb.p, 0, sizeof(unsigned long long), ctx->stream));
    {
        Launch L(ctx, "link_rank");
        if (dtype == LNE_F32)
            k_link_rank<float><<<(unsigned)h, kLinkThreads, 0, ctx->stream>>>(
                (const float *)X, n, ldx, d, pos, neg, K, above, ties,
                bb.as<unsigned long long>());
        else
            k_link_rank<double><<<(unsigned)h, kLinkThreads, 0, ctx->stream>>>(
                (const double *)X, n, ldx, d, pos, neg, K, above, ties,
                bb.as<unsigned long long>());
    }
    LNE_TRY(check_launch(ctx, "link_rank"));
    {
        Launch L(ctx, "link_metrics");
        k_link_metrics<<<1, 1024, 0, ctx->stream>>>(above, ties, h, K, hits_k, metrics);
    }
    LNE_TRY(check_launch(ctx, "link_metrics"));
    unsigned long long nbad = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nbad, bb.p, sizeof(nbad), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nbad)
        return fail(ctx, LNE_EINVAL, "link_rank: %llu vertex ids outside [0, n)", nbad);
    return LNE_OK;
}

}  // extern "C"
