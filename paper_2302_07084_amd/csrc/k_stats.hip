// Graph descriptors for the hyperparameter search's surrogate (section 4.4
// searches trials per graph; which descriptors condition the surrogate is
// this library's choice): degree moments, the median degree and the Hill
// tail exponent above it, wedge-sampled clustering, and the spectral gap of
// D^-1/2 A D^-1/2 by block subspace iteration.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "philox.hpp"

namespace lne {
namespace {

constexpr uint32_t kTagWedge = 6u << 24;   // counter tag of the wedge draws
constexpr int kStatThreads = 256;
constexpr int kStatBlocks = 256;
constexpr int kHistLds = 4096;             // degrees below this count in LDS first
constexpr int kWalkB = 16;                 // widest block of the subspace iteration

// sums: [0] degree sum, [1] sum of squared degrees, [2] vertices of degree
// >= 2, [3] maximum degree (integers, so the order of accumulation is moot)
__global__ void k_deg_moments(const int64_t *__restrict__ rp, int64_t n,
                              unsigned long long *__restrict__ sums) {
    unsigned long long s1 = 0, s2 = 0, c2 = 0, mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = (unsigned long long)(rp[i + 1] - rp[i]);
        s1 += d;
        s2 += d * d;
        c2 += d >= 2 ? 1 : 0;
        mx = d > mx ? d : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
        c2 += __shfl_xor(c2, o, 64);
        const unsigned long long y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sums[0], s1);
        atomicAdd(&sums[1], s2);
        atomicAdd(&sums[2], c2);
        atomicMax(&sums[3], mx);
    }
}

// Degree histogram (hist has at least kHistLds bins): small degrees, where a
// power-law graph puts most vertices, are counted per block in LDS first.
__global__ void k_deg_hist(const int64_t *__restrict__ rp, int64_t n, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kHistLds];
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = rp[i + 1] - rp[i];
        if (d < kHistLds) atomicAdd(&h[d], 1u);
        else atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// The degrees of ranks r0 and r1 in ascending order (cum: exclusive prefix
// counts of the histogram, nb + 1 entries).
__global__ void k_order_stat(const uint64_t *__restrict__ cum, int64_t nb, uint64_t r0,
                             uint64_t r1, int64_t *__restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const uint64_t lo = cum[b], hi = cum[b + 1];
    if (lo <= r0 && r0 < hi) out[0] = b;
    if (lo <= r1 && r1 < hi) out[1] = b;
}

// Per-block sums of log(d / (x_min - 1/2)) over degrees d >= x_min, and
// their count.
__global__ void k_hill(const int64_t *__restrict__ rp, int64_t n, double xmin,
                       double *__restrict__ part, unsigned long long *__restrict__ cnt) {
    __shared__ double ws[kStatThreads / 64];
    double s = 0.0;
    unsigned long long c = 0;
    const double den = xmin - 0.5;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)(rp[i + 1] - rp[i]);
        if (d >= xmin) {
            s += log(d / den);
            ++c;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        ws[threadIdx.x >> 6] = s;
        atomicAdd(cnt, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kStatThreads / 64; ++w) t += ws[w];
        part[blockIdx.x] = t;
    }
}

// out[0] = sum of part[0..np) in a fixed order (one wave).
__global__ void k_sum_parts(const double *__restrict__ part, int np, double *__restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 64) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_flag_deg2(const int64_t *__restrict__ rp, int64_t n, uint32_t *__restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = rp[i + 1] - rp[i] >= 2 ? 1u : 0u;
}

__global__ void k_compact_deg2(const int64_t *__restrict__ rp, int64_t n,
                               const uint64_t *__restrict__ off, int32_t *__restrict__ cand) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && rp[i + 1] - rp[i] >= 2) cand[off[i]] = (int32_t)i;
}

// Wedge t: Philox block of counter (t_lo, t_hi, 0, tag) under key seed;
// centre = cand[((z1 << 32) | z0) mod nc], ends = its neighbours at z2 mod d
// and z3 mod (d - 1) (moved past the first when not smaller); closed when
// the second end is in the first end's sorted row.
__global__ void k_wedges(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                         const int32_t *__restrict__ cand, uint64_t nc, uint64_t seed,
                         int64_t wedges, unsigned long long *__restrict__ closed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= wedges) return;
    const uint4 z = philox4x32_10(make_uint4((uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u,
                                             kTagWedge),
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    const int32_t c = cand[((((uint64_t)z.y) << 32) | z.x) % nc];
    const int64_t r0 = rp[c];
    const uint32_t d = (uint32_t)(rp[c + 1] - r0);
    const uint32_t ia = z.z % d;
    uint32_t ib = z.w % (d - 1);
    if (ib >= ia) ++ib;
    const int32_t a = col[r0 + ia], b = col[r0 + ib];
    int64_t lo = rp[a];
    const int64_t end = rp[a + 1];
    int64_t hi = end;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < b) lo = mid + 1; else hi = mid;
    }
    if (lo < end && col[lo] == b) atomicAdd(closed, 1ull);
}

__global__ void k_inv_sqrt_deg(const int64_t *__restrict__ rp, int64_t n, double *__restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t d = rp[i + 1] - rp[i];
    s[i] = d > 0 ? 1.0 / sqrt((double)d) : 0.0;
}

// Y = (X + S A S X) / 2 for n x b row-major blocks (b <= kWalkB), S =
// diag(s): kWalkB lanes per row, lane c summing column c over the row's
// neighbours in CSR order.
__global__ void k_half_walk(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const double *__restrict__ s, const double *__restrict__ X,
                            double *__restrict__ Y, int64_t n, int b) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = g / kWalkB;
    const int c = (int)(g % kWalkB);
    if (i >= n || c >= b) return;
    double acc = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = col[e];
        acc += s[j] * X[(int64_t)j * b + c];
    }
    Y[i * b + c] = 0.5 * (X[i * b + c] + s[i] * acc);
}

}  // namespace

lne_status graph_stats_impl(lne_ctx *ctx, const Graph *g, uint64_t seed, int32_t wedges,
                            int32_t iters, double *out) {
    const int64_t n = g->n, arcs = g->n_arcs;
    const int64_t *rp = g->row_ptr;
    const unsigned nblk = std::min<unsigned>(grid_of(n, kStatThreads), 1024u);
    // degree moments
    Buf sums(ctx);
    LNE_TRY(alloc(ctx, sums, 4 * sizeof(unsigned long long)));
    LNE_HIP(ctx, hipMemsetAsync(sums.p, 0, 4 * sizeof(unsigned long long), ctx->stream));
    {
        Launch L(ctx, "graph_stats");
        k_deg_moments<<<nblk, kStatThreads, 0, ctx->stream>>>(rp, n, sums.as<unsigned long long>());
    }
    LNE_TRY(check_launch(ctx, "graph_stats"));
    unsigned long long hs[4];
    LNE_HIP(ctx, hipMemcpyAsync(hs, sums.p, sizeof(hs), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned long long s1 = hs[0], s2 = hs[1], ncand = hs[2], maxd = hs[3];
    if (s1 != (unsigned long long)arcs)
        return fail(ctx, LNE_EINVAL, "graph_stats: row_ptr does not span n_arcs");
    const double mean = (double)s1 / (double)n;
    // population variance from exact integers: (n s2 - s1^2) / n^2
    const unsigned __int128 num = (unsigned __int128)n * s2 - (unsigned __int128)s1 * s1;
    const double var = (double)num / ((double)n * (double)n);
    out[0] = std::log((double)n);
    out[1] = std::log((double)std::max<int64_t>(arcs / 2, 1));
    out[2] = std::log(mean);
    out[3] = std::sqrt(var) / mean;
    out[4] = std::log((double)maxd);
    // median degree from the histogram's prefix counts
    const int64_t nb = std::max<int64_t>((int64_t)maxd + 1, kHistLds);
    Buf hist(ctx), cum(ctx), ost(ctx);
    LNE_TRY(alloc(ctx, hist, sizeof(uint32_t) * (size_t)nb));
    LNE_TRY(alloc(ctx, cum, sizeof(uint64_t) * (size_t)(nb + 1)));
    LNE_TRY(alloc(ctx, ost, 2 * sizeof(int64_t)));
    LNE_HIP(ctx, hipMemsetAsync(hist.p, 0, sizeof(uint32_t) * (size_t)nb, ctx->stream));
    {
        Launch L(ctx, "graph_stats");
        k_deg_hist<<<nblk, kStatThreads, 0, ctx->stream>>>(rp, n, hist.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "graph_stats"));
    LNE_TRY(scan_u32(ctx, hist.as<uint32_t>(), cum.as<uint64_t>(), nb));
    {
        Launch L(ctx, "graph_stats");
        k_order_stat<<<grid_of(nb, kStatThreads), kStatThreads, 0, ctx->stream>>>(
            cum.as<uint64_t>(), nb, (uint64_t)(n - 1) / 2, (uint64_t)n / 2, ost.as<int64_t>());
    }
    LNE_TRY(check_launch(ctx, "graph_stats"));
    int64_t med[2];
    LNE_HIP(ctx, hipMemcpyAsync(med, ost.p, sizeof(med), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double xmin = std::max(1.0, 0.5 * ((double)med[0] + (double)med[1]));
    // Hill tail exponent
    Buf part(ctx), hsum(ctx), hcnt(ctx);
    LNE_TRY(alloc(ctx, part, sizeof(double) * kStatBlocks));
    LNE_TRY(alloc(ctx, hsum, sizeof(double)));
    LNE_TRY(alloc(ctx, hcnt, sizeof(unsigned long long)));
    LNE_HIP(ctx, hipMemsetAsync(hcnt.p, 0, sizeof(unsigned long long), ctx->stream));
    {
        Launch L(ctx, "graph_stats");
        k_hill<<<kStatBlocks, kStatThreads, 0, ctx->stream>>>(rp, n, xmin, part.as<double>(),
                                                             hcnt.as<unsigned long long>());
        k_sum_parts<<<1, 64, 0, ctx->stream>>>(part.as<double>(), kStatBlocks, hsum.as<double>());
    }
    LNE_TRY(check_launch(ctx, "graph_stats"));
    double hl = 0.0;
    unsigned long long hc = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&hl, hsum.p, sizeof(hl), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipMemcpyAsync(&hc, hcnt.p, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out[5] = 1.0 + (double)hc / std::max(hl, 1e-9);
    // wedge clustering
    unsigned long long closed = 0;
    if (ncand > 0) {
        Buf flag(ctx), off(ctx), cand(ctx), cl(ctx);
        LNE_TRY(alloc(ctx, flag, sizeof(uint32_t) * (size_t)n));
        LNE_TRY(alloc(ctx, off, sizeof(uint64_t) * (size_t)(n + 1)));
        LNE_TRY(alloc(ctx, cand, sizeof(int32_t) * (size_t)ncand));
        LNE_TRY(alloc(ctx, cl, sizeof(unsigned long long)));
        LNE_HIP(ctx, hipMemsetAsync(cl.p, 0, sizeof(unsigned long long), ctx->stream));
        {
            Launch L(ctx, "graph_stats");
            k_flag_deg2<<<grid_of(n, kStatThreads), kStatThreads, 0, ctx->stream>>>(
                rp, n, flag.as<uint32_t>());
        }
        LNE_TRY(check_launch(ctx, "graph_stats"));
        LNE_TRY(scan_u32(ctx, flag.as<uint32_t>(), off.as<uint64_t>(), n));
        {
            Launch L(ctx, "graph_stats");
            k_compact_deg2<<<grid_of(n, kStatThreads), kStatThreads, 0, ctx->stream>>>(
                rp, n, off.as<uint64_t>(), cand.as<int32_t>());
            k_wedges<<<grid_of(wedges, kStatThreads), kStatThreads, 0, ctx->stream>>>(
                rp, g->col, cand.as<int32_t>(), ncand, seed, wedges,
                cl.as<unsigned long long>());
        }
        LNE_TRY(check_launch(ctx, "graph_stats"));
        LNE_HIP(ctx, hipMemcpyAsync(&closed, cl.p, sizeof(closed), hipMemcpyDeviceToHost,
                                    ctx->stream));
        LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    out[6] = (double)closed / (double)wedges;
    // spectral gap: X = Omega, then iters times X = U of eigSVD((X + S A S X) / 2)
    const int b = (int)std::min<int64_t>(kWalkB, n);
    Buf s(ctx), X(ctx), Y(ctx), S(ctx);
    LNE_TRY(alloc(ctx, s, sizeof(double) * (size_t)n));
    LNE_TRY(alloc(ctx, X, sizeof(double) * (size_t)n * b));
    LNE_TRY(alloc(ctx, Y, sizeof(double) * (size_t)n * b));
    LNE_TRY(alloc(ctx, S, sizeof(double) * (size_t)b));
    {
        Launch L(ctx, "graph_stats");
        k_inv_sqrt_deg<<<grid_of(n, kStatThreads), kStatThreads, 0, ctx->stream>>>(
            rp, n, s.as<double>());
    }
    LNE_TRY(check_launch(ctx, "graph_stats"));
    LNE_TRY(lne_gaussian(ctx, n, b, b, seed, LNE_F64, X.p));
    for (int it = 0; it < iters; ++it) {
        {
            Launch L(ctx, "graph_stats");
            k_half_walk<<<grid_of(n * kWalkB, kStatThreads), kStatThreads, 0, ctx->stream>>>(
                rp, g->col, s.as<double>(), X.as<double>(), Y.as<double>(), n, b);
        }
        LNE_TRY(check_launch(ctx, "graph_stats"));
        LNE_TRY(lne_eigsvd(ctx, Y.p, n, b, b, LNE_F64, X.p, b, S.as<double>(), nullptr));
    }
    double sv[2] = {0.0, 0.0};
    LNE_HIP(ctx, hipMemcpyAsync(sv, S.p, sizeof(double) * (size_t)std::min(b, 2),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out[7] = 1.0 - (2.0 * (b > 1 ? sv[1] : sv[0]) - 1.0);
    return LNE_OK;
}

}  // namespace lne
