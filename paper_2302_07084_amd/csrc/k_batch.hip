// Batched hyperparameter trials sharing one sampling pass (section 4.4: many
// trials of s_1..s_T, k, theta, mu on one graph).
//
// The shared pass draws the walk length r uniformly from 1..T (pi_r = 1/T)
// and keeps r in the count matrix, giving per-length channels W_r.  Trial t
// then uses sum_r (s_r^(t) / pi_r) W_r in place of the counts, which has the
// expectation of its own sampler; the truncated logarithm is applied per
// trial on the shared structure (dropped entries keep an explicit zero).
//
// The rSVD products of all trials run as one "wide" SpMM: the dense operand
// of trial t is columns [t dp, t dp + k') of an n x (trials dp) matrix, so
// every gathered row serves every trial, each multiplied by its own value.
// Propagation likewise runs one wide graph SpMM per step, with the epilogue
// coefficients (1 - mu_t, Chebyshev weights of trial t) looked up per column
// block.
#include "common.hpp"

namespace lne {

namespace {

// number of distinct base columns (extended column >> 4) in each row
__global__ void k_split_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                              int64_t n, uint32_t *__restrict__ cnt) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const int64_t beg = rp[a], end = rp[a + 1];
    uint32_t c = 0;
    for (int64_t i = beg + lane; i < end; i += 64)
        c += (i == beg || (col[i] >> 4) != (col[i - 1] >> 4)) ? 1u : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) cnt[a] = c;
}

__global__ void k_split_fill(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const uint64_t *__restrict__ W, int64_t n,
                             const int64_t *__restrict__ srp, int32_t *__restrict__ scol,
                             uint64_t *__restrict__ chan, int T) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t beg = rp[a], end = rp[a + 1];
    int64_t pos = srp[a];
    for (int64_t i0 = beg; i0 < end; i0 += 64) {
        const int64_t i = i0 + lane;
        const bool valid = i < end;
        int32_t c = 0;
        bool head = false;
        if (valid) {
            c = col[i];
            head = i == beg || (c >> 4) != (col[i - 1] >> 4);
        }
        const uint64_t hm = __ballot(head);
        if (valid) {
            const int64_t u = pos + (int64_t)__popcll(hm & (lt | (1ull << lane))) - 1;
            if (head) scol[u] = c >> 4;
            const int r = c & 15;
            if (r < T) chan[u * T + r] = W[i];
        }
        pos += __popcll(hm);
    }
}

// vals[i * ntr + t] = ln x if x > 1 else 0, x = scale * T * sum_r s_t[r] W_r /
// (d_a d_b) with scale = vol^2 / (2 b M) / 2^16.
__global__ void k_trial_values(const int64_t *__restrict__ grp, const int64_t *__restrict__ srp,
                               const int32_t *__restrict__ scol, const uint64_t *__restrict__ chan,
                               int T, int64_t n, const double *__restrict__ s, int ntr,
                               double scale, float *__restrict__ vals) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const double da = (double)(grp[a + 1] - grp[a]);
    for (int64_t i = srp[a] + lane; i < srp[a + 1]; i += 64) {
        const int32_t b = scol[i];
        const double dd = da * (double)(grp[b + 1] - grp[b]);
        double w[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) w[r] = r < T ? (double)chan[i * T + r] : 0.0;
        for (int t = 0; t < ntr; ++t) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc += s[t * 16 + r] * w[r];
            const double x = (double)T * acc * scale / dd;
            vals[i * ntr + t] = x > 1.0 ? (float)log(x) : 0.0f;
        }
    }
}

// Y[row, c] = sum_i vals[i ntr + c / dp] X[col_i, c] over the row's entries,
// one wave per (row, 256-column block), float4 per lane.
__global__ void __launch_bounds__(256)
k_spmm_multi(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
             const float *__restrict__ vals, int ntr, int64_t n_rows, const float *__restrict__ X,
             int64_t ld, float *__restrict__ Y, int dp, int ncb) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n_rows * ncb) return;
    const int64_t row = w / ncb;
    const int cb = (int)(w - row * ncb);
    const int lane = threadIdx.x & 63;
    const int c0 = cb * 256 + lane * 4;
    const bool active = c0 < ntr * dp;
    const int trial = active ? c0 / dp : 0;
    const int64_t beg = rp[row], end = rp[row + 1];
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t b0 = beg; b0 < end; b0 += 64) {
        const int64_t idx = b0 + lane;
        const int32_t cj = idx < end ? col[idx] : 0;
        const int cnt = (int)min((int64_t)64, end - b0);
        for (int t0 = 0; t0 < cnt; t0 += 4) {
            int32_t j[4];
            float v[4];
            float4 x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) j[q] = __shfl(cj, (t0 + q) & 63);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = active && t0 + q < cnt;
                v[q] = ok ? vals[(b0 + t0 + q) * ntr + trial] : 0.f;
                x[q] = ok ? *reinterpret_cast<const float4 *>(X + (int64_t)j[q] * ld + c0)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[0] += v[q] * x[q].x;
                acc[1] += v[q] * x[q].y;
                acc[2] += v[q] * x[q].z;
                acc[3] += v[q] * x[q].w;
            }
        }
    }
    if (active)
        *reinterpret_cast<float4 *>(Y + row * ld + c0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
}

// out = a_t Z + b_t D^-1 A Z + c1_t E1 + c2_t E2; acc += e_t out; coefficients
// coef[5 t + {0..4}] of the trial owning the column.
__global__ void __launch_bounds__(256)
k_gspmm_multi(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n_rows,
              const float *__restrict__ Z, int64_t ld, int ntr, int dp, int ncb,
              float *__restrict__ out, const float *__restrict__ E1, const float *__restrict__ E2,
              float *__restrict__ accum, const float *__restrict__ coef) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n_rows * ncb) return;
    const int64_t row = w / ncb;
    const int cb = (int)(w - row * ncb);
    const int lane = threadIdx.x & 63;
    const int c0 = cb * 256 + lane * 4;
    const bool active = c0 < ntr * dp;
    const int64_t beg = rp[row], end = rp[row + 1];
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t b0 = beg; b0 < end; b0 += 64) {
        const int64_t idx = b0 + lane;
        const int32_t cj = idx < end ? col[idx] : 0;
        const int cnt = (int)min((int64_t)64, end - b0);
        for (int t0 = 0; t0 < cnt; t0 += 4) {
            int32_t j[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) j[q] = __shfl(cj, (t0 + q) & 63);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (active && t0 + q < cnt) {
                    const float4 x = *reinterpret_cast<const float4 *>(Z + (int64_t)j[q] * ld + c0);
                    s.x += x.x; s.y += x.y; s.z += x.z; s.w += x.w;
                }
            }
        }
    }
    if (!active) return;
    const int t = c0 / dp;
    const float a = coef[5 * t], b = coef[5 * t + 1], c1 = coef[5 * t + 2], c2 = coef[5 * t + 3],
                e = coef[5 * t + 4];
    const float inv = end > beg ? 1.0f / (float)(end - beg) : 0.0f;
    const int64_t o = row * ld + c0;
    const float4 z = *reinterpret_cast<const float4 *>(Z + o);
    float4 r = make_float4(a * z.x + b * inv * s.x, a * z.y + b * inv * s.y,
                           a * z.z + b * inv * s.z, a * z.w + b * inv * s.w);
    if (E1) {
        const float4 q = *reinterpret_cast<const float4 *>(E1 + o);
        r.x += c1 * q.x; r.y += c1 * q.y; r.z += c1 * q.z; r.w += c1 * q.w;
    }
    if (E2) {
        const float4 q = *reinterpret_cast<const float4 *>(E2 + o);
        r.x += c2 * q.x; r.y += c2 * q.y; r.z += c2 * q.z; r.w += c2 * q.w;
    }
    *reinterpret_cast<float4 *>(out + o) = r;
    if (accum) {
        float4 q = *reinterpret_cast<const float4 *>(accum + o);
        q.x += e * r.x; q.y += e * r.y; q.z += e * r.z; q.w += e * r.w;
        *reinterpret_cast<float4 *>(accum + o) = q;
    }
}

}  // namespace

lne_status split_channels(lne_ctx *ctx, const lne_csr *ext, int T, lne_csr *st, Buf &chan) {
    const int64_t n = ext->n_rows;
    Buf cnt(ctx), srp(ctx);
    LNE_TRY(alloc(ctx, cnt, sizeof(uint32_t) * (size_t)(n + 1)));
    LNE_TRY(alloc(ctx, srp, sizeof(int64_t) * (size_t)(n + 1)));
    const unsigned grid = grid_of(n * 64, 256);
    {
        Launch L(ctx, "split_channels");
        k_split_count<<<grid, 256, 0, ctx->stream>>>(ext->row_ptr, ext->col, n, cnt.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "split_channels"));
    LNE_TRY(scan_u32(ctx, cnt.as<uint32_t>(), srp.as<uint64_t>(), n));
    int64_t nnz = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nnz, srp.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    Buf scol(ctx);
    LNE_TRY(alloc(ctx, scol, sizeof(int32_t) * (size_t)(nnz ? nnz : 1)));
    LNE_TRY(alloc(ctx, chan, sizeof(uint64_t) * (size_t)(nnz ? nnz : 1) * T));
    LNE_HIP(ctx, hipMemsetAsync(chan.p, 0, sizeof(uint64_t) * (size_t)(nnz ? nnz : 1) * T,
                                ctx->stream));
    {
        Launch L(ctx, "split_channels");
        k_split_fill<<<grid, 256, 0, ctx->stream>>>(ext->row_ptr, ext->col,
                                                    (const uint64_t *)ext->val, n,
                                                    srp.as<int64_t>(), scol.as<int32_t>(),
                                                    chan.as<uint64_t>(), T);
    }
    LNE_TRY(check_launch(ctx, "split_channels"));
    st->n_rows = n;
    st->n_cols = n;
    st->nnz = nnz;
    st->row_ptr = (int64_t *)srp.detach();
    st->col = (int32_t *)scol.detach();
    st->val = nullptr;
    st->val_type = LNE_F32;
    return LNE_OK;
}

lne_status trial_values(lne_ctx *ctx, const lne_graph *g, const lne_csr *st, const uint64_t *chan,
                        int T, const double *s_dev, int ntr, double scale, float *vals) {
    if (st->n_rows > 0) {
        Launch L(ctx, "trial_values");
        k_trial_values<<<grid_of(st->n_rows * 64, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, st->row_ptr, st->col, chan, T, st->n_rows, s_dev, ntr, scale, vals);
    }
    return check_launch(ctx, "trial_values");
}

lne_status spmm_multi(lne_ctx *ctx, const lne_csr *st, const float *vals, int ntr, const float *X,
                      int64_t ld, float *Y, int dp) {
    if (dp % 4 || ld % 4 || (uintptr_t)X % 16 || (uintptr_t)Y % 16)
        return fail(ctx, LNE_EINVAL, "spmm_multi: 16-byte aligned slices required");
    const int ncb = (ntr * dp + 255) / 256;
    {
        Launch L(ctx, "spmm_multi");
        k_spmm_multi<<<grid_of(st->n_rows * ncb * 64, 256), 256, 0, ctx->stream>>>(
            st->row_ptr, st->col, vals, ntr, st->n_rows, X, ld, Y, dp, ncb);
    }
    return check_launch(ctx, "spmm_multi");
}

lne_status gspmm_multi(lne_ctx *ctx, const lne_graph *g, const float *Z, int64_t ld, int ntr,
                       int dp, float *out, const float *E1, const float *E2, float *acc,
                       const float *coef) {
    if (dp % 4 || ld % 4) return fail(ctx, LNE_EINVAL, "gspmm_multi: aligned slices required");
    const int ncb = (ntr * dp + 255) / 256;
    {
        Launch L(ctx, "graph_spmm_multi");
        k_gspmm_multi<<<grid_of(g->n * ncb * 64, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, g->col, g->n, Z, ld, ntr, dp, ncb, out, E1, E2, acc, coef);
    }
    return check_launch(ctx, "graph_spmm_multi");
}

}  // namespace lne
