// Batched hyperparameter trials sharing one sampling pass (section 4.4: many
// trials of s_1..s_T, k, theta, mu on one graph).
//
// The shared pass draws the walk length r from a sampling distribution pi
// (chosen for the batch) and keeps r in the count matrix, giving per-length
// channels W_r.  Trial t then uses sum_r (s_r^(t) / pi_r) W_r in place of the
// counts, which has the expectation of its own sampler whenever pi_r > 0 for
// every r with s_r^(t) > 0; the truncated logarithm is applied per trial on
// the shared structure (dropped entries keep an explicit zero).
//
// Nothing per trial is materialised at the size of the matrix: each SpMM of
// trial t regenerates M_t's values from the channel CSR while it streams it,
// and the dense blocks of all trials (n x k' each, trial-major) go through
// one launch per step (batched Gram, Cholesky, eigen-solves and projections,
// one channel SpMM over every (trial, row) pair, one graph SpMM per
// propagation step with per-trial epilogue coefficients).
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

// vals[i * ntr + t] = ln x if x > 1 else 0, x = scale * sum_r c_t[r] W_r /
// (d_a d_b) with c_t[r] = s_t[r] / pi_r and scale = vol^2 / (2 b M) / 2^16.
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
            const double x = acc * scale / dd;
            vals[i * ntr + t] = x > 1.0 ? (float)log(x) : 0.0f;
        }
    }
}

// Channel weights in place: W_r (fixed-point counts) -> the FP64 number
// scale W_r / (d_a d_b) (scale = vol^2 / (2 b M 2^16)), so that a trial's
// Eq. (1) argument is x = sum_r coef_t[r] w_r with coef_t[r] = s_t[r] / pi_r.
__global__ void k_norm_chan(const int64_t *__restrict__ rp, const int32_t *__restrict__ ecol,
                            const int64_t *__restrict__ grp, int64_t n, double scale,
                            uint64_t *__restrict__ W) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const double da = (double)(grp[a + 1] - grp[a]);
    double *out = reinterpret_cast<double *>(W);
    for (int64_t i = rp[a] + lane; i < rp[a + 1]; i += 64) {
        const int32_t b = ecol[i] >> 4;
        const double db = (double)(grp[b + 1] - grp[b]);
        out[i] = scale * (double)W[i] / (da * db);
    }
}

// Y_t = M_t X_t for trials t = 0..ntr-1 with M_t generated on the fly from
// the normalised channel CSR: every (row a, column b) structure entry is a
// run of channel entries with the same b (ascending r); a segmented scan over
// the wave sums x = sum_r coef_t[r] w_r with coef_t[r] = s_t[r] / pi_r (FP64,
// so the x > 1 decision is taken in FP64; a run crossing a 64-entry chunk
// carries its partial sum), and the lane holding the run's last entry forms
// the truncated logarithm ln x (FP32; 0 if x <= 1).  The nonzero values of a
// 64-entry chunk are compacted to the low lanes with one ds_permute, then the
// wave gathers the X rows of those entries, U rows in flight per lane, lane l
// holding columns 4l..4l+3 (k <= 256, k % 4 == 0, padding columns of X zero).
// TM: waves enumerate (trial, row) trial-major (consecutive waves share a
// trial's operand) or row-major (consecutive waves share a row's entries).
template <int U, bool TM>
__global__ void __launch_bounds__(256)
k_spmm_chan(const int64_t *__restrict__ rp, const int32_t *__restrict__ ecol,
            const double *__restrict__ wn, int64_t n, int ntr,
            const double *__restrict__ coef, const float *__restrict__ X,
            int64_t ldx, int64_t xs, float *__restrict__ Y, int64_t ldy, int64_t ys, int k) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n * ntr) return;
    int64_t row;
    int t;
    if (TM) {
        t = (int)(w / n);
        row = w - (int64_t)t * n;
    } else {
        row = w / ntr;
        t = (int)(w - row * ntr);
    }
    const int lane = threadIdx.x & 63;
    const int c0 = lane * 4;
    const bool act = c0 < k;
    X += (int64_t)t * xs;
    Y += (int64_t)t * ys;
    coef += 16 * t;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t beg = rp[row], end = rp[row + 1];
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);   // lanes 0..lane
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int32_t prev_b = -1;     // base column of the entry before the chunk
    double carry = 0.0;      // partial sum of the run that reaches into the chunk
    // the next chunk's structure is loaded while the current one is gathered
    int32_t ec_next = beg + lane < end ? ecol[beg + lane] : -16;
    double w_next = beg + lane < end ? wn[beg + lane] : 0.0;
    for (int64_t b0 = beg; b0 < end; b0 += 64) {
        const int64_t i = b0 + lane;
        const bool valid = i < end;
        const int32_t ec = ec_next;
        const double wv = w_next;
        ec_next = i + 64 < end ? ecol[i + 64] : -16;
        w_next = i + 64 < end ? wn[i + 64] : 0.0;
        const int32_t jb = ec >> 4;
        const double cw = valid ? coef[ec & 15] * wv : 0.0;
        const int32_t up_b = __shfl_up(jb, 1, 64);
        const bool head = valid && (lane == 0 ? prev_b : up_b) != jb;
        const uint64_t hm = __ballot(head);
        // segmented inclusive scan: a lane adds the partial of lane - off when
        // no run starts in (lane - off, lane]; a run holds at most one entry
        // per length (<= 16), so four doubling steps cover it
        double sum = cw;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const double o = __shfl_up(sum, off, 64);
            const int src = lane - off;
            const uint64_t below = src < 0 ? 0ull : (src == 63 ? ~0ull : ((2ull << src) - 1));
            if (src >= 0 && (hm & upto & ~below) == 0) sum += o;
        }
        if (valid && (hm & upto) == 0) sum += carry;    // the run carried into the chunk
        const int32_t dn_b = __shfl_down(jb, 1, 64);
        const int32_t first_next = __shfl(ec_next, 0, 64) >> 4;
        int32_t nb = dn_b;
        if (lane == 63) nb = b0 + 64 < end ? first_next : -2;
        const bool last = valid && (i + 1 >= end || nb != jb);
        float v = 0.f;
        if (last) v = sum > 1.0 ? logf((float)sum) : 0.f;
        carry = __shfl(sum, 63, 64);
        prev_b = __shfl(jb, 63, 64);
        const bool take = v != 0.f;
        const uint64_t mask = __ballot(take);
        const int cnt = __popcll(mask);
        // a permutation of the 64 lanes: kept entries first, in order
        const int dst = take ? __popcll(mask & lt) : cnt + __popcll(~mask & lt);
        const int jc = __builtin_amdgcn_ds_permute(dst << 2, jb);
        const float vc = __int_as_float(__builtin_amdgcn_ds_permute(dst << 2, __float_as_int(v)));
        for (int t0 = 0; t0 < cnt; t0 += U) {
            int32_t j[U];
            float vv[U];
            float4 x[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                j[q] = __shfl(jc, (t0 + q) & 63, 64);
                vv[q] = __shfl(vc, (t0 + q) & 63, 64);
            }
#pragma unroll
            for (int q = 0; q < U; ++q)
                x[q] = (act && t0 + q < cnt)
                           ? *reinterpret_cast<const float4 *>(X + (int64_t)j[q] * ldx + c0)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const float f = t0 + q < cnt ? vv[q] : 0.f;
                acc.x += f * x[q].x;
                acc.y += f * x[q].y;
                acc.z += f * x[q].z;
                acc.w += f * x[q].w;
            }
        }
    }
    if (act) *reinterpret_cast<float4 *>(Y + row * ldy + c0) = acc;
}

// Propagation step of every trial: out_t = a_t Z_t + b_t D^-1 A Z_t + c1_t E1_t
// + c2_t E2_t and accum_t += e_t out_t, coefficients coef[5 t + {0..4}].  The
// trials' n x ld blocks are zs apart.  L lanes (float4 each) per gathered row,
// 64 / L gathered rows per step of the wave, U steps in flight.
template <int L, int U, bool TM>
__global__ void __launch_bounds__(256)
k_gspmm_batch(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n,
              int ntr, int k, int64_t ld, int64_t zs, const float *__restrict__ Z,
              float *__restrict__ out, const float *__restrict__ E1, const float *__restrict__ E2,
              float *__restrict__ accum, const float *__restrict__ coef) {
    constexpr int G = 64 / L;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= n * ntr) return;
    int64_t row;
    int t;
    if (TM) {
        t = (int)(w / n);
        row = w - (int64_t)t * n;
    } else {
        row = w / ntr;
        t = (int)(w - row * ntr);
    }
    const int lane = threadIdx.x & 63;
    const int gi = lane / L, c0 = (lane % L) * 4;
    const bool act = c0 < k;
    const int64_t off = (int64_t)t * zs;
    Z += off;
    const int64_t beg = rp[row], end = rp[row + 1];
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t b0 = beg; b0 < end; b0 += 64) {
        const int64_t idx = b0 + lane;
        const int32_t cj = idx < end ? col[idx] : 0;
        const int cnt = (int)min((int64_t)64, end - b0);
        for (int t0 = 0; t0 < cnt; t0 += U * G) {
            int32_t j[U];
            float4 x[U];
#pragma unroll
            for (int q = 0; q < U; ++q) j[q] = __shfl(cj, (t0 + gi + q * G) & 63, 64);
#pragma unroll
            for (int q = 0; q < U; ++q)
                x[q] = (act && t0 + gi + q * G < cnt)
                           ? *reinterpret_cast<const float4 *>(Z + (int64_t)j[q] * ld + c0)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                s.x += x[q].x;
                s.y += x[q].y;
                s.z += x[q].z;
                s.w += x[q].w;
            }
        }
    }
#pragma unroll
    for (int o = L; o < 64; o <<= 1) {
        s.x += __shfl_xor(s.x, o, 64);
        s.y += __shfl_xor(s.y, o, 64);
        s.z += __shfl_xor(s.z, o, 64);
        s.w += __shfl_xor(s.w, o, 64);
    }
    if (gi != 0 || !act) return;
    const float *cf = coef + 5 * t;
    const float a = cf[0], b = cf[1], c1 = cf[2], c2 = cf[3], e = cf[4];
    const float inv = end > beg ? 1.0f / (float)(end - beg) : 0.0f;
    const int64_t o = off + row * ld + c0;
    const float4 z = *reinterpret_cast<const float4 *>(Z + row * ld + c0);
    float4 r = make_float4(a * z.x + b * (inv * s.x), a * z.y + b * (inv * s.y),
                           a * z.z + b * (inv * s.z), a * z.w + b * (inv * s.w));
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

// y = alpha[i / per] x over `count` floats (alpha per trial block of `per`)
__global__ void k_scale_blocks(const float *__restrict__ x, float *__restrict__ y, int64_t count,
                               int64_t per, const float *__restrict__ alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] = alpha[i / per] * x[i];
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
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

lne_status trial_values(lne_ctx *ctx, const Graph *g, const lne_csr *st, const uint64_t *chan,
                        int T, const double *s_dev, int ntr, double scale, float *vals) {
    if (st->n_rows > 0) {
        Launch L(ctx, "trial_values");
        k_trial_values<<<grid_of(st->n_rows * 64, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, st->row_ptr, st->col, chan, T, st->n_rows, s_dev, ntr, scale, vals);
    }
    return check_launch(ctx, "trial_values");
}

lne_status norm_channels(lne_ctx *ctx, lne_csr *ext, const Graph *g, double scale) {
    if (ext->val_type != LNE_U64) return fail(ctx, LNE_EINVAL, "norm_channels: counts expected");
    if (ext->n_rows > 0) {
        Launch L(ctx, "norm_channels");
        k_norm_chan<<<grid_of(ext->n_rows * 64, 256), 256, 0, ctx->stream>>>(
            ext->row_ptr, ext->col, g->row_ptr, ext->n_rows, scale, (uint64_t *)ext->val);
    }
    LNE_TRY(check_launch(ctx, "norm_channels"));
    ext->val_type = LNE_F64;
    return LNE_OK;
}

lne_status spmm_chan(lne_ctx *ctx, const lne_csr *ext, int ntr, const double *coef,
                     const float *X, int64_t ldx, int64_t xs, float *Y, int64_t ldy, int64_t ys,
                     int k, int variant) {
    if (ext->val_type != LNE_F64)
        return fail(ctx, LNE_EINVAL, "spmm_chan: channel weights must be normalised");
    if (k % 4 || k > 256 || ldx % 4 || ldy % 4 || xs % 4 || ys % 4 || (uintptr_t)X % 16 ||
        (uintptr_t)Y % 16)
        return fail(ctx, LNE_EINVAL, "spmm_chan: k <= 256, k %% 4 == 0 and 16-byte aligned rows");
    const int64_t n = ext->n_rows;
    if (n == 0 || ntr == 0) return LNE_OK;
    const unsigned grid = grid_of(n * ntr * 64, 256);
    {
        Launch L(ctx, "spmm_chan");
#define LNE_SC(UU, TMM)                                                                   \
    k_spmm_chan<UU, TMM><<<grid, 256, 0, ctx->stream>>>(ext->row_ptr, ext->col,           \
                                                        (const double *)ext->val, n, ntr, \
                                                        coef, X, ldx, xs, Y, ldy, ys, k)
        switch (variant) {
            case 0: LNE_SC(4, true); break;
            case 1: LNE_SC(2, true); break;
            case 2: LNE_SC(8, true); break;
            case 3: LNE_SC(4, false); break;
            case 4: LNE_SC(2, false); break;
            case 5: LNE_SC(8, false); break;
            default: return fail(ctx, LNE_EINVAL, "spmm_chan: variant %d", variant);
        }
#undef LNE_SC
    }
    return check_launch(ctx, "spmm_chan");
}

lne_status gspmm_batch(lne_ctx *ctx, const Graph *g, int ntr, int k, int64_t ld, int64_t zs,
                       const float *Z, float *out, const float *E1, const float *E2, float *acc,
                       const float *coef, int variant) {
    if (k % 4 || k > 256 || ld % 4 || zs % 4 || (uintptr_t)Z % 16 || (uintptr_t)out % 16)
        return fail(ctx, LNE_EINVAL, "gspmm_batch: k <= 256, k %% 4 == 0 and aligned rows");
    const int64_t n = g->n;
    if (n == 0 || ntr == 0) return LNE_OK;
    const unsigned grid = grid_of(n * ntr * 64, 256);
    const bool wide = k > 128;
    {
        Launch L(ctx, "graph_spmm_batch");
#define LNE_GB(LL, UU, TMM)                                                                  \
    k_gspmm_batch<LL, UU, TMM><<<grid, 256, 0, ctx->stream>>>(g->row_ptr, g->col, n, ntr, k, \
                                                             ld, zs, Z, out, E1, E2, acc,   \
                                                             coef)
        switch (variant * 2 + (wide ? 1 : 0)) {
            case 0: LNE_GB(32, 4, true); break;
            case 1: LNE_GB(64, 4, true); break;
            case 2: LNE_GB(32, 2, true); break;
            case 3: LNE_GB(64, 2, true); break;
            case 4: LNE_GB(32, 4, false); break;
            case 5: LNE_GB(64, 4, false); break;
            case 6: LNE_GB(32, 2, false); break;
            case 7: LNE_GB(64, 2, false); break;
            default: return fail(ctx, LNE_EINVAL, "gspmm_batch: variant %d", variant);
        }
#undef LNE_GB
    }
    return check_launch(ctx, "graph_spmm_batch");
}

lne_status scale_blocks(lne_ctx *ctx, const float *x, float *y, int64_t count, int64_t per,
                        const float *alpha) {
    if (count == 0) return LNE_OK;
    {
        Launch L(ctx, "scale_blocks");
        k_scale_blocks<<<grid_of(count, 256), 256, 0, ctx->stream>>>(x, y, count, per, alpha);
    }
    return check_launch(ctx, "scale_blocks");
}

lne_status fill_u32(lne_ctx *ctx, void *p, int64_t count, uint32_t v) {
    if (count == 0) return LNE_OK;
    {
        Launch L(ctx, "fill");
        k_fill_u32<<<grid_of(count, 256), 256, 0, ctx->stream>>>((uint32_t *)p, count, v);
    }
    return check_launch(ctx, "fill");
}

}  // namespace lne
