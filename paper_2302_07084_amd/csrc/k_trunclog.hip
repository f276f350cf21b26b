// Truncated logarithm of Eq. (1) on the count matrix, compacted in place of
// the paper's in-hash logarithm (section 5.2, "memory tricks").
//   x_ab = vol^2 / (2 b M) * (W_ab / 2^16) / (d_a d_b),  kept iff x_ab > 1.
// The keep decision is exact: W vol^2 > (2 b M 2^16) d_a d_b compared as
// 128-bit products (vol < 2^32 and 2 b M < 2^40 are validated on the host).
// One wave per row; kept entries are compacted with a ballot prefix so the
// output keeps the ascending column order.
#include "common.hpp"

namespace lne {

namespace {

__device__ __forceinline__ bool keep_entry(const TLConst &c, uint64_t W, uint64_t da,
                                           uint64_t db) {
    return tl_keep(c, W, da, db);
}

// deg: the graph's (weighted) vertex degrees (vertex_degrees)
__global__ void k_tl_count(TLConst c, const uint32_t *__restrict__ deg, int64_t row_lo, int64_t n,
                           const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const uint64_t *__restrict__ W, uint32_t *__restrict__ kept) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const uint64_t da = deg[row_lo + a];
    uint32_t cnt = 0;
    for (int64_t i = rp[a] + lane; i < rp[a + 1]; i += 64) {
        const int32_t b = col[i];
        cnt += keep_entry(c, W[i], da, (uint64_t)deg[b]) ? 1u : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0) kept[a] = cnt;
}

template <class VT>
__global__ void k_tl_fill(TLConst c, const uint32_t *__restrict__ deg, int64_t row_lo, int64_t n,
                          const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const uint64_t *__restrict__ W, const int64_t *__restrict__ orp,
                          int32_t *__restrict__ ocol, VT *__restrict__ oval) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t da = deg[row_lo + a];
    int64_t pos = orp[a];
    const int64_t beg = rp[a], end = rp[a + 1];
    for (int64_t i0 = beg; i0 < end; i0 += 64) {
        const int64_t i = i0 + lane;
        bool k = false;
        int32_t b = 0;
        uint64_t w = 0, db = 1;
        if (i < end) {
            b = col[i];
            w = W[i];
            db = deg[b];
            k = keep_entry(c, w, da, db);
        }
        const uint64_t mask = __ballot(k);
        if (k) {
            const int64_t o = pos + __popcll(mask & lt);
            const double x = (double)w * c.scale / ((double)da * (double)db);
            ocol[o] = b;
            oval[o] = (VT)log(x);
        }
        pos += __popcll(mask);
    }
}

// Nonzero count per row (one wave per row) and the compacting copy.
template <class VT>
__global__ void k_nz_count(int64_t n, const int64_t *__restrict__ rp, const VT *__restrict__ v,
                           uint32_t *__restrict__ cnt) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    uint32_t c = 0;
    for (int64_t i = rp[a] + lane; i < rp[a + 1]; i += 64) c += v[i] != (VT)0 ? 1u : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) cnt[a] = c;
}

template <class VT>
__global__ void k_nz_fill(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const VT *__restrict__ v, const int64_t *__restrict__ orp,
                          int32_t *__restrict__ ocol, VT *__restrict__ ov) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t pos = orp[a];
    const int64_t beg = rp[a], end = rp[a + 1];
    for (int64_t i0 = beg; i0 < end; i0 += 64) {
        const int64_t i = i0 + lane;
        const bool k = i < end && v[i] != (VT)0;
        const uint64_t mask = __ballot(k);
        if (k) {
            const int64_t o = pos + __popcll(mask & lt);
            ocol[o] = col[i];
            ov[o] = v[i];
        }
        pos += __popcll(mask);
    }
}

__global__ void k_shift_rows(const int64_t *__restrict__ rp, int64_t rows, int64_t row_lo,
                             int64_t off, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows) out[row_lo + i] = rp[i] + off;
}

}  // namespace

lne_status concat_rows(lne_ctx *ctx, std::vector<lne_csr> &blocks, int64_t n_rows,
                       lne_csr *out) {
    if (blocks.size() == 1 && blocks[0].n_rows == n_rows) {
        *out = blocks[0];
        blocks.clear();
        return LNE_OK;
    }
    const int64_t n_cols = blocks.empty() ? n_rows : blocks[0].n_cols;
    int64_t nnz = 0;
    for (auto &b : blocks) nnz += b.nnz;
    const int32_t vt = blocks.empty() ? LNE_U64 : blocks[0].val_type;
    const size_t es = dtype_size(vt);
    Buf rp(ctx), cc(ctx), vv(ctx);
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)(n_rows + 1)));
    LNE_TRY(alloc(ctx, cc, sizeof(int32_t) * (size_t)(nnz ? nnz : 1)));
    LNE_TRY(alloc(ctx, vv, es * (size_t)(nnz ? nnz : 1)));
    int64_t off = 0, lo = 0;
    for (auto &b : blocks) {
        if (b.n_rows > 0) {
            Launch L(ctx, "concat_rows");
            k_shift_rows<<<grid_of(b.n_rows, 256), 256, 0, ctx->stream>>>(b.row_ptr, b.n_rows, lo,
                                                                          off, rp.as<int64_t>());
        }
        LNE_TRY(check_launch(ctx, "concat_rows"));
        if (b.nnz > 0) {
            LNE_HIP(ctx, hipMemcpyAsync(cc.as<int32_t>() + off, b.col, sizeof(int32_t) * b.nnz,
                                        hipMemcpyDeviceToDevice, ctx->stream));
            LNE_HIP(ctx, hipMemcpyAsync(vv.as<char>() + es * off, b.val, es * b.nnz,
                                        hipMemcpyDeviceToDevice, ctx->stream));
        }
        off += b.nnz;
        lo += b.n_rows;
        dev_free(ctx, b.row_ptr);
        dev_free(ctx, b.col);
        dev_free(ctx, b.val);
    }
    blocks.clear();
    if (lo != n_rows) return fail(ctx, LNE_EINVAL, "concat_rows: blocks cover %lld of %lld rows",
                                  (long long)lo, (long long)n_rows);
    LNE_HIP(ctx, hipMemcpyAsync(rp.as<int64_t>() + n_rows, &off, sizeof(int64_t),
                                hipMemcpyHostToDevice, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out->n_rows = n_rows;
    out->n_cols = n_cols;
    out->nnz = nnz;
    out->row_ptr = (int64_t *)rp.detach();
    out->col = (int32_t *)cc.detach();
    out->val = vv.detach();
    out->val_type = vt;
    return LNE_OK;
}

lne_status drop_zeros(lne_ctx *ctx, lne_csr *m) {
    if (m->val_type != LNE_F32 && m->val_type != LNE_F64)
        return fail(ctx, LNE_EINVAL, "drop_zeros: F32 or F64 values expected");
    const int64_t n = m->n_rows;
    const bool f64 = m->val_type == LNE_F64;
    Buf cnt(ctx), rp(ctx);
    LNE_TRY(alloc(ctx, cnt, sizeof(uint32_t) * (size_t)(n + 1)));
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)(n + 1)));
    const unsigned grid = grid_of(n * 64, 256);
    if (n > 0) {
        Launch L(ctx, "drop_zeros");
        if (f64)
            k_nz_count<double><<<grid, 256, 0, ctx->stream>>>(n, m->row_ptr, (const double *)m->val,
                                                              cnt.as<uint32_t>());
        else
            k_nz_count<float><<<grid, 256, 0, ctx->stream>>>(n, m->row_ptr, (const float *)m->val,
                                                             cnt.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "drop_zeros"));
    LNE_TRY(scan_u32(ctx, cnt.as<uint32_t>(), rp.as<uint64_t>(), n));
    uint64_t nnz = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nnz, rp.as<int64_t>() + n, sizeof(uint64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    Buf cc(ctx), vv(ctx);
    LNE_TRY(alloc(ctx, cc, sizeof(int32_t) * (size_t)(nnz ? nnz : 1)));
    LNE_TRY(alloc(ctx, vv, dtype_size(m->val_type) * (size_t)(nnz ? nnz : 1)));
    if (n > 0) {
        Launch L(ctx, "drop_zeros");
        if (f64)
            k_nz_fill<double><<<grid, 256, 0, ctx->stream>>>(n, m->row_ptr, m->col,
                                                             (const double *)m->val,
                                                             rp.as<int64_t>(), cc.as<int32_t>(),
                                                             vv.as<double>());
        else
            k_nz_fill<float><<<grid, 256, 0, ctx->stream>>>(n, m->row_ptr, m->col,
                                                            (const float *)m->val,
                                                            rp.as<int64_t>(), cc.as<int32_t>(),
                                                            vv.as<float>());
    }
    LNE_TRY(check_launch(ctx, "drop_zeros"));
    const int32_t vt = m->val_type;
    const int64_t ncols = m->n_cols;
    lne_csr_free(ctx, m);
    m->n_rows = n;
    m->n_cols = ncols;
    m->nnz = (int64_t)nnz;
    m->row_ptr = (int64_t *)rp.detach();
    m->col = (int32_t *)cc.detach();
    m->val = vv.detach();
    m->val_type = vt;
    return LNE_OK;
}

lne_status trunc_log_csr(lne_ctx *ctx, const Graph *g, const lne_params *p,
                         const lne_csr *counts, int64_t row_lo, int32_t val_type, lne_csr *out) {
    const int64_t n = counts->n_rows;
    uint64_t vol = (uint64_t)g->n_arcs;
    Buf cw(ctx), deg(ctx);
    if (g->weight) LNE_TRY(weight_info(ctx, g, cw, &vol));
    const TLConst c = tl_const(vol, (uint64_t)g->n_arcs, p);
    LNE_TRY(alloc(ctx, deg, sizeof(uint32_t) * (size_t)(g->n > 0 ? g->n : 1)));
    LNE_TRY(vertex_degrees(ctx, g, deg.as<uint32_t>(), g->weight ? cw.as<uint64_t>() : nullptr));

    Buf kept(ctx), rp(ctx);
    LNE_TRY(alloc(ctx, kept, sizeof(uint32_t) * (size_t)(n + 1)));
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)(n + 1)));
    const unsigned grid = grid_of(n * 64, 256);
    if (n > 0) {
        Launch L(ctx, "trunc_log_count");
        k_tl_count<<<grid, 256, 0, ctx->stream>>>(c, deg.as<uint32_t>(), row_lo, n, counts->row_ptr,
                                                  counts->col, (const uint64_t *)counts->val,
                                                  kept.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "trunc_log_count"));
    LNE_TRY(scan_u32(ctx, kept.as<uint32_t>(), rp.as<uint64_t>(), n));
    uint64_t nnz = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nnz, rp.as<int64_t>() + n, sizeof(uint64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    Buf cc(ctx), vv(ctx);
    LNE_TRY(alloc(ctx, cc, sizeof(int32_t) * (size_t)(nnz ? nnz : 1)));
    LNE_TRY(alloc(ctx, vv, dtype_size(val_type) * (size_t)(nnz ? nnz : 1)));
    if (n > 0) {
        Launch L(ctx, "trunc_log_fill");
        if (val_type == LNE_F64)
            k_tl_fill<double><<<grid, 256, 0, ctx->stream>>>(
                c, deg.as<uint32_t>(), row_lo, n, counts->row_ptr, counts->col,
                (const uint64_t *)counts->val, rp.as<int64_t>(), cc.as<int32_t>(), vv.as<double>());
        else
            k_tl_fill<float><<<grid, 256, 0, ctx->stream>>>(
                c, deg.as<uint32_t>(), row_lo, n, counts->row_ptr, counts->col,
                (const uint64_t *)counts->val, rp.as<int64_t>(), cc.as<int32_t>(), vv.as<float>());
    }
    LNE_TRY(check_launch(ctx, "trunc_log_fill"));
    out->n_rows = n;
    out->n_cols = counts->n_cols;
    out->nnz = (int64_t)nnz;
    out->row_ptr = (int64_t *)rp.detach();
    out->col = (int32_t *)cc.detach();
    out->val = vv.detach();
    out->val_type = val_type;
    return LNE_OK;
}

}  // namespace lne
