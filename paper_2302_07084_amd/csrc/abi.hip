// C ABI of the library: argument validation, the sampler's host constants,
// context and scratch management, and the orchestration of the stages
// (sparsify -> trunc_log -> fast randomized SVD -> spectral propagation).
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <limits>

#include "common.hpp"

namespace lne {

lne_status fail(lne_ctx *ctx, lne_status code, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

void *dev_alloc(lne_ctx *ctx, size_t bytes) {
    if (bytes == 0) bytes = 1;
    const size_t rounded = (bytes + 255) / 256 * 256;
    if (ctx->arena_on) {
        if (ctx->arena_used + rounded > ctx->arena_cap) return nullptr;
        void *p = ctx->arena + ctx->arena_used;
        ctx->arena_used += rounded;
        return p;
    }
    if (ctx->arena_measure) ctx->arena_need += rounded;
    if (ctx->alloc) return ctx->alloc(bytes, ctx->user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(lne_ctx *ctx, void *p) {
    if (!p) return;
    if (ctx->arena && (char *)p >= ctx->arena && (char *)p < ctx->arena + ctx->arena_cap) return;
    if (ctx->free_fn) ctx->free_fn(p, ctx->user);
    else (void)hipFree(p);
}

void Buf::release() {
    if (p && ctx) dev_free(ctx, p);
    p = nullptr;
    bytes = 0;
}

lne_status alloc(lne_ctx *ctx, Buf &b, size_t bytes) {
    b.release();
    b.ctx = ctx;
    b.p = dev_alloc(ctx, bytes);
    if (!b.p) return fail(ctx, LNE_ENOMEM, "device allocation of %zu bytes failed", bytes);
    b.bytes = bytes;
    return LNE_OK;
}

Launch::Launch(lne_ctx *c, const char *n) : ctx(c), name(n) {
    if (ctx->prof && !ctx->capturing && !ctx->no_events) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, ctx->stream);
    }
}

Launch::~Launch() {
    if (ctx->prof && a && b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->marks.push_back({name, a, b});
    }
}

lne_status check_launch(lne_ctx *ctx, const char *name) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(ctx, LNE_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e));
    return LNE_OK;
}

size_t dtype_size(int32_t t) {
    switch (t) {
        case LNE_F64: return 8;
        case LNE_F32: return 4;
        case LNE_BF16: return 2;
        case LNE_U64: return 8;
        default: return 0;
    }
}

lne_status validate_graph(lne_ctx *ctx, const lne_graph *g) {
    if (!g) return fail(ctx, LNE_EINVAL, "graph is NULL");
    if (g->n < 1 || g->n >= (int64_t)1 << 31)
        return fail(ctx, LNE_EINVAL, "graph: n = %lld outside [1, 2^31)", (long long)g->n);
    if (g->n_arcs < 0 || (g->n_arcs & 1) || g->n_arcs >= (int64_t)1 << 32)
        return fail(ctx, LNE_EINVAL, "graph: n_arcs = %lld must be even and below 2^32",
                    (long long)g->n_arcs);
    if (!g->row_ptr || (g->n_arcs > 0 && !g->col))
        return fail(ctx, LNE_EINVAL, "graph: NULL row_ptr or col");
    if (g->index_bits != 0 && g->index_bits != 32 && g->index_bits != 64)
        return fail(ctx, LNE_EINVAL, "graph: index_bits = %d (32 or 64)", g->index_bits);
    if (g->index_bits == 32 && g->n_arcs >= (int64_t)1 << 31)
        return fail(ctx, LNE_EINVAL, "graph: 32-bit offsets with n_arcs = %lld >= 2^31",
                    (long long)g->n_arcs);
    return LNE_OK;
}

namespace {
__global__ void k_widen_offsets(const int32_t *__restrict__ in, int64_t *__restrict__ out,
                                int64_t n1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) out[i] = (int64_t)in[i];
}
}  // namespace

lne_status bind_graph(lne_ctx *ctx, const lne_graph *g, Buf &rp, Graph &out) {
    out.n = g->n;
    out.n_arcs = g->n_arcs;
    out.col = g->col;
    out.weight = g->weight;
    if (g->index_bits != 32) {
        out.row_ptr = static_cast<const int64_t *>(g->row_ptr);
        return LNE_OK;
    }
    const int64_t n1 = g->n + 1;
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)n1));
    {
        Launch L(ctx, "widen_offsets");
        k_widen_offsets<<<grid_of(n1, 256), 256, 0, ctx->stream>>>(
            static_cast<const int32_t *>(g->row_ptr), rp.as<int64_t>(), n1);
    }
    LNE_TRY(check_launch(ctx, "widen_offsets"));
    out.row_ptr = rp.as<int64_t>();
    return LNE_OK;
}

lne_status validate_params(lne_ctx *ctx, const lne_params *p, int64_t n, int64_t n_arcs,
                           bool need_linalg) {
    if (!p) return fail(ctx, LNE_EINVAL, "params is NULL");
    if (p->T < 1 || p->T > 16) return fail(ctx, LNE_EINVAL, "T = %d outside 1..16", p->T);
    double tot = 0.0;
    for (int t = 0; t < p->T; ++t) {
        if (!(p->s[t] >= 0.0) || !std::isfinite(p->s[t]))
            return fail(ctx, LNE_EINVAL, "s[%d] must be finite and >= 0", t);
        tot += p->s[t];
    }
    if (!(tot > 0.0)) return fail(ctx, LNE_EINVAL, "s must have a positive sum");
    if (p->b < 1) return fail(ctx, LNE_EINVAL, "b must be >= 1");
    const unsigned __int128 bm = (unsigned __int128)2 * p->b * p->M;
    if (bm >= ((unsigned __int128)1 << 40)) return fail(ctx, LNE_EINVAL, "2 b M must be below 2^40");
    if (std::isnan(p->C)) return fail(ctx, LNE_EINVAL, "C is NaN");
    if (!need_linalg) return LNE_OK;
    if (p->d < 1 || p->oversample < 0) return fail(ctx, LNE_EINVAL, "d >= 1, oversample >= 0");
    const int64_t kp = (int64_t)p->d + p->oversample;
    if (kp > n) return fail(ctx, LNE_EINVAL, "d + oversample = %lld exceeds n", (long long)kp);
    if (kp > 288) return fail(ctx, LNE_EUNSUPPORTED, "d + oversample = %lld above 288", (long long)kp);
    if (p->q < 1) return fail(ctx, LNE_EINVAL, "q must be >= 1");
    if (p->cheb_k < 0 || p->cheb_k > 64) return fail(ctx, LNE_EINVAL, "cheb_k outside 0..64");
    if (!std::isfinite(p->theta) || p->theta < 0.0 || !std::isfinite(p->mu))
        return fail(ctx, LNE_EINVAL, "theta must be finite and >= 0, mu finite");
    if (p->precision < LNE_F64 || p->precision > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "precision must be LNE_F64, LNE_F32 or LNE_BF16");
    (void)n_arcs;
    return LNE_OK;
}

static void host_plan(const lne_params *p, int64_t n, int64_t n_arcs, SamplePlan &pl) {
    std::memset(&pl, 0, sizeof(pl));
    const int64_t m = n_arcs / 2;
    pl.seed = p->seed;
    pl.T = p->T;
    pl.wt = nullptr;
    pl.cw = nullptr;
    pl.guide = nullptr;
    pl.ea = nullptr;
    if (m > 0) {
        pl.base = p->M / (uint64_t)m;
        const uint64_t rem = p->M % (uint64_t)m;
        pl.frac_thr = (uint64_t)(((unsigned __int128)rem << 32) / (uint64_t)m);
        pl.S = (int64_t)pl.base + (rem > 0 ? 1 : 0);
    }
    double total = 0.0;
    for (int t = 0; t < p->T; ++t) total += p->s[t];
    double cum = 0.0;
    for (int t = 0; t < p->T; ++t) {
        cum += p->s[t];
        uint64_t th = (uint64_t)std::floor(cum / total * 4294967296.0);
        if (th > 4294967296ull) th = 4294967296ull;
        pl.theta[t] = th;
    }
    pl.theta[p->T - 1] = 4294967296ull;
    for (int t = p->T; t < 16; ++t) pl.theta[t] = 4294967296ull;
    if (std::isinf(p->C) && p->C > 0) {
        pl.no_ds = 1;
        pl.C = 0.0;
    } else {
        pl.no_ds = 0;
        pl.C = p->C > 0.0 ? p->C : std::log((double)n);
    }
    // one thread per chunk of J slots of one edge, about 2^20 threads overall
    const int64_t slots = m * (pl.S > 0 ? pl.S : 1);
    int64_t J = (slots + (1 << 20) - 1) >> 20;
    if (J < 1) J = 1;
    if (J > pl.S) J = pl.S > 0 ? pl.S : 1;
    pl.J = J;
    pl.chunks = pl.S > 0 ? (pl.S + J - 1) / J : 1;
    int cb = 1;
    while (((int64_t)1 << cb) < n) ++cb;
    pl.colbits = cb;
}

lne_status make_plan(lne_ctx *ctx, const lne_params *p, int64_t n, int64_t n_arcs,
                     SamplePlan &pl) {
    (void)ctx;
    host_plan(p, n, n_arcs, pl);
    return LNE_OK;
}

// Modified Bessel function of the first kind, integer order, by its power
// series sum_j (x/2)^(2j+n) / (j! (j+n)!).
double bessel_i(int n, double x) {
    double term = 1.0;
    for (int i = 1; i <= n; ++i) term *= (x / 2.0) / i;
    double sum = term;
    for (int j = 1; j < 500; ++j) {
        term *= (x / 2.0) * (x / 2.0) / ((double)j * (double)(j + n));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// ------------------------------------------------------------------- stages
// Pair-buffer budget in bytes: LNE_HBM_BUDGET_GB if set, else 70% of HBM.
static double pair_budget(lne_ctx *ctx) {
    const char *env = getenv("LNE_HBM_BUDGET_GB");
    if (env && *env) return atof(env) * 1e9;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess || tot == 0) return 64e9;
    (void)ctx;
    return 0.7 * (double)tot;
}

// Device bytes one row range needs while it is aggregated: two (key, weight)
// ping-pong pairs and, at worst, a count CSR entry per pair entry.
static double range_bytes(uint64_t entries) { return 36.0 * (double)entries; }

struct Sampler {
    SamplePlan pl;
    Buf eu, ev, wc, wo, ea, cw, guide;
    int64_t m = 0, nw = 0;
    uint64_t attempted = 0, accepted = 0;
};

// Edge list of the sampler and, on a weighted graph, its weight tables: the
// prefix sums of the arc weights and each edge's weight.
static lne_status sampler_edges(lne_ctx *ctx, const Graph *g, Sampler &S) {
    LNE_TRY(build_edges(ctx, g, S.eu, S.ev, S.m, g->weight ? &S.ea : nullptr));
    if (!g->weight) return LNE_OK;
    uint64_t vol = 0;
    LNE_TRY(weight_info(ctx, g, S.cw, &vol));
    LNE_TRY(weight_guide(ctx, g, S.cw.as<uint64_t>(), S.guide));
    S.pl.wt = g->weight;
    S.pl.cw = S.cw.as<uint64_t>();
    S.pl.ea = S.ea.as<uint32_t>();
    S.pl.guide = S.guide.as<uint32_t>();
    return LNE_OK;
}

static lne_status count_range(lne_ctx *ctx, const Graph *g, Sampler &S, int64_t lo,
                              int64_t hi, uint64_t *entries, bool stats) {
    Buf scal(ctx);
    LNE_TRY(alloc(ctx, scal, 24));
    LNE_HIP(ctx, hipMemsetAsync(scal.p, 0, 24, ctx->stream));
    LNE_TRY(launch_sample_count(ctx, g, S.pl, S.eu.as<int32_t>(), S.ev.as<int32_t>(), S.m, lo, hi,
                                S.wc.as<uint32_t>(), S.nw,
                                stats ? scal.as<unsigned long long>() : nullptr));
    LNE_TRY(scan_u32(ctx, S.wc.as<uint32_t>(), S.wo.as<uint64_t>(), S.nw));
    uint64_t host[4] = {0, 0, 0, 0};
    LNE_HIP(ctx, hipMemcpyAsync(&host[0], S.wo.as<uint64_t>() + S.nw, 8, hipMemcpyDeviceToHost,
                                ctx->stream));
    if (stats)
        LNE_HIP(ctx, hipMemcpyAsync(&host[1], scal.p, 24, hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *entries = host[0];
    if (stats) {
        S.attempted = host[1];
        S.accepted = host[3];
        const uint32_t max_w = (uint32_t)host[2];
        if (max_w == 0xFFFFFFFFu)
            return fail(ctx, LNE_EUNSUPPORTED, "a per-sample weight exceeds 2^32 - 1");
    }
    return LNE_OK;
}

// With a TruncLogFuse the aggregation writes Eq. (1)'s matrix directly.
struct TruncLogFuse {
    TLConst c;
    int32_t val_type;
    const uint32_t *deg = nullptr;   // vertex degrees (vertex_degrees)
    uint64_t kept = 0;               // nonzero entries over all blocks so far
};

// Aggregates the pair entries of rows [lo, hi) (already counted into S.wo)
// into a count CSR block with hi - lo rows (or, with tl, the truncated-log
// block with explicit zeros for dropped pairs).
static lne_status aggregate_range(lne_ctx *ctx, const Graph *g, Sampler &S, int64_t lo,
                                  int64_t hi, uint64_t entries, lne_csr *out,
                                  TruncLogFuse *tl = nullptr) {
    const int64_t P = (int64_t)entries;
    Buf k0(ctx), v0(ctx), k1(ctx), v1(ctx);
    LNE_TRY(alloc(ctx, k0, sizeof(uint64_t) * (size_t)(P > 0 ? P : 1)));
    LNE_TRY(alloc(ctx, v0, sizeof(uint32_t) * (size_t)(P > 0 ? P : 1)));
    if (P > 0)
        LNE_TRY(launch_sample_emit(ctx, g, S.pl, S.eu.as<int32_t>(), S.ev.as<int32_t>(), S.m, lo,
                                   hi, S.wo.as<uint64_t>(), k0.as<uint64_t>(), v0.as<uint32_t>()));
    int which = 0;
    bool tagged = false;
    if (P > 1) {
        int rowbits = 0;
        while (((int64_t)1 << rowbits) < hi - lo) ++rowbits;
        LNE_TRY(alloc(ctx, k1, sizeof(uint64_t) * (size_t)P));
        LNE_TRY(alloc(ctx, v1, sizeof(uint32_t) * (size_t)P));
        // with the fused truncated log, the keys come out tagged with their
        // column's degree (read while the pairs are in column order)
        const int bits = rowbits + S.pl.colbits + S.pl.cbits;
        tagged = tl && S.pl.cbits == 0 && radix_tag_shift(bits, S.pl.colbits) >= 0;
        LNE_TRY(radix_sort(ctx, k0.as<uint64_t>(), v0.as<uint32_t>(), k1.as<uint64_t>(),
                           v1.as<uint32_t>(), P, bits, &which, tagged ? tl->deg : nullptr,
                           S.pl.colbits));
        // the other ping-pong pair is free before the CSR is allocated
        if (which) { k0.release(); v0.release(); } else { k1.release(); v1.release(); }
    }
    const uint64_t *keys = which ? k1.as<uint64_t>() : k0.as<uint64_t>();
    const uint32_t *vals = which ? v1.as<uint32_t>() : v0.as<uint32_t>();
    if (tl) {
        uint64_t kept = 0;
        LNE_TRY(reduce_to_matrix(ctx, keys, vals, P, hi - lo, S.pl.colbits, g, tl->deg, lo,
                                 tl->c, tl->val_type, out, &kept, tagged));
        tl->kept += kept;
        return LNE_OK;
    }
    LNE_TRY(reduce_to_csr(ctx, keys, vals, P, hi - lo, S.pl.colbits + S.pl.cbits, out));
    out->n_cols = g->n << S.pl.cbits;
    return LNE_OK;
}

// The embedding's matrix in one pass from one entry per sample, (min, max) of
// its endpoints: the upper triangle is sorted and reduced (Eq. (1) fused, a
// diagonal sum doubled), its distinct pairs sorted again by column give the
// lower triangle, and the two are merged into the symmetric matrix -- the
// same entries as reducing both orientations of every sample, with half the
// items in the six-pass sort (S.pl.upper set, entries counted that way).
static lne_status aggregate_sym(lne_ctx *ctx, const Graph *g, Sampler &S, uint64_t entries,
                                lne_csr *out, TruncLogFuse *tl) {
    const int64_t P = (int64_t)entries;
    const int colbits = S.pl.colbits;
    Buf k0(ctx), v0(ctx), k1(ctx), v1(ctx);
    LNE_TRY(alloc(ctx, k0, sizeof(uint64_t) * (size_t)(P > 0 ? P : 1)));
    LNE_TRY(alloc(ctx, v0, sizeof(uint32_t) * (size_t)(P > 0 ? P : 1)));
    if (P > 0)
        LNE_TRY(launch_sample_emit(ctx, g, S.pl, S.eu.as<int32_t>(), S.ev.as<int32_t>(), S.m, 0,
                                   g->n, S.wo.as<uint64_t>(), k0.as<uint64_t>(),
                                   v0.as<uint32_t>()));
    int which = 0;
    const bool tagged = P > 1;   // the sort writes the column degree tags
    if (P > 1) {
        LNE_TRY(alloc(ctx, k1, sizeof(uint64_t) * (size_t)P));
        LNE_TRY(alloc(ctx, v1, sizeof(uint32_t) * (size_t)P));
        LNE_TRY(radix_sort(ctx, k0.as<uint64_t>(), v0.as<uint32_t>(), k1.as<uint64_t>(),
                           v1.as<uint32_t>(), P, 2 * colbits, &which, tl->deg, colbits));
        if (which) { k0.release(); v0.release(); } else { k1.release(); v1.release(); }
    }
    const uint64_t *keys = which ? k1.as<uint64_t>() : k0.as<uint64_t>();
    const uint32_t *vals = which ? v1.as<uint32_t>() : v0.as<uint32_t>();
    lne_csr U;
    std::memset(&U, 0, sizeof(U));
    SymOut sym(ctx);
    uint64_t kept_u = 0;
    lne_status s = reduce_to_matrix(ctx, keys, vals, P, g->n, colbits, g, tl->deg, 0, tl->c,
                                    LNE_F32, &U, &kept_u, tagged, &sym);
    k0.release(); v0.release(); k1.release(); v1.release();
    if (s != LNE_OK) {
        lne_csr_free(ctx, &U);
        return s;
    }
    uint64_t kept = 0;
    s = sym_assemble(ctx, &U, sym, colbits, kept_u, out, &kept);
    if (s != LNE_OK) {
        lne_csr_free(ctx, &U);
        return s;
    }
    tl->kept += kept;
    return LNE_OK;
}

// Runs the sparsifier and hands each row block of the count matrix, in row
// order, to `sink(block, row_lo)`, which takes ownership of the block.  One
// block covers all rows unless the pair buffers would exceed the budget; then
// the rows are split into ranges of about equal arc count (and halved again
// while a range is still too large), each range walking every sample again
// and keeping the entries whose row falls inside it.
template <class Sink>
static lne_status sparsify_impl(lne_ctx *ctx, const Graph *g, const lne_params *p,
                                lne_stats *st, Sink &&sink, bool channels = false,
                                TruncLogFuse *tl = nullptr) {
    Sampler S;
    LNE_TRY(make_plan(ctx, p, g->n, g->n_arcs, S.pl));
    // one pass shared by trials with different s: the length r is kept in
    // the key (column b << 4 | r - 1)
    if (channels) S.pl.cbits = 4;
    if (channels && g->weight)
        return fail(ctx, LNE_EUNSUPPORTED, "batched trials take unweighted graphs");
    // the embedding's FP32 matrix from the upper triangle (aggregate_sym) when
    // the sort can carry the column degree tags
    const bool sym = tl && !channels && tl->val_type == LNE_F32 &&
                     radix_tag_shift(2 * S.pl.colbits, S.pl.colbits) >= 0;
    S.pl.upper = sym ? 1 : 0;
    S.m = g->n_arcs / 2;
    uint64_t total = 0;
    if (S.m > 0 && S.pl.S > 0) {
        LNE_TRY(sampler_edges(ctx, g, S));
        S.nw = sample_threads(S.pl, S.m) / 64;
        LNE_TRY(alloc(ctx, S.wc, sizeof(uint32_t) * (size_t)S.nw));
        LNE_TRY(alloc(ctx, S.wo, sizeof(uint64_t) * (size_t)(S.nw + 1)));
        LNE_TRY(count_range(ctx, g, S, 0, g->n, &total, true));
    }
    if (st) {
        st->attempted = S.attempted;
        st->accepted = S.accepted;
        st->nnz_counts = 0;
        st->entries = total;
    }
    const double budget = pair_budget(ctx);
    // the upper-triangle pass needs about as much memory as the two-orientation
    // one for half the entries
    if (sym && total > 0 && range_bytes(2 * total) <= budget) {
        lne_csr blk;
        std::memset(&blk, 0, sizeof(blk));
        LNE_TRY(aggregate_sym(ctx, g, S, total, &blk, tl));
        if (st) st->nnz_counts = (uint64_t)blk.nnz;
        return sink(blk, (int64_t)0);
    }
    if (sym && total > 0) {
        // too large for one pass: count both orientations for the row ranges
        S.pl.upper = 0;
        LNE_TRY(count_range(ctx, g, S, 0, g->n, &total, false));
        if (st) st->entries = total;
    }
    if (total == 0 || range_bytes(total) <= budget) {
        lne_csr blk;
        std::memset(&blk, 0, sizeof(blk));
        if (total == 0 && tl) {
            uint64_t kept = 0;
            LNE_TRY(reduce_to_matrix(ctx, nullptr, nullptr, 0, g->n, S.pl.colbits, g, tl->deg, 0,
                                     tl->c, tl->val_type, &blk, &kept));
        } else if (total == 0) {
            LNE_TRY(reduce_to_csr(ctx, nullptr, nullptr, 0, g->n, S.pl.colbits + S.pl.cbits, &blk));
            blk.n_cols = g->n << S.pl.cbits;
        } else {
            LNE_TRY(aggregate_range(ctx, g, S, 0, g->n, total, &blk, tl));
        }
        if (st) st->nnz_counts = (uint64_t)blk.nnz;
        return sink(blk, (int64_t)0);
    }
    // equal-arc row ranges from the graph offsets
    const int64_t K = (int64_t)std::ceil(range_bytes(total) / budget * 1.25);
    std::vector<int64_t> rp(g->n + 1);
    LNE_HIP(ctx, hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int64_t) * (size_t)(g->n + 1),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<std::pair<int64_t, int64_t>> todo;
    int64_t lo = 0;
    for (int64_t k = 1; k <= K; ++k) {
        const int64_t target = g->n_arcs * k / K;
        int64_t hi = (int64_t)(std::lower_bound(rp.begin(), rp.end(), target) - rp.begin());
        if (k == K) hi = g->n;
        hi = std::max(hi, lo + 1);
        hi = std::min(hi, g->n);
        if (hi > lo) todo.push_back({lo, hi});
        lo = hi;
        if (lo >= g->n) break;
    }
    if (lo < g->n) todo.push_back({lo, g->n});
    std::reverse(todo.begin(), todo.end());   // used as a stack, lowest rows on top
    while (!todo.empty()) {
        const auto rg = todo.back();
        todo.pop_back();
        uint64_t entries = 0;
        LNE_TRY(count_range(ctx, g, S, rg.first, rg.second, &entries, false));
        if (range_bytes(entries) > budget && rg.second - rg.first > 1) {
            const int64_t mid = rg.first + (rg.second - rg.first) / 2;
            todo.push_back({mid, rg.second});
            todo.push_back({rg.first, mid});
            continue;
        }
        lne_csr blk;
        std::memset(&blk, 0, sizeof(blk));
        LNE_TRY(aggregate_range(ctx, g, S, rg.first, rg.second, entries, &blk, tl));
        if (st) st->nnz_counts += (uint64_t)blk.nnz;
        LNE_TRY(sink(blk, rg.first));
    }
    return LNE_OK;
}

struct Flags {
    Buf b;
    int32_t *status() const { return b.as<int32_t>(); }
    int32_t *shifted() const { return b.as<int32_t>() + 1; }
    int32_t *run3() const { return b.as<int32_t>() + 2; }
};

static lne_status make_flags(lne_ctx *ctx, Flags &f) {
    f.b.ctx = ctx;
    LNE_TRY(alloc(ctx, f.b, 16));
    LNE_HIP(ctx, hipMemsetAsync(f.b.p, 0, 16, ctx->stream));
    return LNE_OK;
}

static lne_status read_flags(lne_ctx *ctx, const Flags &f, lne_stats *st) {
    int32_t h[4] = {0, 0, 0, 0};
    LNE_HIP(ctx, hipMemcpyAsync(h, f.b.p, 16, hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (st) st->shifted += (uint32_t)h[1];
    if (h[0]) return fail(ctx, LNE_ENUMERIC, "Cholesky breakdown even after a shift");
    return LNE_OK;
}

// CholeskyQR2 in place; a shifted first pass triggers a third pass (flag on
// the device, so no host round trip).
static lne_status orth_impl(lne_ctx *ctx, void *Y, int64_t n, int32_t k, int64_t ld,
                            int32_t dtype, const Flags &f) {
    Buf G(ctx), W(ctx);
    LNE_TRY(alloc(ctx, G, sizeof(double) * (size_t)k * k));
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)k * k));
    for (int pass = 0; pass < 3; ++pass) {
        const int32_t *skip = pass == 2 ? f.run3() : nullptr;
        int32_t *next = pass == 0 ? f.run3() : nullptr;
        LNE_TRY(gram(ctx, Y, dtype, n, k, ld, G.as<double>(), skip));
        LNE_TRY(chol_inv(ctx, G.as<double>(), k, W.as<double>(), f.status(), f.shifted(), n,
                         skip, next));
        LNE_TRY(project(ctx, Y, dtype, ld, n, k, W.as<double>(), k, Y, dtype, ld, skip));
    }
    return LNE_OK;
}

// C = Y^T Y, eigenpairs sorted descending into V (k x k), lam (k).
static lne_status eig_of_gram(lne_ctx *ctx, const void *Y, int32_t dtype, int64_t n,
                              int32_t k, int64_t ld, Buf &V, Buf &lam) {
    Buf G(ctx);
    LNE_TRY(alloc(ctx, G, sizeof(double) * (size_t)k * k));
    LNE_TRY(alloc(ctx, V, sizeof(double) * (size_t)k * k));
    LNE_TRY(alloc(ctx, lam, sizeof(double) * (size_t)k));
    LNE_TRY(gram(ctx, Y, dtype, n, k, ld, G.as<double>(), nullptr));
    return sym_eig(ctx, G.as<double>(), k, V.as<double>(), lam.as<double>());
}

// Row stride of the dense n x k blocks: whole 128-byte cache lines, so a
// gathered row touches ceil(k e / 128) lines wherever it starts (a stride of
// k rounded to 8 elements lets rows straddle one more line).
static int64_t line_ld(int64_t k, size_t es) {
    const int64_t q = (int64_t)(128 / es);
    return (k + q - 1) / q * q;
}

// ---- sparsifier in host memory ---------------------------------------------
// For graphs whose sparsifier exceeds HBM (LNE_FLAG_HOST_SPARSIFIER): the row
// blocks of M live in pinned host memory in chunks of at most
// host_chunk_nnz() entries (a longer row makes a chunk of its own), and every
// product with M streams them: a copy stream stages chunk b + 1 while chunk b
// is multiplied, two staging buffers ordered by events.
// Entries per chunk: LNE_HOST_CHUNK_NNZ if set, else 2^28 (2 GB of column and
// FP32 value, two staging copies of which sit in HBM).
static int64_t host_chunk_nnz() {
    const char *env = getenv("LNE_HOST_CHUNK_NNZ");
    if (env && *env) {
        const long long v = atoll(env);
        if (v >= 1) return (int64_t)v;
    }
    return (int64_t)1 << 28;
}

struct HostChunk {
    int64_t row_lo = 0, n_rows = 0, nnz = 0;
    int64_t *rp = nullptr;   // pinned, n_rows + 1 entries from 0
    int32_t *col = nullptr;  // pinned
    void *val = nullptr;     // pinned
};

struct HostMatrix {
    std::vector<HostChunk> chunks;
    int64_t n = 0, rows = 0, max_rows = 0, max_nnz = 0;
    int32_t val_type = LNE_F32;
    HostMatrix() = default;
    HostMatrix(const HostMatrix &) = delete;
    HostMatrix &operator=(const HostMatrix &) = delete;
    ~HostMatrix() {
        for (auto &c : chunks) {
            if (c.rp) (void)hipHostFree(c.rp);
            if (c.col) (void)hipHostFree(c.col);
            if (c.val) (void)hipHostFree(c.val);
        }
    }
};

// Moves a device row block (rows [H.rows, H.rows + blk.n_rows)) to pinned host
// chunks and frees it.  Synchronises the stream.
static lne_status block_to_host(lne_ctx *ctx, lne_csr &blk, HostMatrix &H) {
    const size_t es = dtype_size(blk.val_type);
    H.val_type = blk.val_type;
    H.n = blk.n_cols;
    const int64_t chunk = host_chunk_nnz();
    std::vector<int64_t> rp((size_t)blk.n_rows + 1);
    LNE_HIP(ctx, hipMemcpyAsync(rp.data(), blk.row_ptr, sizeof(int64_t) * rp.size(),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t r0 = 0, r1; r0 < blk.n_rows; r0 = r1) {
        r1 = r0 + 1;
        while (r1 < blk.n_rows && rp[r1 + 1] - rp[r0] <= chunk) ++r1;
        HostChunk c;
        c.row_lo = H.rows + r0;
        c.n_rows = r1 - r0;
        c.nnz = rp[r1] - rp[r0];
        if (hipHostMalloc((void **)&c.rp, sizeof(int64_t) * (size_t)(c.n_rows + 1)) != hipSuccess ||
            hipHostMalloc((void **)&c.col, sizeof(int32_t) * (size_t)(c.nnz ? c.nnz : 1)) !=
                hipSuccess ||
            hipHostMalloc(&c.val, es * (size_t)(c.nnz ? c.nnz : 1)) != hipSuccess) {
            H.chunks.push_back(c);
            return fail(ctx, LNE_ENOMEM, "host sparsifier: pinned allocation failed");
        }
        for (int64_t r = 0; r <= c.n_rows; ++r) c.rp[r] = rp[r0 + r] - rp[r0];
        if (c.nnz) {
            LNE_HIP(ctx, hipMemcpyAsync(c.col, blk.col + rp[r0], sizeof(int32_t) * c.nnz,
                                        hipMemcpyDeviceToHost, ctx->stream));
            LNE_HIP(ctx, hipMemcpyAsync(c.val, (const char *)blk.val + es * rp[r0], es * c.nnz,
                                        hipMemcpyDeviceToHost, ctx->stream));
        }
        H.max_rows = std::max(H.max_rows, c.n_rows);
        H.max_nnz = std::max(H.max_nnz, c.nnz);
        H.chunks.push_back(c);
    }
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    H.rows += blk.n_rows;
    lne_csr_free(ctx, &blk);
    return LNE_OK;
}

// The sparsifier of a product: a device CSR, or host chunks.
struct MatOp {
    const lne_csr *M = nullptr;
    const HostMatrix *H = nullptr;
    int64_t n = 0;
};

// Runs fn(view, row_lo) on every chunk of H staged in device memory, the copy
// of the next chunk overlapping the work on the current one.
template <class F>
static lne_status stream_chunks(lne_ctx *ctx, const HostMatrix &H, F &&fn) {
    const size_t es = dtype_size(H.val_type);
    Buf rp[2] = {Buf(ctx), Buf(ctx)}, cc[2] = {Buf(ctx), Buf(ctx)}, vv[2] = {Buf(ctx), Buf(ctx)};
    for (int i = 0; i < 2; ++i) {
        LNE_TRY(alloc(ctx, rp[i], sizeof(int64_t) * (size_t)(H.max_rows + 1)));
        LNE_TRY(alloc(ctx, cc[i], sizeof(int32_t) * (size_t)(H.max_nnz ? H.max_nnz : 1)));
        LNE_TRY(alloc(ctx, vv[i], es * (size_t)(H.max_nnz ? H.max_nnz : 1)));
    }
    hipStream_t cs = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr}, ready = nullptr;
    lne_status st = LNE_OK;
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && st == LNE_OK)
            st = fail(ctx, LNE_EHIP, "host sparsifier: %s: %s", what, hipGetErrorString(e));
        return e == hipSuccess;
    };
    if (hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream"))
        for (int i = 0; i < 2; ++i)
            if (!hip_ok(hipEventCreateWithFlags(&copied[i], hipEventDisableTiming), "event") ||
                !hip_ok(hipEventCreateWithFlags(&used[i], hipEventDisableTiming), "event"))
                break;
    // a caller's stream-ordered allocator may hand out staging memory that
    // work already queued on the context stream still reads: the copy stream
    // starts behind that work
    if (st == LNE_OK && hip_ok(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "event") &&
        hip_ok(hipEventRecord(ready, ctx->stream), "record"))
        hip_ok(hipStreamWaitEvent(cs, ready, 0), "wait");
    for (size_t b = 0; st == LNE_OK && b < H.chunks.size(); ++b) {
        const HostChunk &c = H.chunks[b];
        const int sl = (int)(b & 1);
        if (b >= 2 && !hip_ok(hipStreamWaitEvent(cs, used[sl], 0), "wait")) break;
        if (!hip_ok(hipMemcpyAsync(rp[sl].p, c.rp, sizeof(int64_t) * (size_t)(c.n_rows + 1),
                                   hipMemcpyHostToDevice, cs), "copy"))
            break;
        if (c.nnz && (!hip_ok(hipMemcpyAsync(cc[sl].p, c.col, sizeof(int32_t) * (size_t)c.nnz,
                                             hipMemcpyHostToDevice, cs), "copy") ||
                      !hip_ok(hipMemcpyAsync(vv[sl].p, c.val, es * (size_t)c.nnz,
                                             hipMemcpyHostToDevice, cs), "copy")))
            break;
        if (!hip_ok(hipEventRecord(copied[sl], cs), "record") ||
            !hip_ok(hipStreamWaitEvent(ctx->stream, copied[sl], 0), "wait"))
            break;
        lne_csr view;
        std::memset(&view, 0, sizeof(view));
        view.n_rows = c.n_rows;
        view.n_cols = H.n;
        view.nnz = c.nnz;
        view.row_ptr = rp[sl].as<int64_t>();
        view.col = cc[sl].as<int32_t>();
        view.val = vv[sl].p;
        view.val_type = H.val_type;
        if (c.n_rows > 0) st = fn(view, c.row_lo);
        if (st == LNE_OK) hip_ok(hipEventRecord(used[sl], ctx->stream), "record");
    }
    // the staging buffers are released when this returns: drain both streams
    if (cs) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(cs);
    }
    for (int i = 0; i < 2; ++i) {
        if (copied[i]) (void)hipEventDestroy(copied[i]);
        if (used[i]) (void)hipEventDestroy(used[i]);
    }
    if (ready) (void)hipEventDestroy(ready);
    return st;
}

// Y = M X for a device or host sparsifier.
static lne_status apply_M(lne_ctx *ctx, const MatOp &op, const void *X, int64_t ldx, void *Y,
                          int64_t ldy, int32_t k, int32_t dt) {
    if (!op.H) return spmm(ctx, op.M, X, ldx, Y, ldy, k, dt);
    const size_t es = dtype_size(dt);
    return stream_chunks(ctx, *op.H, [&](const lne_csr &v, int64_t lo) {
        return spmm(ctx, &v, X, ldx, (char *)Y + es * (size_t)(lo * ldy), ldy, k, dt);
    });
}

static lne_status apply_M_sparse_omega(lne_ctx *ctx, const MatOp &op, const int16_t *om, void *Y,
                                       int64_t ldy, int32_t k, int32_t dt) {
    if (!op.H) return spmm_sparse_omega(ctx, op.M, om, Y, ldy, k, dt);
    const size_t es = dtype_size(dt);
    return stream_chunks(ctx, *op.H, [&](const lne_csr &v, int64_t lo) {
        return spmm_sparse_omega(ctx, &v, om, (char *)Y + es * (size_t)(lo * ldy), ldy, k, dt);
    });
}

static lne_status rsvd_impl(lne_ctx *ctx, const MatOp &op, const lne_params *p, void *U,
                            double *sigma, void *V, void *X0, lne_stats *st) {
    const int64_t n = op.n;
    const int32_t kp = p->d + p->oversample, d = p->d;
    const int32_t dt = p->precision;
    const int32_t out_t = dt == LNE_F64 ? LNE_F64 : LNE_F32;
    const size_t es = dtype_size(dt);
    const int64_t ld = line_ld(kp, es);
    Buf A(ctx), B(ctx);
    LNE_TRY(alloc(ctx, A, es * (size_t)n * ld));
    LNE_TRY(alloc(ctx, B, es * (size_t)n * ld));
    Flags f;
    LNE_TRY(make_flags(ctx, f));
    void *Q = A.p, *Y = B.p;
    if (p->flags & LNE_FLAG_SPARSE_OMEGA) {
        Buf om(ctx);
        LNE_TRY(alloc(ctx, om, sizeof(int16_t) * kSparseOmega * (size_t)n));
        LNE_TRY(launch_sparse_omega(ctx, n, kp, p->seed, om.as<int16_t>()));
        LNE_TRY(apply_M_sparse_omega(ctx, op, om.as<int16_t>(), Y, ld, kp, dt));
    } else {
        LNE_TRY(launch_gaussian(ctx, n, kp, ld, p->seed, dt, Q));
        LNE_TRY(apply_M(ctx, op, Q, ld, Y, ld, kp, dt));
    }
    LNE_TRY(orth_impl(ctx, Y, n, kp, ld, dt, f));
    std::swap(Q, Y);
    Buf Vk(ctx), lam(ctx);
    for (int it = 1; it <= p->q; ++it) {
        LNE_TRY(apply_M(ctx, op, Q, ld, Y, ld, kp, dt));
        if (it < p->q) {
            LNE_TRY(orth_impl(ctx, Y, n, kp, ld, dt, f));
            std::swap(Q, Y);
        } else {
            LNE_TRY(eig_of_gram(ctx, Y, dt, n, kp, ld, Vk, lam));
        }
    }
    // Q holds T (the basis of the last power step), Y holds M T.
    Buf W(ctx), S(ctx);
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)kp * d));
    LNE_TRY(alloc(ctx, S, sizeof(double) * (size_t)d));
    // With Z = M T = Uz S Vz^T (eigenpairs of Z^T Z = Vz S^2 Vz^T): the fast
    // randomized SVD keeps U = Z Vz S^-1, V = T Vz; the vanilla one (the
    // randomized SVD the paper improves on: B = T^T M = Z^T, SVD of B) keeps
    // U = T Vz, V = Z Vz S^-1.  X0 = U S^(1/2) either way.
    const bool vanilla = (p->flags & LNE_FLAG_VANILLA_RSVD) != 0;
    void *Ubase = vanilla ? Q : Y, *Vbase = vanilla ? Y : Q;
    const double pu = vanilla ? 0.0 : -0.5, pv = vanilla ? -0.5 : 0.0;
    if (U) {
        LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), kp, d, pu, W.as<double>(),
                            nullptr));
        LNE_TRY(project(ctx, Ubase, dt, ld, n, kp, W.as<double>(), d, U, out_t, d, nullptr));
    }
    if (V) {
        LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), kp, d, pv, W.as<double>(),
                            nullptr));
        LNE_TRY(project(ctx, Vbase, dt, ld, n, kp, W.as<double>(), d, V, out_t, d, nullptr));
    }
    if (X0) {
        LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), kp, d, pu + 0.25,
                            W.as<double>(), nullptr));
        LNE_TRY(project(ctx, Ubase, dt, ld, n, kp, W.as<double>(), d, X0, out_t, d, nullptr));
    }
    LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), kp, d, 0.0, nullptr,
                        S.as<double>()));
    if (sigma)
        LNE_HIP(ctx, hipMemcpyAsync(sigma, S.p, sizeof(double) * d, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    return read_flags(ctx, f, st);
}

static lne_status propagate_impl(lne_ctx *ctx, const Graph *g, const lne_params *p,
                                 const void *X0, void *X) {
    const int64_t n = g->n;
    const int32_t d = p->d;
    const int32_t dt = p->precision == LNE_F64 ? LNE_F64 : LNE_F32;
    const size_t es = dtype_size(dt);
    if (p->cheb_k == 0 || p->theta < 1e-12) {
        LNE_HIP(ctx, hipMemcpyAsync(X, X0, es * (size_t)n * d, hipMemcpyDeviceToDevice,
                                    ctx->stream));
        return LNE_OK;
    }
    const int64_t ld = line_ld(d, es);
    const int K = p->cheb_k;
    const double th = p->theta, mu = p->mu;
    std::vector<double> c(K + 1);
    for (int i = 0; i <= K; ++i)
        c[i] = (i == 0 ? 1.0 : 2.0 * ((i & 1) ? -1.0 : 1.0)) * std::exp(-th / 2.0) * bessel_i(i, th);
    Buf b0(ctx), b1(ctx), b2(ctx), bz(ctx), bc(ctx);
    for (Buf *b : {&b0, &b1, &b2, &bz, &bc}) LNE_TRY(alloc(ctx, *b, es * (size_t)n * ld));
    // X0 already in the padded layout (ld == d, 16-byte aligned) serves as T0
    // itself (read only; the first rotation hands its slot to b0) instead of
    // being copied
    const bool direct = ld == d && (uintptr_t)X0 % 16 == 0;
    void *x0 = const_cast<void *>(X0);
    void *T0 = direct ? x0 : b0.p, *T1 = b1.p, *T2 = b2.p, *Z = bz.p, *conv = bc.p;
    if (!direct) LNE_TRY(dense_scale(ctx, X0, dt, d, T0, dt, ld, n, d, 1.0));
    // conv holds X0 - sum_i c_i T_i, the operand of the final product: it
    // starts as (1 - c_0) T0 (T0 = X0) in the pass that makes T1, and every
    // term is subtracted in the pass that makes it
    // T1 = (B^2 / 2 - I) T0 with B = L - mu I = (1 - mu) I - D^-1 A
    LNE_TRY(graph_spmm(ctx, g, T0, Z, ld, d, dt, 1.0 - mu, -1.0, nullptr, 0, nullptr, 0,
                       nullptr, 0));
    LNE_TRY(graph_spmm(ctx, g, Z, T1, ld, d, dt, 0.5 * (1.0 - mu), -0.5, T0, -1.0, nullptr, 0,
                       conv, -c[1], true, 1.0 - c[0]));
    for (int i = 2; i <= K; ++i) {
        // T_i = B^2 T_{i-1} - 2 T_{i-1} - T_{i-2}
        LNE_TRY(graph_spmm(ctx, g, T1, Z, ld, d, dt, 1.0 - mu, -1.0, nullptr, 0, nullptr, 0,
                           nullptr, 0));
        LNE_TRY(graph_spmm(ctx, g, Z, T2, ld, d, dt, 1.0 - mu, -1.0, T1, -2.0, T0, -1.0, conv,
                           -c[i]));
        void *t = T0;
        T0 = T1;
        T1 = T2;
        T2 = t == x0 ? b0.p : t;   // X0 is never written
    }
    // X_sp = D^-1 A (X0 - sum_i c_i T_i)
    LNE_TRY(graph_spmm(ctx, g, conv, Z, ld, d, dt, 0.0, 1.0, nullptr, 0, nullptr, 0, nullptr, 0));
    if (p->flags & LNE_FLAG_NO_FINAL_EIGSVD)
        return dense_scale(ctx, Z, dt, ld, X, dt, d, n, d, 1.0);
    // X = U_p S_p^(1/2) = X_sp V S^(-1/2)
    Buf V(ctx), lam(ctx), W(ctx);
    LNE_TRY(eig_of_gram(ctx, Z, dt, n, d, ld, V, lam));
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)d * d));
    LNE_TRY(eig_weights(ctx, V.as<double>(), lam.as<double>(), d, d, -0.25, W.as<double>(),
                        nullptr));
    return project(ctx, Z, dt, ld, n, d, W.as<double>(), d, X, dt, d, nullptr);
}

// The embedding's sparsifier: the aggregation writes Eq. (1)'s matrix
// directly (no count CSR); a row block keeps its dropped pairs as explicit
// zeros unless they are more than 1/32 of its entries, in which case it is
// compacted (the same decision with M in HBM or in host memory, so that both
// give the same products).  In HBM the blocks are concatenated into *M; with
// host they move to pinned host memory (H) as they are built.  *kept = the
// number of nonzero entries (st->nnz_log too).
static lne_status embed_matrix(lne_ctx *ctx, const Graph *g, const lne_params *p,
                               lne_stats *st, bool host, lne_csr *M, HostMatrix &H,
                               uint64_t *kept_out) {
    TruncLogFuse tl;
    uint64_t vol = (uint64_t)g->n_arcs;
    Buf cw(ctx);
    if (g->weight) LNE_TRY(weight_info(ctx, g, cw, &vol));
    tl.c = tl_const(vol, (uint64_t)g->n_arcs, p);
    tl.val_type = p->precision == LNE_F64 ? LNE_F64 : LNE_F32;
    Buf deg(ctx);
    LNE_TRY(alloc(ctx, deg, sizeof(uint32_t) * (size_t)(g->n > 0 ? g->n : 1)));
    LNE_TRY(vertex_degrees(ctx, g, deg.as<uint32_t>(), g->weight ? cw.as<uint64_t>() : nullptr));
    tl.deg = deg.as<uint32_t>();
    std::vector<lne_csr> mblocks;
    uint64_t kept_before = 0;
    auto sink = [&](lne_csr &blk, int64_t) -> lne_status {
        const uint64_t kept = tl.kept - kept_before;
        kept_before = tl.kept;
        lne_status r = LNE_OK;
        if ((uint64_t)blk.nnz - kept > (uint64_t)blk.nnz / 32) r = drop_zeros(ctx, &blk);
        if (r == LNE_OK && host) r = block_to_host(ctx, blk, H);
        if (r != LNE_OK) {
            lne_csr_free(ctx, &blk);
            return r;
        }
        if (!host) mblocks.push_back(blk);
        return LNE_OK;
    };
    LNE_TRY(validate_graph_device(ctx, g));
    lne_status s = sparsify_impl(ctx, g, p, st, sink, false, &tl);
    if (s == LNE_OK && !host) s = concat_rows(ctx, mblocks, g->n, M);
    if (s == LNE_OK && host && H.rows != g->n)
        s = fail(ctx, LNE_EINVAL, "host sparsifier: blocks cover %lld of %lld rows",
                 (long long)H.rows, (long long)g->n);
    for (auto &b : mblocks) lne_csr_free(ctx, &b);
    if (s != LNE_OK) {
        lne_csr_free(ctx, M);
        return s;
    }
    if (st) st->nnz_log = tl.kept;
    *kept_out = tl.kept;
    return LNE_OK;
}

// The channel sampling pass of the batched trials: the sparsifier with the
// walk length r kept in the key (column b << 4 | r - 1), as one CSR.
lne_status channels_pass(lne_ctx *ctx, const Graph *g, const lne_params *p, lne_csr *out,
                         lne_stats *st) {
    if (g->n > ((int64_t)1 << 30))
        return fail(ctx, LNE_EUNSUPPORTED, "channel sparsifier: n above 2^30");
    std::vector<lne_csr> blocks;
    auto sink = [&](lne_csr &blk, int64_t) -> lne_status {
        blocks.push_back(blk);
        return LNE_OK;
    };
    lne_status s = sparsify_impl(ctx, g, p, st, sink, true);
    if (s == LNE_OK) s = concat_rows(ctx, blocks, g->n, out);
    for (auto &b : blocks) lne_csr_free(ctx, &b);
    return s;
}

}  // namespace lne

using namespace lne;

// ===================================================================== ABI
extern "C" {

lne_status lne_ctx_create(lne_ctx **out, void *stream, lne_alloc_fn alloc_fn,
                          lne_free_fn free_fn, void *user) {
    if (!out) return LNE_EINVAL;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return LNE_EINVAL;
    lne_ctx *c = new (std::nothrow) lne_ctx();
    if (!c) return LNE_ENOMEM;
    c->stream = (hipStream_t)stream;
    c->alloc = alloc_fn;
    c->free_fn = free_fn;
    c->user = user;
    *out = c;
    return LNE_OK;
}

void lne_ctx_destroy(lne_ctx *ctx) {
    if (!ctx) return;
    for (auto &m : ctx->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    delete ctx;
}

const char *lne_last_error(const lne_ctx *ctx) { return ctx ? ctx->err : "NULL context"; }

const char *lne_version(void) { return "lne 0.1 (gfx950)"; }

lne_status lne_prof_enable(lne_ctx *ctx, int32_t on) {
    if (!ctx) return LNE_EINVAL;
    ctx->prof = on != 0;
    return LNE_OK;
}

static lne_status prof_collect(lne_ctx *ctx) {
    if (ctx->marks.empty()) return LNE_OK;
    LNE_HIP(ctx, hipEventSynchronize(ctx->marks.back().b));
    for (auto &m : ctx->marks) {
        float ms = 0.f;
        LNE_HIP(ctx, hipEventElapsedTime(&ms, m.a, m.b));
        auto &acc = ctx->prof_acc[m.name];
        acc.first += ms;
        acc.second += 1;
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    ctx->marks.clear();
    return LNE_OK;
}

lne_status lne_prof_get(lne_ctx *ctx, const char *name, double *total_ms, int64_t *launches) {
    if (!ctx || !name) return LNE_EINVAL;
    LNE_TRY(prof_collect(ctx));
    auto it = ctx->prof_acc.find(name);
    if (total_ms) *total_ms = it == ctx->prof_acc.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == ctx->prof_acc.end() ? 0 : it->second.second;
    return LNE_OK;
}

lne_status lne_prof_reset(lne_ctx *ctx) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(prof_collect(ctx));
    ctx->prof_acc.clear();
    return LNE_OK;
}

lne_status lne_philox(lne_ctx *ctx, uint64_t seed, const uint32_t *ctr, int64_t count,
                      uint32_t *out) {
    if (!ctx) return LNE_EINVAL;
    if (count < 0 || (count > 0 && (!ctr || !out)))
        return fail(ctx, LNE_EINVAL, "philox: bad arguments");
    return launch_philox(ctx, seed, ctr, count, out);
}

lne_status lne_sparse_omega(lne_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int16_t *out) {
    if (!ctx) return LNE_EINVAL;
    if (n < 0 || k < 1 || k > 1024 || (n > 0 && !out))
        return fail(ctx, LNE_EINVAL, "sparse_omega: bad arguments");
    if ((uintptr_t)out % 16) return fail(ctx, LNE_EINVAL, "sparse_omega: out must be 16-byte aligned");
    return launch_sparse_omega(ctx, n, k, seed, out);
}

lne_status lne_spmm_sparse_omega(lne_ctx *ctx, const lne_csr *A, const int16_t *om, void *Y,
                                 int64_t ldy, int32_t k, int32_t dtype) {
    if (!ctx) return LNE_EINVAL;
    if (!A || (uintptr_t)om % 16) return fail(ctx, LNE_EINVAL, "spmm_sparse_omega: bad arguments");
    return spmm_sparse_omega(ctx, A, om, Y, ldy, k, dtype);
}

lne_status lne_gaussian(lne_ctx *ctx, int64_t n, int32_t k, int64_t ld, uint64_t seed,
                        int32_t dtype, void *out) {
    if (!ctx) return LNE_EINVAL;
    if (n < 0 || k < 0 || ld < k || (n * k > 0 && !out) || dtype < LNE_F64 || dtype > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "gaussian: bad arguments");
    return launch_gaussian(ctx, n, k, ld, seed, dtype, out);
}

int64_t lne_slots_per_edge(const lne_params *p, int64_t n_arcs) {
    if (!p || n_arcs < 2) return 0;
    const uint64_t m = (uint64_t)(n_arcs / 2);
    return (int64_t)(p->M / m + (p->M % m ? 1 : 0));
}

lne_status lne_sampler_plan(const lne_params *p, int64_t n_arcs, uint64_t *base,
                            uint64_t *frac_thr, uint64_t *theta) {
    if (!p || p->T < 1 || p->T > 16 || n_arcs < 2 || !base || !frac_thr || !theta)
        return LNE_EINVAL;
    SamplePlan pl;
    {
        lne_ctx tmp;
        LNE_TRY(validate_params(&tmp, p, 1, n_arcs, false));
        make_plan(&tmp, p, 2, n_arcs, pl);
    }
    *base = pl.base;
    *frac_thr = pl.frac_thr;
    for (int t = 0; t < p->T; ++t) theta[t] = pl.theta[t];
    return LNE_OK;
}

lne_status lne_sample_slots(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                            int64_t e_begin, int64_t e_end, int32_t *a, int32_t *b, uint64_t *w,
                            uint8_t *r) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    const int64_t m = gin->n_arcs / 2;
    if (e_begin < 0 || e_end < e_begin || e_end > m)
        return fail(ctx, LNE_EINVAL, "sample_slots: edge range [%lld, %lld) outside [0, %lld)",
                    (long long)e_begin, (long long)e_end, (long long)m);
    if (e_end > e_begin && (!a || !b || !w || !r))
        return fail(ctx, LNE_EINVAL, "sample_slots: NULL output");
    if (e_end == e_begin) return LNE_OK;
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    Sampler S;
    LNE_TRY(make_plan(ctx, p, g->n, g->n_arcs, S.pl));
    S.m = m;
    LNE_TRY(sampler_edges(ctx, g, S));
    return launch_sample_slots(ctx, g, S.pl, S.eu.as<int32_t>(), S.ev.as<int32_t>(), e_begin,
                               e_end, a, b, w, r);
}

lne_status lne_sparsify(lne_ctx *ctx, const lne_graph *gin, const lne_params *p, lne_csr *out,
                        lne_stats *st) {
    if (!ctx) return LNE_EINVAL;
    if (!out) return fail(ctx, LNE_EINVAL, "sparsify: out is NULL");
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    std::memset(out, 0, sizeof(*out));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    std::vector<lne_csr> blocks;
    auto sink = [&](lne_csr &blk, int64_t) -> lne_status {
        blocks.push_back(blk);
        return LNE_OK;
    };
    lne_status s = sparsify_impl(ctx, g, p, st, sink);
    if (s == LNE_OK) s = concat_rows(ctx, blocks, g->n, out);
    for (auto &b : blocks) lne_csr_free(ctx, &b);
    return s;
}

lne_status lne_sparsify_rows(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                            int64_t row_lo, int64_t row_hi, lne_csr *out, lne_stats *st) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    if (!out) return fail(ctx, LNE_EINVAL, "sparsify_rows: out is NULL");
    if (row_lo < 0 || row_hi > gin->n || row_lo >= row_hi)
        return fail(ctx, LNE_EINVAL, "sparsify_rows: rows [%lld, %lld) outside [0, %lld)",
                    (long long)row_lo, (long long)row_hi, (long long)gin->n);
    std::memset(out, 0, sizeof(*out));
    if (st) std::memset(st, 0, sizeof(*st));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    Sampler S;
    LNE_TRY(make_plan(ctx, p, g->n, g->n_arcs, S.pl));
    S.m = g->n_arcs / 2;
    uint64_t total = 0, entries = 0;
    if (S.m > 0 && S.pl.S > 0) {
        LNE_TRY(sampler_edges(ctx, g, S));
        S.nw = sample_threads(S.pl, S.m) / 64;
        LNE_TRY(alloc(ctx, S.wc, sizeof(uint32_t) * (size_t)S.nw));
        LNE_TRY(alloc(ctx, S.wo, sizeof(uint64_t) * (size_t)(S.nw + 1)));
        LNE_TRY(count_range(ctx, g, S, 0, g->n, &total, true));
        LNE_TRY(count_range(ctx, g, S, row_lo, row_hi, &entries, false));
    }
    if (st) {
        st->attempted = S.attempted;
        st->accepted = S.accepted;
    }
    if (entries == 0) {
        LNE_TRY(reduce_to_csr(ctx, nullptr, nullptr, 0, row_hi - row_lo, S.pl.colbits, out));
        out->n_cols = g->n;
    } else {
        LNE_TRY(aggregate_range(ctx, g, S, row_lo, row_hi, entries, out));
    }
    if (st) st->nnz_counts = (uint64_t)out->nnz;
    return LNE_OK;
}

lne_status lne_trunc_log(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                         const lne_csr *counts, lne_csr *out) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    if (!counts || !out || counts->val_type != LNE_U64 || counts->n_rows != gin->n)
        return fail(ctx, LNE_EINVAL, "trunc_log: counts must be the U64 count matrix of g");
    if (p->precision < LNE_F64 || p->precision > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "trunc_log: bad precision");
    std::memset(out, 0, sizeof(*out));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    return trunc_log_csr(ctx, g, p, counts, 0, p->precision == LNE_F64 ? LNE_F64 : LNE_F32, out);
}

lne_status lne_csr_copy(lne_ctx *ctx, const lne_csr *m, int64_t *row_ptr, int32_t *col,
                        void *val) {
    if (!ctx) return LNE_EINVAL;
    if (!m || !row_ptr || (m->nnz > 0 && (!col || !val)))
        return fail(ctx, LNE_EINVAL, "csr_copy: NULL argument");
    LNE_HIP(ctx, hipMemcpyAsync(row_ptr, m->row_ptr, sizeof(int64_t) * (size_t)(m->n_rows + 1),
                                hipMemcpyDeviceToDevice, ctx->stream));
    if (m->nnz > 0) {
        LNE_HIP(ctx, hipMemcpyAsync(col, m->col, sizeof(int32_t) * (size_t)m->nnz,
                                    hipMemcpyDeviceToDevice, ctx->stream));
        LNE_HIP(ctx, hipMemcpyAsync(val, m->val, dtype_size(m->val_type) * (size_t)m->nnz,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    }
    return LNE_OK;
}

void lne_csr_free(lne_ctx *ctx, lne_csr *m) {
    if (!ctx || !m) return;
    dev_free(ctx, m->row_ptr);
    dev_free(ctx, m->col);
    dev_free(ctx, m->val);
    std::memset(m, 0, sizeof(*m));
}

lne_status lne_spmm(lne_ctx *ctx, const lne_csr *A, const void *X, int64_t ldx, void *Y,
                    int64_t ldy, int32_t k, int32_t dtype) {
    if (!ctx) return LNE_EINVAL;
    if (!A || k < 1 || ldx < k || ldy < k || !X || !Y)
        return fail(ctx, LNE_EINVAL, "spmm: bad arguments");
    return spmm(ctx, A, X, ldx, Y, ldy, k, dtype);
}

lne_status lne_eigsvd(lne_ctx *ctx, const void *Y, int64_t n, int32_t k, int64_t ld,
                      int32_t dtype, void *U, int64_t ldu, double *S, double *V) {
    if (!ctx) return LNE_EINVAL;
    if (!Y || n < 1 || k < 1 || ld < k || (U && ldu < k) || dtype < LNE_F64 || dtype > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "eigsvd: bad arguments");
    if (k > 288) return fail(ctx, LNE_EUNSUPPORTED, "eigsvd: k above 288");
    Buf Vk(ctx), lam(ctx), W(ctx);
    LNE_TRY(eig_of_gram(ctx, Y, dtype, n, k, ld, Vk, lam));
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)k * k));
    if (U) {
        LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), k, k, -0.5, W.as<double>(),
                            nullptr));
        const int32_t ut = dtype == LNE_BF16 ? LNE_F32 : dtype;
        LNE_TRY(project(ctx, Y, dtype, ld, n, k, W.as<double>(), k, U, ut, ldu, nullptr));
    }
    if (S) LNE_TRY(eig_weights(ctx, Vk.as<double>(), lam.as<double>(), k, k, 0.0, nullptr, S));
    if (V)
        LNE_HIP(ctx, hipMemcpyAsync(V, Vk.p, sizeof(double) * (size_t)k * k,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    return LNE_OK;
}

lne_status lne_graph_stats(lne_ctx *ctx, const lne_graph *gin, uint64_t seed, int32_t wedges,
                           int32_t iters, double *out) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    if (!out || wedges < 1 || iters < 1 || gin->n_arcs < 2)
        return fail(ctx, LNE_EINVAL, "graph_stats: needs out, wedges >= 1, iters >= 1, an edge");
    if (gin->weight) return fail(ctx, LNE_EUNSUPPORTED, "graph_stats: unweighted graphs only");
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    return graph_stats_impl(ctx, g, seed, wedges, iters, out);
}

lne_status lne_orthonormalize(lne_ctx *ctx, void *Y, int64_t n, int32_t k, int64_t ld,
                              int32_t dtype) {
    if (!ctx) return LNE_EINVAL;
    if (!Y || n < 1 || k < 1 || k > n || ld < k || dtype < LNE_F64 || dtype > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "orthonormalize: bad arguments");
    if (k > 288) return fail(ctx, LNE_EUNSUPPORTED, "orthonormalize: k above 288");
    Flags f;
    LNE_TRY(make_flags(ctx, f));
    LNE_TRY(orth_impl(ctx, Y, n, k, ld, dtype, f));
    return read_flags(ctx, f, nullptr);
}

lne_status lne_rsvd(lne_ctx *ctx, const lne_csr *M, const lne_params *p, void *U,
                    double *sigma, void *V, void *X0) {
    if (!ctx) return LNE_EINVAL;
    if (!M || M->n_rows != M->n_cols || M->n_rows < 1)
        return fail(ctx, LNE_EINVAL, "rsvd: M must be square");
    LNE_TRY(validate_params(ctx, p, M->n_rows, 0, true));
    const int32_t need = p->precision == LNE_F64 ? LNE_F64 : LNE_F32;
    if (M->val_type != need)
        return fail(ctx, LNE_EINVAL, "rsvd: values must be %s for this precision",
                    need == LNE_F64 ? "F64" : "F32");
    MatOp op;
    op.M = M;
    op.n = M->n_rows;
    return rsvd_impl(ctx, op, p, U, sigma, V, X0, nullptr);
}

lne_status lne_propagate(lne_ctx *ctx, const lne_graph *gin, const lne_params *p, const void *X0,
                         void *X) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, true));
    if (!X0 || !X) return fail(ctx, LNE_EINVAL, "propagate: NULL matrix");
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    return propagate_impl(ctx, g, p, X0, X);
}

lne_status lne_graph_spmm(lne_ctx *ctx, const lne_graph *gin, const void *Z, int64_t ld,
                          int32_t k, int32_t dtype, double a, double b, void *out) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    if (!Z || !out || k < 1 || ld < k || (dtype != LNE_F64 && dtype != LNE_F32))
        return fail(ctx, LNE_EINVAL, "graph_spmm: bad arguments");
    if (Z == out) return fail(ctx, LNE_EINVAL, "graph_spmm: out must not alias Z");
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    return graph_spmm(ctx, g, Z, out, ld, k, dtype, a, b, nullptr, 0.0, nullptr, 0.0, nullptr,
                      0.0);
}

lne_status lne_sparsify_log(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                            lne_csr *out, lne_stats *st) {
    if (!ctx) return LNE_EINVAL;
    if (!out) return fail(ctx, LNE_EINVAL, "sparsify_log: out is NULL");
    std::memset(out, 0, sizeof(*out));
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    if (p->precision < LNE_F64 || p->precision > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "precision must be LNE_F64, LNE_F32 or LNE_BF16");
    if (st) std::memset(st, 0, sizeof(*st));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    HostMatrix H;
    uint64_t kept = 0;
    return embed_matrix(ctx, g, p, st, false, out, H, &kept);
}

lne_status lne_embed(lne_ctx *ctx, const lne_graph *gin, const lne_params *p, void *X,
                     lne_stats *st) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, true));
    if (!X) return fail(ctx, LNE_EINVAL, "embed: X is NULL");
    if (st) std::memset(st, 0, sizeof(*st));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    lne_csr M;
    std::memset(&M, 0, sizeof(M));
    const bool host = (p->flags & LNE_FLAG_HOST_SPARSIFIER) != 0;
    HostMatrix H;
    uint64_t kept = 0;
    LNE_TRY(embed_matrix(ctx, g, p, st, host, &M, H, &kept));
    lne_status s = LNE_OK;
    const int32_t out_t = p->precision == LNE_F64 ? LNE_F64 : LNE_F32;
    Buf X0(ctx);
    s = alloc(ctx, X0, dtype_size(out_t) * (size_t)g->n * p->d);
    MatOp op;
    op.M = host ? nullptr : &M;
    op.H = host ? &H : nullptr;
    op.n = g->n;
    // a sparsifier with no entry left is the zero matrix: every singular
    // value is 0, so U S^1/2 = 0 whatever basis an SVD would return (the
    // orthonormalisation of its all-zero products has no basis to find)
    if (s == LNE_OK && kept == 0) {
        const hipError_t e = hipMemsetAsync(X0.p, 0, X0.bytes, ctx->stream);
        if (e != hipSuccess) s = fail(ctx, LNE_EHIP, "embed: memset: %s", hipGetErrorString(e));
    } else if (s == LNE_OK) {
        s = rsvd_impl(ctx, op, p, nullptr, nullptr, nullptr, X0.p, st);
    }
    lne_csr_free(ctx, &M);
    if (s != LNE_OK) return s;
    return propagate_impl(ctx, g, p, X0.p, X);
}

}  // extern "C"
